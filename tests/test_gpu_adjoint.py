"""GPU parity of the filter adjoint, the Hellmann-Feynman block gradient, the
spring chain rule and the eigenvalue count against the oracle."""
import numpy as np
import pytest

import paper_1902_07041_amd as P
from oracle import adjoint, count, filters as F
from synth import gaussian_block

from gpu_common import GlassCase, banner, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tiny():
    banner("glass N=125 (adjoint)")
    c = GlassCase(125, seed=3)
    c.h = c.handle()
    c.ub = float(c.lam[-1]) * 1.02
    P.pfe_set_bounds(c.h, 0.0, c.ub)
    yield c
    P.pfe_destroy(c.h)


@pytest.mark.parametrize("d,stride,q,resident",
                         [(12, 0, 3, False), (12, 5, 3, False), (1, 0, 2, False), (0, 0, 2, False),
                          (31, 4, 64, False), (7, 1, 70, False), (60, 10, 64, False),
                          (150, 0, 16, False), (200, 0, 8, False), (150, 0, 16, True),
                          (60, 0, 70, True), (60, 0, 96, True), (60, 0, 96, False)])
def test_adjoint_parity(tiny, d, stride, q, resident):
    """Segments of the checkpointed reverse sweep hold `stride` steps
    (ceil(sqrt d) by default): up to 5 here with the first five cases, 8, 10
    and 13 (d = 150, the benchmark's degree) and 15 (d = 200) with the later
    ones, so every register-resident segment kernel (8, 13 and 16 steps)
    and the q > 64 path are compared with the oracle.  The resident cases
    keep both trajectories and advance them side by side (they fit at this
    size): at q = 70 and 96 that fused step runs over 2 ld = 144 and 192
    columns, in two column passes, and the block gradient reads the adjoint
    vectors with a negative stride."""
    banner(f"adjoint d={d} stride={stride} q={q} resident={resident}")
    c, e = F.spectral_map(0.0, tiny.ub)
    xi, eta = (0.05 * tiny.lam[-1] - c) / e, (0.15 * tiny.lam[-1] - c) / e
    coef = F.filter_coefficients(xi, eta, 0.05, d, F.NONE)
    f = P.Filter(d, 0, c, e, xi, eta, 0.05, coef)
    X = gaussian_block(tiny.n, q, 21)
    W = gaussian_block(tiny.n, q, 22)
    dX, dB = P.pfe_apply_filter_adjoint(tiny.h, f, X, W, tiny.g.nnzb, stride, resident=resident)
    rX, rG = adjoint.filter_vjp_blocks(tiny.H, tiny.g.row_ptr, tiny.g.col_idx, c, e, coef, X, W)
    assert rel_err(dX, rX) < 1e-12
    if d >= 1:
        assert rel_err(dB, rG) < 1e-11
    else:
        assert np.all(dB == 0)


def test_adjoint_trajectory_equals_checkpoints(tiny):
    """The resident mode keeps both trajectories and advances them side by
    side when they fit (they do at this size), or the forward one alone when
    the rows are padded; the default (stride 0, ceil(sqrt d) = 13) and an
    explicit stride of 13 recompute each segment from checkpoints.  Same
    segments, same per-element arithmetic: identical bits in all four."""
    banner("adjoint, trajectory kept vs checkpoints, d=150")
    c, e = F.spectral_map(0.0, tiny.ub)
    xi, eta = (0.05 * tiny.lam[-1] - c) / e, (0.15 * tiny.lam[-1] - c) / e
    d = 150
    coef = F.filter_coefficients(xi, eta, 0.05, d, F.NONE)
    f = P.Filter(d, 0, c, e, xi, eta, 0.05, coef)
    X = gaussian_block(tiny.n, 16, 23)
    W = gaussian_block(tiny.n, 16, 24)
    dX0, dB0 = P.pfe_apply_filter_adjoint(tiny.h, f, X, W, tiny.g.nnzb, 0, resident=True)
    dX1, dB1 = P.pfe_apply_filter_adjoint(tiny.h, f, X, W, tiny.g.nnzb, 13)
    dX3, dB3 = P.pfe_apply_filter_adjoint(tiny.h, f, X, W, tiny.g.nnzb, 0)
    np.testing.assert_array_equal(dX0, dX1)
    np.testing.assert_array_equal(dB0, dB1)
    np.testing.assert_array_equal(dX3, dX1)
    np.testing.assert_array_equal(dB3, dB1)
    # rows padded to 24 columns: the recurrences cannot sit side by side in
    # one step of 2 ld columns, so only the forward trajectory is kept
    Xp = np.zeros((tiny.n, 24))
    Wp = np.zeros((tiny.n, 24))
    Xp[:, :16], Wp[:, :16] = X, W
    dX2, dB2 = P.pfe_apply_filter_adjoint(tiny.h, f, Xp, Wp, tiny.g.nnzb, 0, nvec=16,
                                          resident=True)
    np.testing.assert_array_equal(dX2[:, :16], dX0)
    np.testing.assert_array_equal(dB2, dB0)


def test_hellmann_feynman_and_chain_rule(tiny):
    banner("eigvec block gradient + spring chain rule")
    g = tiny.g
    idx = [10, 40, 41]
    V = np.ascontiguousarray(tiny.U[:, idx].T)
    w = np.array([1.0, 0.5, 2.0])
    dB = P.pfe_eigvec_block_gradient(tiny.h, V, g.nnzb, w)
    ref = sum(wi * adjoint.hellmann_feynman_blocks(V[s], g.row_ptr, g.col_idx) for s, wi in enumerate(w))
    assert rel_err(dB, ref) < 1e-13
    dk, dm = P.pfe_spring_gradient(tiny.h, g.pairs, g.unit, dB, g.n_atoms)
    rk, rm = adjoint.spring_chain_rule(ref, tiny.hb, g.row_ptr, g.col_idx, g.pairs, g.unit, g.masses)
    assert rel_err(dk, rk) < 1e-12
    assert rel_err(dm, rm) < 1e-12
    # homogeneity: sum k dL/dk = sum_s w_s lambda_s = -sum m dL/dm
    lam = tiny.lam[idx]
    assert np.sum(g.k * dk) == pytest.approx(np.sum(w * lam), rel=1e-11)
    assert np.sum(g.masses * dm) == pytest.approx(-np.sum(w * lam), rel=1e-11)


def test_count_parity(tiny):
    banner("estimate_count")
    c, e = F.spectral_map(0.0, tiny.ub)
    lo, hi = 0.05 * tiny.lam[-1], 0.3 * tiny.lam[-1]
    V = gaussian_block(tiny.n, 30, 13)
    est = P.pfe_estimate_count(tiny.h, lo, hi, 200, P.PFE_SMOOTH_JACKSON, V=V)
    ref = count.count_estimate(tiny.H, c, e, (lo - c) / e, (hi - c) / e, V, k=200)
    assert est == pytest.approx(ref, rel=1e-11)
