"""GPU parity of the thick-restart block Lanczos solver on the Dirac-delta
filter (Sec. 2.5 and Sec. 3) against the plain definition (dense LAPACK)."""
import numpy as np
import pytest
import torch

import paper_1902_07041_amd as P
from oracle import dense, hessian, lanczos
from synth import gaussian_vector, lattice_glass

from gpu_common import GlassCase, banner

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def case():
    banner("glass N=1000 (Lanczos)")
    c = GlassCase(1000)
    c.h = c.handle()
    _, c.ub, c.th = lanczos.lanczos_bounds(c.H, gaussian_vector(c.n, 7), 30)
    P.pfe_set_bounds(c.h, 0.0, c.ub)
    c.lo, c.hi = 0.01 * c.th, 0.03 * c.th
    yield c
    P.pfe_destroy(c.h)


def check(H, lam, U, ub, lo, hi, out, ev_tol=1e-10):
    want, V = dense.window(lam, U, lo, hi)
    got = out["evals"]
    assert got.shape == want.shape, (got, want)
    assert np.max(np.abs(got - want) / np.abs(want)) <= ev_tol
    Vg = out["evecs"] if isinstance(out["evecs"], np.ndarray) else out["evecs"].cpu().numpy()
    Vg = Vg.T
    r = np.linalg.norm(H @ Vg - Vg * got[None, :], axis=0) / ub
    assert r.max() <= 1e-9
    assert np.abs(Vg.T @ Vg - np.eye(Vg.shape[1])).max() <= 1e-10
    sv = np.linalg.svd(V.T @ Vg, compute_uv=False)
    assert sv.min() > 1 - 1e-10


@pytest.mark.parametrize("block,basis,smoothing", [(8, 48, P.PFE_SMOOTH_NONE),
                                                   (16, 64, P.PFE_SMOOTH_LANCZOS),
                                                   (4, 40, P.PFE_SMOOTH_JACKSON),
                                                   (24, 408, P.PFE_SMOOTH_NONE)])
def test_lanczos_matches_dense(case, block, basis, smoothing):
    """Against dense LAPACK for three block sizes and dampings; the basis of
    408 columns (plus a residual block of 24) takes the projected matrix's
    eigensolve over many work-groups."""
    banner(f"TR-Lanczos N=1000 b={block} m={basis} smoothing={smoothing}")
    out = P.pfe_solve_lanczos(case.h, case.lo, case.hi, 40, block=block, max_basis=basis,
                              smoothing=smoothing, tol=1e-10)
    assert out["status"] == "PFE_OK"
    assert out["stats"]["iterations"] >= 2
    check(case.H, case.lam, case.U, case.ub, case.lo, case.hi, out)


def test_lanczos_device_vectors(case):
    banner("TR-Lanczos, vectors on the device")
    out = P.pfe_solve_lanczos(case.h, case.lo, case.hi, 40, block=8, max_basis=48, tol=1e-10,
                              vectors_on_device=True)
    assert isinstance(out["evecs"], torch.Tensor) and out["evecs"].is_cuda
    check(case.H, case.lam, case.U, case.ub, case.lo, case.hi, out)


def test_lanczos_capacity(case):
    banner("TR-Lanczos, basis too small")
    with pytest.raises(P.PfeError) as e:
        P.pfe_solve_lanczos(case.h, case.lo, case.hi, 40, block=4, max_basis=16, tol=1e-10)
    assert e.value.status == -6
    with pytest.raises(P.PfeError) as e:
        P.pfe_solve_lanczos(case.h, case.lo, case.hi, 5, block=8, max_basis=48, tol=1e-10)
    assert e.value.status == -6


def test_lanczos_degenerate_lattice():
    """24- and 12-fold eigenvalues: a block Krylov space holds at most `block`
    directions of one eigenspace, so the block is 24, the largest
    multiplicity; the Rayleigh-Ritz step on H over every Ritz vector above tau
    then returns each eigenspace whole."""
    banner("TR-Lanczos, perfect lattice N=216")
    g = lattice_glass(216, seed=1, jitter=0.0, mass_b=63.5, k_lo=1.0, k_hi=1.0)
    H, hb = hessian.glass_H(g)
    lam, U = np.linalg.eigh(H.toarray())
    ub = 1.02 * lam[-1]
    lo, hi = 0.05 * lam[-1], 0.19 * lam[-1]
    h = P.pfe_create(0)
    try:
        P.pfe_set_hessian(h, g.row_ptr, g.col_idx, g.blocks, g.masses)
        P.pfe_set_bounds(h, 0.0, ub)
        out = P.pfe_solve_lanczos(h, lo, hi, 60, block=24, max_basis=144, tol=1e-10)
        check(H, lam, U, ub, lo, hi, out)
        # with a block of 16 the 24-fold eigenvalue comes back 16 times
        out = P.pfe_solve_lanczos(h, lo, hi, 60, block=16, max_basis=128, tol=1e-10)
        assert out["evals"].size == 12 + 16
    finally:
        P.pfe_destroy(h)
