"""Pins of the oracle's Hessian, Algorithm 2, Lanczos bounds, subspace
iteration and eigenvalue count against closed forms, invariants and dense
LAPACK (Sec. 1, 2.1, 2.2, 2.4, 3; Algorithms 1, 2, 4)."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import chebyshev, count, dense, filters as F, hessian, lanczos, subspace
from synth import gaussian_block, gaussian_vector, lattice_glass


@pytest.fixture(scope="module")
def g1000():
    g = lattice_glass(1000, seed=1)
    H, hb = hessian.glass_H(g)
    Hd = H.toarray()
    lam, U = np.linalg.eigh(Hd)
    return g, H, hb, Hd, lam, U


def test_hessian_symmetric_and_weighted(g1000):
    g, H, hb, Hd, lam, U = g1000
    assert np.array_equal(Hd, Hd.T)
    # independent assembly of H from the spring list: sum over springs of
    # k (e_i - e_j)(e_i - e_j)^T (x) u u^T, then M^{-1/2} . M^{-1/2}
    N = g.n_atoms
    D = np.zeros((3 * N, 3 * N))
    for (i, j), u, k in zip(g.pairs, g.unit, g.k):
        uu = k * np.outer(u, u)
        D[3*i:3*i+3, 3*i:3*i+3] += uu
        D[3*j:3*j+3, 3*j:3*j+3] += uu
        D[3*i:3*i+3, 3*j:3*j+3] -= uu
        D[3*j:3*j+3, 3*i:3*i+3] -= uu
    s = 1.0 / np.sqrt(np.repeat(g.masses, 3))
    np.testing.assert_allclose(Hd, s[:, None] * D * s[None, :], rtol=0, atol=1e-15)


def test_translation_zero_modes_psd_trace(g1000):
    g, H, hb, Hd, lam, U = g1000
    T = hessian.translation_modes(g.masses)
    assert np.linalg.norm(H @ T) < 1e-13 * lam[-1]
    assert lam[0] >= -1e-14 * lam[-1]
    assert np.count_nonzero(np.abs(lam) < 1e-10 * lam[-1]) == 3
    tr = hessian.trace_from_springs(g.pairs, g.k, g.masses)
    assert lam.sum() == pytest.approx(tr, rel=1e-12)
    assert np.trace(Hd) == pytest.approx(tr, rel=1e-13)


def test_window_count_brute_force(g1000):
    g, H, hb, Hd, lam, U = g1000
    lo, hi = 0.01 * lam[-1], 0.03 * lam[-1]
    assert dense.count_in(lam, lo, hi) == int(sum(1 for v in lam if lo <= v <= hi))
    # projector trace (eq. intro.5) equals the count
    _, V = dense.window(lam, U, lo, hi)
    assert np.trace(V @ V.T) == pytest.approx(dense.count_in(lam, lo, hi), rel=1e-12)


def test_alg2_on_diagonal_matches_closed_form():
    rng = np.random.default_rng(3)
    n = 400
    lam = np.sort(rng.uniform(0.0, 2.0, n))
    H = sp.diags(lam)
    c, e = 1.0, 1.0
    coef = F.filter_coefficients(-0.5, -0.3, 0.05, 120, F.LANCZOS)
    X = rng.standard_normal((n, 5))
    Y = chebyshev.apply_filter(H, c, e, coef, X)
    x = (lam - c) / e
    pv = np.array([sum(coef[j] * math.cos(j * math.acos(xi)) for j in range(len(coef))) for xi in x])
    np.testing.assert_allclose(Y, pv[:, None] * X, rtol=0, atol=1e-12 * np.abs(X).max())


def test_alg2_low_degrees_by_hand():
    rng = np.random.default_rng(4)
    A = rng.standard_normal((30, 30)); A = A + A.T
    X = rng.standard_normal((30, 2))
    c, e = 0.3, 7.0
    Ah = (A - c * np.eye(30)) / e
    # d = 0, 1, 2, 3 written out: T_0 = I, T_1 = x, T_2 = 2x^2 - 1, T_3 = 4x^3 - 3x
    g = [0.7, -1.3, 0.4, 2.1]
    T = [np.eye(30), Ah, 2 * Ah @ Ah - np.eye(30), 4 * Ah @ Ah @ Ah - 3 * Ah]
    for d in range(4):
        ref = sum(g[j] * T[j] for j in range(d + 1)) @ X
        np.testing.assert_allclose(chebyshev.apply_filter(A, c, e, g[:d + 1], X), ref, atol=1e-12)


def test_alg2_dense_spectral(g1000):
    g, H, hb, Hd, lam, U = g1000
    ub = lam[-1] * 1.001
    c, e = F.spectral_map(0.0, ub)
    coef = F.filter_coefficients(-0.98, -0.94, 0.01, 90)
    X = gaussian_block(Hd.shape[0], 4, 5)
    Y = chebyshev.apply_filter(H, c, e, coef, X)
    np.testing.assert_allclose(Y, chebyshev.filter_via_eig(lam, U, c, e, coef, X), atol=1e-12 * np.abs(Y).max())


def test_lanczos_bounds(g1000):
    g, H, hb, Hd, lam, U = g1000
    lb, ub, th = lanczos.lanczos_bounds(H, gaussian_vector(Hd.shape[0], 7), 30)
    assert lb == 0.0
    assert th <= lam[-1] * (1 + 1e-14)
    assert ub >= lam[-1]
    assert (lam[-1] - th) / lam[-1] < 1e-3 and (ub - lam[-1]) / lam[-1] < 1e-2


def test_lanczos_bracket_on_diagonal():
    # theta_max <= lambda_max <= theta_max + |beta_m s_m| (Ritz residual bound)
    for n, m in ((12, 11), (400, 30), (2000, 30)):
        lam = np.linspace(1.0, 3.0, n)
        lb, ub, th = lanczos.lanczos_bounds(sp.diags(lam), np.ones(n), m)
        assert th <= 3.0 <= ub
    # a start vector inside a 4-dimensional invariant subspace: 3 steps leave
    # a 4th direction, and the 4-step tridiagonal matrix has the exact top eigenvalue
    lam = np.linspace(1.0, 3.0, 50)
    v = np.zeros(50); v[[3, 17, 30, 49]] = 1.0
    alpha, beta = lanczos.lanczos_tridiag(sp.diags(lam), v, 3)
    T = np.diag(alpha) + np.diag(beta[:-1], 1) + np.diag(beta[:-1], -1)
    assert np.linalg.eigvalsh(T)[-1] < 3.0


def test_subspace_iteration_matches_dense(g1000):
    g, H, hb, Hd, lam, U = g1000
    n = Hd.shape[0]
    lb, ub, th = lanczos.lanczos_bounds(H, gaussian_vector(n, 7), 30)
    lo, hi = 0.01 * th, 0.03 * th
    c, e = F.spectral_map(lb, ub)
    xi, eta = (lo - c) / e, (hi - c) / e
    d = 80
    eps = F.eps_rule(xi, eta, d, 0.1 ** 0.25)
    coef = F.filter_coefficients(xi, eta, eps, d)
    theta, X, res, it = subspace.subspace_iteration(H, c, e, coef, gaussian_block(n, 32, 11), lo, hi, ub, tol=1e-12)
    ref, V = dense.window(lam, U, lo, hi)
    assert theta.shape == ref.shape and ref.size == 12
    np.testing.assert_allclose(theta, ref, rtol=1e-12)
    assert res.max() <= 1e-12
    # subspaces agree: principal angles via singular values of V^T X
    sv = np.linalg.svd(V.T @ X, compute_uv=False)
    assert sv.min() > 1 - 1e-10


def test_count_estimator(g1000):
    g, H, hb, Hd, lam, U = g1000
    n = Hd.shape[0]
    ub = lam[-1] * 1.01
    c, e = F.spectral_map(0.0, ub)
    lo, hi = 0.05 * lam[-1], 0.25 * lam[-1]
    exact = dense.count_in(lam, lo, hi)
    est = count.count_estimate(H, c, e, (lo - c) / e, (hi - c) / e, gaussian_block(n, 30, 13), k=300)
    # Gaussian estimator with M = 30: relative standard deviation ~ sqrt(2/(M n)) * n / sqrt(mu)
    assert abs(est - exact) < 0.15 * exact, (est, exact)
    # exact trace of the same polynomial (full eigendecomposition) is close to the count
    coef = count.chi_coefficients((lo - c) / e, (hi - c) / e, 300)
    tr = np.sum(F.cheb_eval(coef, np.clip((lam - c) / e, -1, 1)))
    assert abs(tr - exact) < 2.0


def test_chebyshev_moments_closed_form_and_trace():
    """Moments against the eigen-expansion sum_i (u_i.v)^2 cos(k acos lam_i);
    with the unit basis as probes (M = n) the count from the moments is the
    exact trace of the damped series, and any window count equals the
    direct estimator on the same probes."""
    g = lattice_glass(125, seed=3)
    H, _ = hessian.glass_H(g)
    Hd = H.toarray()
    lam, U = np.linalg.eigh(Hd)
    n = Hd.shape[0]
    ub = lam[-1] * 1.02
    c, e = F.spectral_map(0.0, ub)
    V = gaussian_block(n, 7, 5)
    K = 60
    mu = count.chebyshev_moments(H, c, e, V, K)
    Vn = V / np.linalg.norm(V, axis=0)
    w = np.mean((U.T @ Vn) ** 2, axis=1)                      # spectral weights
    x = np.clip((lam - c) / e, -1.0, 1.0)        # zero modes sit at -1 up to rounding
    th = np.arccos(x)
    ref = np.array([np.sum(w * np.cos(k * th)) for k in range(K + 1)])
    np.testing.assert_allclose(mu, ref, rtol=0, atol=1e-12)
    xi, eta = (0.1 * lam[-1] - c) / e, (0.4 * lam[-1] - c) / e
    est = count.count_from_moments(mu, n, xi, eta)
    direct = count.count_estimate(H, c, e, xi, eta, V, k=K)
    assert est == pytest.approx(direct, rel=1e-12)
    mu_all = count.chebyshev_moments(H, c, e, np.eye(n), K)
    tr = np.sum(F.cheb_eval(count.chi_coefficients(xi, eta, K), x))
    assert count.count_from_moments(mu_all, n, xi, eta) == pytest.approx(tr, rel=1e-11)
