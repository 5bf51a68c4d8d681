"""Pins of the oracle's filter adjoint and eigenvalue gradients against
Daleckii-Krein, central finite differences, torch CPU autograd, the
Hellmann-Feynman closed forms and homogeneity identities."""
import numpy as np
import pytest
import torch

from oracle import adjoint, chebyshev, filters as F, hessian
from synth import gaussian_block, lattice_glass


@pytest.fixture(scope="module")
def tiny():
    g = lattice_glass(125, seed=3)
    H, hb = hessian.glass_H(g)
    Hd = H.toarray()
    lam, U = np.linalg.eigh(Hd)
    ub = lam[-1] * 1.02
    c, e = F.spectral_map(0.0, ub)
    coef = F.filter_coefficients(-0.9, -0.8, 0.05, 12, F.NONE)
    n = Hd.shape[0]
    X = gaussian_block(n, 3, 21)
    W = gaussian_block(n, 3, 22)
    return g, H, hb, Hd, lam, U, c, e, coef, X, W


def loss(H, c, e, coef, X, W):
    return float(np.sum(W * chebyshev.apply_filter(H, c, e, coef, X)))


def test_self_adjoint(tiny):
    g, H, hb, Hd, lam, U, c, e, coef, X, W = tiny
    Xbar, G = adjoint.filter_vjp_blocks(H, g.row_ptr, g.col_idx, c, e, coef, X, W)
    np.testing.assert_allclose(Xbar, chebyshev.apply_filter(H, c, e, coef, W), atol=1e-12 * np.abs(Xbar).max())


def test_daleckii_krein(tiny):
    """dL/dH for L = <W, p(A) X>, A = (H - cI)/e, equals
    U[(U^T W X^T U) o Gamma]U^T / e, Gamma_ab = (p(a)-p(b))/(a-b), Gamma_aa = p'(a)."""
    g, H, hb, Hd, lam, U, c, e, coef, X, W = tiny
    x = (lam - c) / e
    d = len(coef) - 1
    th = np.arccos(np.clip(x, -1, 1))
    pv = np.cos(np.outer(th, np.arange(d + 1))) @ coef
    # T_j'(x) = j U_{j-1}(x) = j sin(j th)/sin(th)
    j = np.arange(d + 1)
    st = np.sin(th)
    edge = np.abs(st) < 1e-6
    st[edge] = 1.0
    dT = np.sin(np.outer(th, j)) * j[None, :] / st[:, None]
    # at x = +-1: T_j'(+-1) = (+-1)^(j-1) j^2
    dT[edge] = (np.sign(x[edge])[:, None] ** (j[None, :] - 1)) * (j[None, :] ** 2)
    dp = dT @ coef
    dx = x[:, None] - x[None, :]
    with np.errstate(divide="ignore", invalid="ignore"):
        Gam = (pv[:, None] - pv[None, :]) / dx
    close = np.abs(dx) < 1e-9
    Gam[close] = 0.5 * (dp[:, None] + dp[None, :])[close]
    full = U @ ((U.T @ W @ X.T @ U) * Gam) @ U.T / e
    _, G = adjoint.filter_vjp_blocks(H, g.row_ptr, g.col_idx, c, e, coef, X, W)
    ref = np.stack([full[3*i:3*i+3, 3*j:3*j+3] for i, j in
                    zip(hessian.block_rows(g.row_ptr), g.col_idx)])
    np.testing.assert_allclose(G, ref, atol=1e-9 * np.abs(ref).max())


def test_block_gradient_vs_finite_differences(tiny):
    g, H, hb, Hd, lam, U, c, e, coef, X, W = tiny
    _, G = adjoint.filter_vjp_blocks(H, g.row_ptr, g.col_idx, c, e, coef, X, W)
    rng = np.random.default_rng(5)
    h = 1e-6
    for b in rng.choice(hb.shape[0], 12, replace=False):
        p, q = rng.integers(0, 3, 2)
        hp = hb.copy(); hp[b, p, q] += h
        hm = hb.copy(); hm[b, p, q] -= h
        Lp = loss(hessian.to_bsr(g.row_ptr, g.col_idx, hp), c, e, coef, X, W)
        Lm = loss(hessian.to_bsr(g.row_ptr, g.col_idx, hm), c, e, coef, X, W)
        assert G[b, p, q] == pytest.approx((Lp - Lm) / (2 * h), rel=1e-6, abs=1e-8)


def test_block_gradient_vs_torch_autograd(tiny):
    g, H, hb, Hd, lam, U, c, e, coef, X, W = tiny
    Ht = torch.tensor(Hd, dtype=torch.float64, requires_grad=True)
    Xt = torch.tensor(X, dtype=torch.float64, requires_grad=True)
    A = (Ht - c * torch.eye(Hd.shape[0], dtype=torch.float64)) / e
    t0 = Xt; t1 = A @ Xt
    Y = coef[0] * t0 + coef[1] * t1
    for k in range(2, len(coef)):
        t0, t1 = t1, 2 * A @ t1 - t0
        Y = Y + coef[k] * t1
    (torch.tensor(W) * Y).sum().backward()
    Xbar, G = adjoint.filter_vjp_blocks(H, g.row_ptr, g.col_idx, c, e, coef, X, W)
    full = Ht.grad.numpy()
    ref = np.stack([full[3*i:3*i+3, 3*j:3*j+3] for i, j in
                    zip(hessian.block_rows(g.row_ptr), g.col_idx)])
    np.testing.assert_allclose(G, ref, atol=1e-11 * np.abs(ref).max())
    np.testing.assert_allclose(Xbar, Xt.grad.numpy(), atol=1e-11 * np.abs(Xbar).max())


def test_spring_chain_rule_vs_finite_differences(tiny):
    g, H, hb, Hd, lam, U, c, e, coef, X, W = tiny
    Xbar, G = adjoint.filter_vjp_blocks(H, g.row_ptr, g.col_idx, c, e, coef, X, W)
    dk, dm = adjoint.spring_chain_rule(G, hb, g.row_ptr, g.col_idx, g.pairs, g.unit, g.masses)
    from synth.glass import assemble_blocks

    def L_of(k, m):
        rp, ci, kb = assemble_blocks(g.n_atoms, g.pairs, g.unit, k)
        return loss(hessian.to_bsr(rp, ci, hessian.weight_blocks(rp, ci, kb, m)), c, e, coef, X, W)
    rng = np.random.default_rng(17)
    h = 1e-6
    for p in rng.choice(g.k.shape[0], 10, replace=False):
        kp = g.k.copy(); kp[p] += h
        km = g.k.copy(); km[p] -= h
        assert dk[p] == pytest.approx((L_of(kp, g.masses) - L_of(km, g.masses)) / (2 * h), rel=1e-6, abs=1e-9)
    for i in rng.choice(g.n_atoms, 5, replace=False):
        mp = g.masses.copy(); mp[i] += 1e-4
        mm = g.masses.copy(); mm[i] -= 1e-4
        assert dm[i] == pytest.approx((L_of(g.k, mp) - L_of(g.k, mm)) / 2e-4, rel=1e-6, abs=1e-10)


def test_spring_central_difference_recurrence(tiny):
    """The cancellation-free central difference of the filter loss in one
    spring constant equals the plain two-evaluation quotient: to rounding at
    a large step (where the plain quotient loses nothing to cancellation,
    and the h^2 term matters), to the plain quotient's own rounding at
    h = 1e-6, and to the chain-rule derivative of the adjoint to O(h^2)."""
    g, H, hb, Hd, lam, U, c, e, coef, X, W = tiny
    from synth.glass import assemble_blocks
    Xbar, G = adjoint.filter_vjp_blocks(H, g.row_ptr, g.col_idx, c, e, coef, X, W)
    dk, _ = adjoint.spring_chain_rule(G, hb, g.row_ptr, g.col_idx, g.pairs, g.unit, g.masses)

    def L_of(k):
        rp, ci, kb = assemble_blocks(g.n_atoms, g.pairs, g.unit, k)
        return loss(hessian.to_bsr(rp, ci, hessian.weight_blocks(rp, ci, kb, g.masses)), c, e, coef, X, W)
    rng = np.random.default_rng(31)
    for p in rng.choice(g.k.shape[0], 6, replace=False):
        i, j = int(g.pairs[p, 0]), int(g.pairs[p, 1])
        args = (chebyshev.mapped_matvec(H, c, e), e, coef, X, W, i, j, g.unit[p], g.masses[i],
                g.masses[j])
        # the plain quotient at h = 1e-6 carries its own rounding, about
        # 1e-15 |L| / h = 5e-9 here
        for hstep, rel, ab in [(0.3, 1e-11, 0.0), (1e-6, 1e-6, 1e-9 * abs(dk).max())]:
            kp = g.k.copy(); kp[p] += hstep
            km = g.k.copy(); km[p] -= hstep
            plain = (L_of(kp) - L_of(km)) / (2 * hstep)
            quot = adjoint.spring_loss_central_difference(*args, hstep)
            assert quot == pytest.approx(plain, rel=rel, abs=ab)
        assert adjoint.spring_loss_central_difference(*args, 1e-6) == pytest.approx(dk[p], rel=1e-9)


def test_block_sample_vjp_equals_full_vjp(tiny):
    """The memory-lean block-sample VJP reproduces the full one on the
    sampled blocks and in Xbar (same sums, other bookkeeping)."""
    g, H, hb, Hd, lam, U, c, e, coef, X, W = tiny
    Xbar, G = adjoint.filter_vjp_blocks(H, g.row_ptr, g.col_idx, c, e, coef, X, W)
    pick = np.random.default_rng(3).choice(hb.shape[0], 25, replace=False)
    for co in (coef, coef[:2], coef[:1]):
        Xb, Gs = adjoint.filter_vjp_block_sample(chebyshev.mapped_matvec(H, c, e), e, co, X, W,
                                                 g.row_ptr, g.col_idx, pick)
        Xr, Gr = adjoint.filter_vjp_blocks(H, g.row_ptr, g.col_idx, c, e, co, X, W)
        np.testing.assert_allclose(Xb, Xr, rtol=0, atol=1e-13 * np.abs(Xr).max())
        np.testing.assert_allclose(Gs, Gr[pick], rtol=0, atol=1e-13 * max(np.abs(Gr).max(), 1e-300))


def test_mapped_blocks(tiny):
    """H_hat's blocks (eq. transf.1) against (H - c I) / e formed densely."""
    g, H, hb, Hd, lam, U, c, e, coef, X, W = tiny
    Hh = hessian.to_dense(g.row_ptr, g.col_idx, hessian.mapped_blocks(g.row_ptr, g.col_idx, hb, c, e))
    np.testing.assert_allclose(Hh, (Hd - c * np.eye(Hd.shape[0])) / e, rtol=0, atol=1e-15)


def test_hellmann_feynman(tiny):
    g, H, hb, Hd, lam, U, c, e, coef, X, W = tiny
    from synth.glass import assemble_blocks
    # pick two well-separated eigenvalues (the near-cubic lattice has clusters)
    gaps = np.minimum(np.diff(lam)[3:-1], np.diff(lam)[4:])
    picks = 4 + np.argsort(gaps / lam[-1])[::-1][:2]
    assert np.all(gaps[picks - 4] > 1e-4 * lam[-1])
    for idx in picks:
        lam_s, v = lam[idx], U[:, idx]
        G = adjoint.hellmann_feynman_blocks(v, g.row_ptr, g.col_idx)
        dk, dm = adjoint.spring_chain_rule(G, hb, g.row_ptr, g.col_idx, g.pairs, g.unit, g.masses)
        dk2, dm2 = adjoint.hellmann_feynman_springs(lam_s, v, g.pairs, g.unit, g.masses)
        np.testing.assert_allclose(dk, dk2, atol=1e-14 * np.abs(dk2).max() + 1e-18)
        np.testing.assert_allclose(dm, dm2, rtol=1e-12, atol=1e-18)
        # homogeneity: H is linear in k and of degree -1 in the masses
        assert np.sum(g.k * dk) == pytest.approx(lam_s, rel=1e-12)
        assert np.sum(g.masses * dm) == pytest.approx(-lam_s, rel=1e-12)
        # finite differences of a dense eigenvalue (simple, well separated at this size)
        for p in (3, 77):
            # a single spring moves lambda by ~1e-6 per unit of k: a step of 1e-3
            # keeps the dense eigensolver's rounding (~1e-16 ||H||) out of the quotient
            kp = g.k.copy(); kp[p] += 1e-3
            km = g.k.copy(); km[p] -= 1e-3
            def ev(k):
                rp, ci, kb = assemble_blocks(g.n_atoms, g.pairs, g.unit, k)
                return np.linalg.eigvalsh(hessian.to_dense(rp, ci, hessian.weight_blocks(rp, ci, kb, g.masses)))[idx]
            assert dk[p] == pytest.approx((ev(kp) - ev(km)) / 2e-3, rel=1e-5, abs=1e-13)
