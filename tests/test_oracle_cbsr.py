"""The oracle's C block-CSR product against the dense matrix assembled
independently from the spring list, and against scipy's BSR product."""
import numpy as np
import pytest

from oracle import cbsr, hessian
from synth import gaussian_block, lattice_glass


def test_cbsr_matches_dense_and_scipy():
    g = lattice_glass(343, seed=4)
    hb = hessian.weight_blocks(g.row_ptr, g.col_idx, g.blocks, g.masses)
    op = cbsr.BsrOperator(g.row_ptr, g.col_idx, hb)
    D = hessian.to_dense(g.row_ptr, g.col_idx, hb)
    X = gaussian_block(g.n, 7, 5)
    Y = op @ X
    assert Y.shape == X.shape
    np.testing.assert_allclose(Y, D @ X, rtol=0, atol=1e-13 * np.abs(D).max() * np.abs(X).max() * 60)
    np.testing.assert_array_equal(op @ X[:, 2], Y[:, 2])
    S = hessian.to_bsr(g.row_ptr, g.col_idx, hb)
    np.testing.assert_allclose(Y, S @ X, rtol=1e-14, atol=1e-14 * np.abs(Y).max())


def test_cbsr_empty_rows_and_width_one():
    # two atoms with a single spring plus an isolated third atom
    row_ptr = np.array([0, 2, 4, 5], dtype=np.int64)
    col_idx = np.array([0, 1, 0, 1, 2], dtype=np.int64)
    u = np.array([0.6, 0.0, 0.8])
    K = np.outer(u, u)
    blocks = np.stack([K, -K, -K, K, np.zeros((3, 3))])
    op = cbsr.BsrOperator(row_ptr, col_idx, blocks)
    x = np.arange(9, dtype=np.float64)
    y = op @ x
    want = np.concatenate([K @ (x[0:3] - x[3:6]), K @ (x[3:6] - x[0:3]), np.zeros(3)])
    np.testing.assert_allclose(y, want, rtol=1e-15, atol=1e-15)


def test_spring_blocks_energy_quadratic_form():
    """x^T K x equals sum_p k_p (u_p . (x_j - x_i))^2, twice the harmonic bond
    energy (eq. intro.1); translations cost nothing; the generator's blocks
    agree to rounding."""
    g = lattice_glass(216, seed=6)
    K = hessian.spring_blocks(g.row_ptr, g.col_idx, g.pairs, g.unit, g.k)
    D = hessian.to_dense(g.row_ptr, g.col_idx, K)
    rng = np.random.default_rng(3)
    x = rng.standard_normal((g.n_atoms, 3))
    i, j = g.pairs[:, 0], g.pairs[:, 1]
    want = float(np.sum(g.k * np.einsum("pa,pa->p", g.unit, x[j] - x[i]) ** 2))
    assert float(x.ravel() @ D @ x.ravel()) == pytest.approx(want, rel=1e-13)
    t = np.tile(np.array([0.3, -1.1, 0.7]), g.n_atoms)
    assert np.abs(D @ t).max() <= 1e-13
    np.testing.assert_allclose(K, g.blocks, rtol=0, atol=1e-14 * np.abs(g.blocks).max())
