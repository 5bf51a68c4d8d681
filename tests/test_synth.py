"""The seeded input generator: determinism and the stated recipe."""
import numpy as np

from synth import gaussian_block, lattice_glass, offdiag_count


def test_glass_recipe_and_determinism():
    g = lattice_glass(1000, seed=1)
    g2 = lattice_glass(1000, seed=1)
    assert np.array_equal(g.blocks, g2.blocks) and np.array_equal(g.col_idx, g2.col_idx)
    assert g.n_atoms == 1000 and g.n == 3000
    assert np.count_nonzero(g.masses == 63.5) == 640 and np.count_nonzero(g.masses == 91.2) == 360
    assert abs(g.box - (1000 / 0.06) ** (1 / 3)) < 1e-12
    assert 16.0 < offdiag_count(g) < 17.5
    # sorted columns, diagonal present in every row, pairs i < j, unit vectors
    for i in range(g.n_atoms):
        cols = g.col_idx[g.row_ptr[i]:g.row_ptr[i + 1]]
        assert np.all(np.diff(cols) > 0) and i in cols
    assert np.all(g.pairs[:, 0] < g.pairs[:, 1])
    np.testing.assert_allclose(np.linalg.norm(g.unit, axis=1), 1.0, rtol=1e-14)
    assert g.k.min() >= 0.5 and g.k.max() <= 1.5
    # minimum-image distances below the cutoff
    d = g.positions[g.pairs[:, 1]] - g.positions[g.pairs[:, 0]]
    d -= g.box * np.round(d / g.box)
    assert np.linalg.norm(d, axis=1).max() < 1.6 * g.spacing


def test_glass_with_vacancies():
    g = lattice_glass(3000, seed=2)   # 15^3 = 3375 sites, 375 vacancies
    assert g.n_atoms == 3000
    assert g.row_ptr[-1] == g.nnzb == 2 * g.pairs.shape[0] + 3000


def test_gaussian_block_seeded():
    a = gaussian_block(50, 4, 11)
    assert a.flags["C_CONTIGUOUS"] and a.shape == (50, 4)
    assert np.array_equal(a, gaussian_block(50, 4, 11))
    assert not np.array_equal(a, gaussian_block(50, 4, 12))


def test_relabel_is_the_same_network():
    """Renumbered glass: every block moves with its atoms, K'(a, b) = K(perm a, perm b)."""
    from synth import relabel
    g = lattice_glass(216, seed=3)
    r = relabel(g, 9)
    perm = np.random.Generator(np.random.PCG64(9)).permutation(g.n_atoms)
    def dense(x):
        K = np.zeros((x.n, x.n))
        for i in range(x.n_atoms):
            for k in range(x.row_ptr[i], x.row_ptr[i + 1]):
                j = x.col_idx[k]
                K[3 * i:3 * i + 3, 3 * j:3 * j + 3] = x.blocks[k]
        return K
    p3 = (3 * perm[:, None] + np.arange(3)).ravel()
    # off-diagonal blocks move exactly; a diagonal block is a sum whose order
    # follows the numbering, so it agrees to rounding
    D0, D1 = dense(g)[np.ix_(p3, p3)], dense(r)
    np.testing.assert_allclose(D1, D0, rtol=0, atol=1e-14 * np.abs(D0).max())
    off = ~np.kron(np.eye(g.n_atoms, dtype=bool), np.ones((3, 3), dtype=bool))
    np.testing.assert_array_equal(D1[off], D0[off])
    np.testing.assert_array_equal(r.masses, g.masses[perm])
    assert np.all(r.pairs[:, 0] < r.pairs[:, 1])
    assert np.all(np.diff(r.pairs[:, 0]) >= 0)
    # the numbering is scrambled: most springs join atoms far apart in it
    assert np.median(np.abs(r.pairs[:, 1] - r.pairs[:, 0])) > g.n_atoms / 8
