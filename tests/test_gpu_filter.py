"""GPU parity of the fused Chebyshev filter (Algorithm 2), the Lanczos bounds
and the Hessian import against the CPU oracle."""
import numpy as np
import pytest

import paper_1902_07041_amd as P
from oracle import chebyshev, filters as F, hessian, lanczos
from synth import gaussian_block, gaussian_vector, relabel

from gpu_common import GlassCase, banner, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def case():
    banner("glass N=1000")
    c = GlassCase(1000)
    c.h = c.handle()
    c.ub = float(c.lam[-1]) * 1.01
    P.pfe_set_bounds(c.h, 0.0, c.ub)
    yield c
    P.pfe_destroy(c.h)


def design(case, d, smoothing=P.PFE_SMOOTH_NONE):
    return P.pfe_design_filter(0.01 * case.lam[-1], 0.03 * case.lam[-1], 0.0, case.ub,
                               degree=d, smoothing=smoothing)


@pytest.mark.parametrize("q", [1, 3, 32, 96, 100, 160, 256, 1030])
@pytest.mark.parametrize("d", [0, 1, 2, 3, 30])
def test_filter_fp64_parity(case, q, d):
    banner(f"apply_filter fp64 q={q} d={d}")
    f = design(case, max(d, 1))
    if d < f.degree:
        f.coef = f.coef[: d + 1].copy()
        f.degree = d
    X = gaussian_block(case.n, q, 100 + q)
    Y = P.pfe_apply_filter(case.h, f, X)
    ref = chebyshev.apply_filter(case.H, f.c, f.e, f.coef, X)
    assert rel_err(Y, ref) < 1e-12


@pytest.mark.parametrize("q", [1, 8, 96, 160, 256])
@pytest.mark.parametrize("d", [0, 1, 2, 3, 30])
def test_filter_fp32_parity(case, q, d):
    """Degrees 0-3 take the special first and last launches (degree 0 has no
    matrix term at all: Y = g_0 X)."""
    banner(f"apply_filter fp32 q={q} d={d}")
    f = design(case, max(d, 1))
    if d < f.degree:
        f.coef = f.coef[: d + 1].copy()
        f.degree = d
    X = gaussian_block(case.n, q, 200 + q)
    Y = P.pfe_apply_filter(case.h, f, X.astype(np.float32))
    ref = chebyshev.apply_filter(case.H, f.c, f.e, f.coef, X)
    # FP32 values/vectors: rounding ~6e-8 per operation grows with the degree
    assert rel_err(Y, ref) < 5e-5


def test_filter_device_pointers(case):
    import torch
    banner("apply_filter torch device tensors")
    f = design(case, 20)
    X = gaussian_block(case.n, 64, 7)
    Xt = torch.tensor(X, device="cuda")
    Yt = P.pfe_apply_filter(case.h, f, Xt)
    torch.cuda.synchronize()
    ref = chebyshev.apply_filter(case.H, f.c, f.e, f.coef, X)
    assert rel_err(Yt.cpu().numpy(), ref) < 1e-12


def test_bounds_parity(case):
    banner("estimate_bounds")
    v0 = gaussian_vector(case.n, 7)
    lb, ub, th = P.pfe_estimate_bounds(case.h, 30, v0)
    rlb, rub, rth = lanczos.lanczos_bounds(case.H, v0, 30)
    assert lb == 0.0
    assert th == pytest.approx(rth, rel=1e-12)
    assert ub == pytest.approx(rub, rel=1e-10)
    assert th <= case.lam[-1] * (1 + 1e-13) <= ub
    P.pfe_set_bounds(case.h, 0.0, case.ub)


def test_bounds_own_generator(case):
    banner("estimate_bounds seeded")
    lb, ub, th = P.pfe_estimate_bounds(case.h, 30, None, 5)
    assert th <= case.lam[-1] * (1 + 1e-13) <= ub
    assert (case.lam[-1] - th) / case.lam[-1] < 1e-3
    P.pfe_set_bounds(case.h, 0.0, case.ub)


def test_set_hessian_validation():
    banner("set_hessian validation")
    c = GlassCase(125, seed=2, dense=False)
    h = P.pfe_create(0)
    try:
        g = c.g
        bad = g.blocks.copy()
        bad[1, 0, 1] += 1e-3                       # breaks K_ij = K_ji^T
        with pytest.raises(P.PfeError) as e:
            P.pfe_set_hessian(h, g.row_ptr, g.col_idx, bad, g.masses)
        assert e.value.status == -2
        m = g.masses.copy(); m[5] = -1.0
        with pytest.raises(P.PfeError) as e:
            P.pfe_set_hessian(h, g.row_ptr, g.col_idx, g.blocks, m)
        assert e.value.status == -1
        nanb = g.blocks.copy(); nanb[7, 2, 2] = np.nan
        with pytest.raises(P.PfeError) as e:
            P.pfe_set_hessian(h, g.row_ptr, g.col_idx, nanb, g.masses)
        assert e.value.status == -1
        ci = g.col_idx.copy(); ci[[0, 1]] = ci[[1, 0]]   # unsorted row
        with pytest.raises(P.PfeError):
            P.pfe_set_hessian(h, g.row_ptr, ci, g.blocks, g.masses)
        # calls out of order
        with pytest.raises(P.PfeError) as e:
            P.pfe_solve_interval(h, 0.0, 1.0, 4, 4, degree=10)
        assert e.value.status == -8
        P.pfe_set_hessian(h, g.row_ptr, g.col_idx, g.blocks, g.masses)
    finally:
        P.pfe_destroy(h)


@pytest.mark.parametrize("tile_rows", ["1", "2", "4"])
@pytest.mark.parametrize("q", [1, 96, 160])
def test_filter_row_tile_variants(case, tile_rows, q, monkeypatch):
    """Every tiling of the fused step (rows per tile read at Hessian import)."""
    banner(f"apply_filter tile_rows={tile_rows} q={q}")
    monkeypatch.setenv("PFEIG_TILE_ROWS", tile_rows)
    g = case.g
    h = P.pfe_create(0)
    try:
        # N = 1000 is not a multiple of 4 * 64 rows: ragged last tile and chunk
        P.pfe_set_hessian(h, g.row_ptr, g.col_idx, g.blocks, g.masses)
        P.pfe_set_bounds(h, 0.0, case.ub)
        f = design(case, 25)
        for prec in (np.float64, np.float32):
            X = gaussian_block(case.n, q, 300 + q).astype(prec)
            Y = P.pfe_apply_filter(h, f, X)
            ref = chebyshev.apply_filter(case.H, f.c, f.e, f.coef, X.astype(np.float64))
            assert rel_err(Y, ref) < (1e-12 if prec == np.float64 else 5e-5)
    finally:
        P.pfe_destroy(h)


@pytest.mark.parametrize("tile_rows", ["2", "3"])
@pytest.mark.parametrize("numbering", ["lattice", "random"])
def test_filter_row_orders(case, numbering, tile_rows, monkeypatch):
    """The row tiles in the given numbering and in graph-locality order (and
    the automatic choice) give the same bits, and match the oracle; a random
    numbering exercises tiles of rows far apart in memory."""
    banner(f"apply_filter row orders, {numbering} numbering, tile_rows={tile_rows}")
    monkeypatch.setenv("PFEIG_TILE_ROWS", tile_rows)
    g = case.g if numbering == "lattice" else relabel(case.g, 4)
    H = case.H if numbering == "lattice" else hessian.glass_H(g)[0]
    f = design(case, 25)
    X = gaussian_block(case.n, 96, 77)
    out = {}
    for mode in ["0", "1", None]:
        if mode is None:
            monkeypatch.delenv("PFEIG_ROW_ORDER", raising=False)
        else:
            monkeypatch.setenv("PFEIG_ROW_ORDER", mode)
        h = P.pfe_create(0)
        try:
            P.pfe_set_hessian(h, g.row_ptr, g.col_idx, g.blocks, g.masses)
            P.pfe_set_bounds(h, 0.0, case.ub)
            out[mode] = (P.pfe_apply_filter(h, f, X), P.pfe_apply_filter(h, f, X.astype(np.float32)))
        finally:
            P.pfe_destroy(h)
    ref = chebyshev.apply_filter(H, f.c, f.e, f.coef, X)
    assert rel_err(out["0"][0], ref) < 1e-12
    assert rel_err(out["0"][1], ref) < 5e-5
    for mode in ["1", None]:
        np.testing.assert_array_equal(out[mode][0], out["0"][0])
        np.testing.assert_array_equal(out[mode][1], out["0"][1])


@pytest.mark.parametrize("tile_rows", ["3", "4"])
def test_filter_window_grouping(case, tile_rows, monkeypatch):
    """Tiles of three or more rows regroup the natural order inside windows
    of rows (default, a 64-row window, and none): the same bits in FP64 and
    FP32 (each row sums its blocks in column order), matching the oracle."""
    banner(f"apply_filter with regrouped tiles, tile_rows={tile_rows}")
    monkeypatch.setenv("PFEIG_TILE_ROWS", tile_rows)
    monkeypatch.setenv("PFEIG_TILE_ROWS_F32", tile_rows)
    monkeypatch.setenv("PFEIG_ROW_ORDER", "0")
    f = design(case, 25)
    X = gaussian_block(case.n, 96, 79)
    out = {}
    for w in [None, "64", "0"]:
        if w is None:
            monkeypatch.delenv("PFEIG_TILE_WINDOW", raising=False)
        else:
            monkeypatch.setenv("PFEIG_TILE_WINDOW", w)
        h = P.pfe_create(0)
        try:
            P.pfe_set_hessian(h, case.g.row_ptr, case.g.col_idx, case.g.blocks, case.g.masses)
            P.pfe_set_bounds(h, 0.0, case.ub)
            out[w] = (P.pfe_apply_filter(h, f, X), P.pfe_apply_filter(h, f, X.astype(np.float32)))
        finally:
            P.pfe_destroy(h)
    ref = chebyshev.apply_filter(case.H, f.c, f.e, f.coef, X)
    assert rel_err(out[None][0], ref) < 1e-12
    assert rel_err(out[None][1], ref) < 5e-5
    for w in ["64", "0"]:
        np.testing.assert_array_equal(out[w][0], out[None][0])
        np.testing.assert_array_equal(out[w][1], out[None][1])


def test_device_inputs_ordered_after_torch_default_stream(case):
    """A block that torch is still computing on its default stream when the
    call is made is read complete: the handle's stream is ordered against it."""
    import torch
    banner("apply_filter on a device block still being written by torch")
    f = design(case, 25)
    h = P.pfe_create(0)
    try:
        P.pfe_set_hessian(h, case.g.row_ptr, case.g.col_idx, case.g.blocks, case.g.masses)
        P.pfe_set_bounds(h, 0.0, case.ub)
        for trial in range(3):
            torch.cuda.synchronize()
            X = torch.full((case.n, 64), 0.5, dtype=torch.float64, device="cuda")
            for i in range(200):          # a queue of kernels that X depends on
                X = X + 1e-3 * torch.sin(X + i)
            Y = torch.empty_like(X)
            P.pfe_apply_filter(h, f, X, Y)     # enqueued while torch is busy
            torch.cuda.synchronize()
            ref = P.pfe_apply_filter(h, f, X.cpu().numpy())
            np.testing.assert_array_equal(Y.cpu().numpy(), ref)
    finally:
        P.pfe_destroy(h)


@pytest.mark.parametrize("q", [96, 160, 256])
def test_filter_schedule_does_not_change_bits(case, q, monkeypatch):
    """Work-groups per XCD chunk and columns per pass only change which wave
    computes a row when: every output element sums its blocks in the same
    order, so the results are identical bit for bit."""
    banner(f"apply_filter under other XCD chunkings and column passes, q={q}")
    f = design(case, 25)
    X = gaussian_block(case.n, q, 41)
    out = []
    # column limits: 64 and 128 give equal passes (q = 160: 3 x 54 or 2 x 80),
    # 1024 a single pass on the widest lane layout
    for chunk, cols in [(None, None), ("1", None), ("7", None), ("100000", None), (None, "64"),
                        (None, "128"), (None, "1024")]:
        for name, val in (("PFEIG_CHEB_CHUNK", chunk), ("PFEIG_CHEB_PASS_COLS", cols)):
            if val is None:
                monkeypatch.delenv(name, raising=False)
            else:
                monkeypatch.setenv(name, val)
        out.append(P.pfe_apply_filter(case.h, f, X))
    for Y in out[1:]:
        np.testing.assert_array_equal(Y, out[0])


@pytest.mark.parametrize("shape", ["one_atom", "isolated_atom", "chain5"])
@pytest.mark.parametrize("q", [1, 3])
def test_filter_tiny_patterns(shape, q):
    """The smallest patterns: a single atom (H = 0), an atom without springs
    beside a bonded pair, a 5-atom chain; ragged column counts."""
    from synth.glass import assemble_blocks
    banner(f"apply_filter tiny pattern {shape} q={q}")
    pairs = {"one_atom": [], "isolated_atom": [(0, 1)], "chain5": [(i, i + 1) for i in range(4)]}[shape]
    N = {"one_atom": 1, "isolated_atom": 3, "chain5": 5}[shape]
    rng = np.random.default_rng(8)
    P_ = np.array(pairs, dtype=np.int64).reshape(-1, 2)
    unit = rng.standard_normal((P_.shape[0], 3))
    unit /= np.maximum(np.linalg.norm(unit, axis=1, keepdims=True), 1e-300)
    k = rng.uniform(0.5, 1.5, P_.shape[0])
    masses = rng.uniform(60.0, 90.0, N)
    row_ptr, col_idx, blocks = assemble_blocks(N, P_, unit, k)
    hb = hessian.weight_blocks(row_ptr, col_idx, blocks, masses)
    Hd = hessian.to_dense(row_ptr, col_idx, hb)
    ub = max(1.0, 1.01 * np.linalg.eigvalsh(Hd).max())
    h = P.pfe_create(0)
    try:
        P.pfe_set_hessian(h, row_ptr, col_idx, blocks, masses)
        P.pfe_set_bounds(h, 0.0, ub)
        f = P.pfe_design_filter(0.1 * ub, 0.3 * ub, 0.0, ub, degree=7)
        X = gaussian_block(3 * N, q, 5)
        Y = P.pfe_apply_filter(h, f, X)
        ref = chebyshev.apply_filter(Hd, f.c, f.e, f.coef, X)
        assert np.abs(Y - ref).max() <= 1e-12 * max(np.abs(ref).max(), 1.0)
    finally:
        P.pfe_destroy(h)



def test_set_hessian_requires_the_diagonal_block():
    """Every block row must store its diagonal block (the spectral map's shift
    enters the fused step through it): a 5-atom chain with the diagonal
    blocks of atoms 0 and 3 left out, and one with an empty sixth row, are
    both rejected with EINVAL before any filter runs."""
    from synth.glass import assemble_blocks
    banner("set_hessian rejects rows without their diagonal block")
    rng = np.random.default_rng(9)
    pairs = np.array([(i, i + 1) for i in range(4)], dtype=np.int64)
    unit = rng.standard_normal((4, 3))
    unit /= np.linalg.norm(unit, axis=1, keepdims=True)
    row_ptr5, col_idx5, blocks5 = assemble_blocks(5, pairs, unit, rng.uniform(0.5, 1.5, 4))
    keep = np.ones(col_idx5.size, dtype=bool)
    for i in (0, 3):
        for b in range(row_ptr5[i], row_ptr5[i + 1]):
            keep[b] &= col_idx5[b] != i
    rows = np.repeat(np.arange(5), np.diff(row_ptr5))[keep]
    row_ptr = np.zeros(6, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    masses = rng.uniform(60.0, 90.0, 6)
    h = P.pfe_create(0)
    try:
        with pytest.raises(P.PfeError) as e:      # diagonal blocks of atoms 0 and 3 missing
            P.pfe_set_hessian(h, row_ptr, col_idx5[keep].astype(np.int32), blocks5[keep],
                              masses[:5])
        assert e.value.status == -1
        empty = np.append(row_ptr5, row_ptr5[-1])   # a sixth atom without any block
        with pytest.raises(P.PfeError) as e:
            P.pfe_set_hessian(h, empty, col_idx5, blocks5, masses)
        assert e.value.status == -1
        P.pfe_set_hessian(h, row_ptr5, col_idx5, blocks5, masses[:5])   # the full chain loads
    finally:
        P.pfe_destroy(h)


@pytest.fixture(scope="module")
def dense_cluster():
    """80 atoms with a spring between every pair: 80 blocks per row, so a row
    tile carries more than 64 (column, mask) records."""
    from synth.glass import assemble_blocks
    N = 80
    rng = np.random.default_rng(12)
    pairs = np.array([(i, j) for i in range(N) for j in range(i + 1, N)], dtype=np.int64)
    unit = rng.standard_normal((pairs.shape[0], 3))
    unit /= np.linalg.norm(unit, axis=1, keepdims=True)
    k = rng.uniform(0.5, 1.5, pairs.shape[0])
    masses = rng.uniform(60.0, 90.0, N)
    row_ptr, col_idx, blocks = assemble_blocks(N, pairs, unit, k)
    Hd = hessian.to_dense(row_ptr, col_idx, hessian.weight_blocks(row_ptr, col_idx, blocks, masses))
    ub = 1.01 * np.linalg.eigvalsh(Hd)[-1]
    return row_ptr, col_idx, blocks, masses, Hd, ub


@pytest.mark.parametrize("tile_rows", ["2", "4"])
def test_filter_rows_with_more_than_64_records(dense_cluster, tile_rows, monkeypatch):
    """Tiles whose records fill more than one 64-lane window: FP64 and FP32
    filter and the adjoint (block gradient) against the oracle."""
    from oracle import adjoint
    banner(f"apply_filter / adjoint, 80 blocks per row, tile_rows={tile_rows}")
    monkeypatch.setenv("PFEIG_TILE_ROWS", tile_rows)
    row_ptr, col_idx, blocks, masses, Hd, ub = dense_cluster
    h = P.pfe_create(0)
    try:
        P.pfe_set_hessian(h, row_ptr, col_idx, blocks, masses)
        P.pfe_set_bounds(h, 0.0, ub)
        f = P.pfe_design_filter(0.2 * ub, 0.4 * ub, 0.0, ub, degree=20)
        X = gaussian_block(240, 5, 31)
        ref = chebyshev.apply_filter(Hd, f.c, f.e, f.coef, X)
        Y = P.pfe_apply_filter(h, f, X)
        assert rel_err(Y, ref) < 1e-12
        Y32 = P.pfe_apply_filter(h, f, X.astype(np.float32))
        assert rel_err(Y32, ref) < 5e-5
        W = gaussian_block(240, 5, 32)
        dX, dB = P.pfe_apply_filter_adjoint(h, f, X, W, int(row_ptr[-1]), 0)
        rX, rG = adjoint.filter_vjp_blocks(Hd, row_ptr, col_idx, f.c, f.e, f.coef, X, W)
        assert rel_err(dX, rX) < 1e-12
        assert rel_err(dB, rG) < 1e-11
    finally:
        P.pfe_destroy(h)


def test_fp32_tile_heights_on_one_handle(case, monkeypatch):
    """The FP32 filter walks its own row tiles (three rows by default, the FP64
    filter two); switching their height between calls on one handle rebuilds
    the tiles and the FP32 block order, and every height gives the same bits
    (each row sums its blocks in column order) and matches the oracle."""
    banner("apply_filter fp32, tile heights 2/3/4 on one handle")
    monkeypatch.delenv("PFEIG_TILE_ROWS", raising=False)
    g = case.g
    f = design(case, 25)
    X = gaussian_block(case.n, 96, 51).astype(np.float32)
    ref = chebyshev.apply_filter(case.H, f.c, f.e, f.coef, X.astype(np.float64))
    h = P.pfe_create(0)
    try:
        P.pfe_set_hessian(h, g.row_ptr, g.col_idx, g.blocks, g.masses)
        P.pfe_set_bounds(h, 0.0, case.ub)
        out = []
        for r32 in [None, "2", "4", "3", None]:
            if r32 is None:
                monkeypatch.delenv("PFEIG_TILE_ROWS_F32", raising=False)
            else:
                monkeypatch.setenv("PFEIG_TILE_ROWS_F32", r32)
            out.append(P.pfe_apply_filter(h, f, X))
        assert rel_err(out[0], ref) < 5e-5
        for Y in out[1:]:
            np.testing.assert_array_equal(Y, out[0])
        Y64 = P.pfe_apply_filter(h, f, X.astype(np.float64))   # FP64 tiles untouched
        assert rel_err(Y64, ref) < 1e-12
    finally:
        P.pfe_destroy(h)


def test_new_pattern_on_a_handle_rebuilds_both_tile_sets(case):
    """One handle, two patterns: the glass, then the same glass with its atoms
    renumbered at random (same sizes; the scattered numbering takes the
    locality order).  The second import must rebuild the FP64 and the FP32
    row tiles; both filters match the oracle before and after."""
    banner("apply_filter after a new pattern on the same handle (FP64 and FP32)")
    f = design(case, 25)
    X = gaussian_block(case.n, 96, 61)
    g2 = relabel(case.g, 6)
    H2 = hessian.glass_H(g2)[0]
    h = P.pfe_create(0)
    try:
        for g, H in ((case.g, case.H), (g2, H2), (case.g, case.H)):
            P.pfe_set_hessian(h, g.row_ptr, g.col_idx, g.blocks, g.masses)
            P.pfe_set_bounds(h, 0.0, case.ub)
            ref = chebyshev.apply_filter(H, f.c, f.e, f.coef, X)
            assert rel_err(P.pfe_apply_filter(h, f, X.astype(np.float32)), ref) < 5e-5
            assert rel_err(P.pfe_apply_filter(h, f, X), ref) < 1e-12
    finally:
        P.pfe_destroy(h)


def test_wide_tile_sets_on_one_handle(case, monkeypatch):
    """Blocks wider than 192 columns walk tile sets of their own: four-row
    tiles in FP32 and three-row tiles with a copy of the block values in FP64
    (two-row tiles below).  Every height gives the same bits, a new value set
    on the same pattern refreshes the wide copy, and both match the oracle."""
    banner("apply_filter at q=256: wide tile sets vs the handle's own")
    for v in ("PFEIG_TILE_ROWS", "PFEIG_TILE_ROWS_F32", "PFEIG_TILE_ROWS_F64W"):
        monkeypatch.delenv(v, raising=False)
    g = case.g
    f = design(case, 20)
    X = gaussian_block(case.n, 256, 71)
    h = P.pfe_create(0)
    try:
        for scale in (1.0, 1.5):   # the second value set: H scaled, same pattern
            P.pfe_set_hessian(h, g.row_ptr, g.col_idx, g.blocks * scale, g.masses)
            P.pfe_set_bounds(h, 0.0, case.ub * scale)
            fs = P.pfe_design_filter(0.01 * case.lam[-1] * scale, 0.03 * case.lam[-1] * scale,
                                     0.0, case.ub * scale, degree=20)
            ref = chebyshev.apply_filter(case.H * scale, fs.c, fs.e, fs.coef, X)
            wide64 = P.pfe_apply_filter(h, fs, X)
            wide32 = P.pfe_apply_filter(h, fs, X.astype(np.float32))
            monkeypatch.setenv("PFEIG_TILE_ROWS_F64W", "0")
            monkeypatch.setenv("PFEIG_TILE_ROWS_F32", "3")
            own64 = P.pfe_apply_filter(h, fs, X)
            own32 = P.pfe_apply_filter(h, fs, X.astype(np.float32))
            monkeypatch.delenv("PFEIG_TILE_ROWS_F64W")
            monkeypatch.delenv("PFEIG_TILE_ROWS_F32")
            np.testing.assert_array_equal(wide64, own64)
            np.testing.assert_array_equal(wide32, own32)
            assert rel_err(wide64, ref) < 1e-12
            assert rel_err(wide32, ref) < 5e-5
    finally:
        P.pfe_destroy(h)
