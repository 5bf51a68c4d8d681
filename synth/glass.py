"""Seeded harmonic spring-network glass in a periodic cube.

Stand-in for the molecular-dynamics glass Hessians of the paper's experiments
(Section 4.2/4.3), which are not available: same structure (symmetric 3x3
second-derivative blocks between short-range neighbours, a binary mixture of
masses, a periodic box), but sparser (about 17 stored blocks per block row).

Recipe (all draws from one numpy PCG64 stream, in this order):

* ``m = ceil(N^(1/3))`` lattice sites per edge, box side ``B = (N/rho)^(1/3)``
  with number density ``rho = 0.06`` per cubic Angstrom, spacing ``s = B/m``.
* Sites of the simple-cubic ``m^3`` lattice in x-fastest order; if ``m^3 > N``
  a uniform subset of N sites is kept (draw 1), in increasing site order.
* Positions ``(site + U[-0.3, 0.3]^3) * s  mod B`` (draw 2).
* Masses: exactly ``round(0.64 N)`` atoms of 63.5 chosen by a permutation
  (draw 3), the rest 91.2.
* Springs: every minimum-image pair closer than ``1.6 s``, ordered by (i, j)
  with i < j; unit vector u from i to j; stiffness ``k ~ U[0.5, 1.5]`` drawn
  in pair order (draw 4).
* Force-constant blocks (unweighted): ``K_ij = K_ji = -k u u^T`` for a spring,
  ``K_ii = -sum_{j != i} K_ij``.  Assembled as block-CSR with sorted columns
  and the diagonal block always present.

Only the *unweighted* blocks and the masses are produced here; the mass
weighting ``H_ij = K_ij / sqrt(m_i m_j)`` (Section 1, eq. intro.2) is part of
the method and is done separately by the library and by the oracle.
"""
from __future__ import annotations

import dataclasses
import itertools

import numpy as np


@dataclasses.dataclass
class Glass:
    n_atoms: int
    box: float
    spacing: float
    positions: np.ndarray     # [N, 3] float64, Angstrom
    masses: np.ndarray        # [N] float64
    pairs: np.ndarray         # [P, 2] int64, i < j, sorted lexicographically
    unit: np.ndarray          # [P, 3] float64, unit vector i -> j (minimum image)
    k: np.ndarray             # [P] float64 spring constants
    row_ptr: np.ndarray       # [N+1] int64
    col_idx: np.ndarray       # [nnzb] int32, sorted per row, diagonal present
    blocks: np.ndarray        # [nnzb, 3, 3] float64, unweighted K blocks (row-major)

    @property
    def n(self) -> int:
        return 3 * self.n_atoms

    @property
    def nnzb(self) -> int:
        return int(self.col_idx.shape[0])


def _icbrt_ceil(n: int) -> int:
    m = max(1, int(round(n ** (1.0 / 3.0))))
    while m ** 3 < n:
        m += 1
    while m > 1 and (m - 1) ** 3 >= n:
        m -= 1
    return m


def _half_offsets(jitter: float, cutoff: float):
    """Lattice offsets D (one of each +-D pair) whose sites can be within cutoff."""
    out = []
    rng = range(-3, 4)
    for d in itertools.product(rng, rng, rng):
        if d == (0, 0, 0) or d < (0, 0, 0):
            continue
        gap = sum(max(0.0, abs(c) - 2.0 * jitter) ** 2 for c in d)
        if gap < cutoff * cutoff:
            out.append(d)
    return out


def lattice_glass(n_atoms: int, seed: int = 1, density: float = 0.06,
                  jitter: float = 0.3, cutoff: float = 1.6,
                  mass_a: float = 63.5, mass_b: float = 91.2, frac_a: float = 0.64,
                  k_lo: float = 0.5, k_hi: float = 1.5) -> Glass:
    N = int(n_atoms)
    m = _icbrt_ceil(N)
    if m < 5:
        raise ValueError("need at least 5 lattice sites per edge (N >= 65)")
    box = (N / density) ** (1.0 / 3.0)
    s = box / m
    rng = np.random.Generator(np.random.PCG64(seed))
    nsites = m ** 3
    if nsites > N:
        sites = np.sort(rng.choice(nsites, size=N, replace=False)).astype(np.int64)
    else:
        sites = np.arange(N, dtype=np.int64)
    ix = sites % m
    iy = (sites // m) % m
    iz = sites // (m * m)
    lat = np.stack([ix, iy, iz], axis=1).astype(np.float64)
    pos = np.mod((lat + rng.uniform(-jitter, jitter, size=(N, 3))) * s, box)
    perm = rng.permutation(N)
    na = int(round(frac_a * N))
    masses = np.full(N, mass_b, dtype=np.float64)
    masses[perm[:na]] = mass_a

    site_to_atom = np.full(nsites, -1, dtype=np.int64)
    site_to_atom[sites] = np.arange(N, dtype=np.int64)
    rc = cutoff * s
    pi_list, pj_list, d_list = [], [], []
    atoms = np.arange(N, dtype=np.int64)
    for (dx, dy, dz) in _half_offsets(jitter, cutoff):
        nb_site = ((ix + dx) % m) + m * (((iy + dy) % m) + m * ((iz + dz) % m))
        j = site_to_atom[nb_site]
        ok = j >= 0
        i_ok = atoms[ok]
        j_ok = j[ok]
        d = pos[j_ok] - pos[i_ok]
        d -= box * np.round(d / box)
        r2 = np.einsum("ij,ij->i", d, d)
        keep = r2 < rc * rc
        i_k, j_k, d_k = i_ok[keep], j_ok[keep], d[keep]
        swap = i_k > j_k
        lo = np.where(swap, j_k, i_k)
        hi = np.where(swap, i_k, j_k)
        d_k = np.where(swap[:, None], -d_k, d_k)
        pi_list.append(lo)
        pj_list.append(hi)
        d_list.append(d_k)
    pi = np.concatenate(pi_list)
    pj = np.concatenate(pj_list)
    dv = np.concatenate(d_list)
    order = np.lexsort((pj, pi))
    pi, pj, dv = pi[order], pj[order], dv[order]
    if pi.size > 1:
        dup = (pi[1:] == pi[:-1]) & (pj[1:] == pj[:-1])
        if np.any(dup):
            raise RuntimeError("duplicate spring pairs; lattice too small for the cutoff")
    r = np.sqrt(np.einsum("ij,ij->i", dv, dv))
    unit = dv / r[:, None]
    kk = rng.uniform(k_lo, k_hi, size=pi.shape[0])
    pairs = np.stack([pi, pj], axis=1)

    row_ptr, col_idx, blocks = assemble_blocks(N, pairs, unit, kk)
    return Glass(n_atoms=N, box=box, spacing=s, positions=pos, masses=masses,
                 pairs=pairs, unit=unit, k=kk, row_ptr=row_ptr, col_idx=col_idx,
                 blocks=blocks)


def assemble_blocks(N: int, pairs: np.ndarray, unit: np.ndarray, k: np.ndarray):
    """Block-CSR of the unweighted force-constant matrix K of a spring network."""
    P = pairs.shape[0]
    off = -k[:, None, None] * (unit[:, :, None] * unit[:, None, :])     # [P,3,3]
    diag = np.zeros((N, 3, 3), dtype=np.float64)
    np.add.at(diag, pairs[:, 0], -off)
    np.add.at(diag, pairs[:, 1], -off)
    rows = np.concatenate([pairs[:, 0], pairs[:, 1], np.arange(N, dtype=np.int64)])
    cols = np.concatenate([pairs[:, 1], pairs[:, 0], np.arange(N, dtype=np.int64)])
    vals = np.concatenate([off, off, diag], axis=0)
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    counts = np.bincount(rows, minlength=N)
    row_ptr = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    assert row_ptr[-1] == 2 * P + N
    return row_ptr, cols.astype(np.int32), np.ascontiguousarray(vals)


def relabel(g: Glass, seed: int) -> Glass:
    """The same glass with its atoms renumbered by a seeded random permutation,
    as atom ids of a molecular-dynamics snapshot carry no spatial order: new
    atom a is old atom ``perm[a]``.  Springs keep their constants and are
    re-sorted as (i, j), i < j; a unit vector flips with its pair's ends."""
    rng = np.random.Generator(np.random.PCG64(seed))
    N = g.n_atoms
    perm = rng.permutation(N)
    inv = np.empty(N, dtype=np.int64)
    inv[perm] = np.arange(N, dtype=np.int64)
    a, b = inv[g.pairs[:, 0]], inv[g.pairs[:, 1]]
    swap = a > b
    lo, hi = np.where(swap, b, a), np.where(swap, a, b)
    unit = np.where(swap[:, None], -g.unit, g.unit)
    order = np.lexsort((hi, lo))
    pairs = np.stack([lo[order], hi[order]], axis=1)
    unit, k = np.ascontiguousarray(unit[order]), g.k[order]
    row_ptr, col_idx, blocks = assemble_blocks(N, pairs, unit, k)
    return Glass(n_atoms=N, box=g.box, spacing=g.spacing, positions=g.positions[perm],
                 masses=g.masses[perm], pairs=pairs, unit=unit, k=k, row_ptr=row_ptr,
                 col_idx=col_idx, blocks=blocks)


def offdiag_count(g: Glass) -> float:
    """Mean number of spring neighbours per atom."""
    return 2.0 * g.pairs.shape[0] / g.n_atoms
