"""Mass-weighted Hessian H (oracle).  TEST INFRASTRUCTURE ONLY.

Sec. 1, eq. intro.2: H_ij = Delta_ij / sqrt(m_i m_j), where the 3x3 blocks
Delta_ij are the second derivatives of the energy; assembled here from
block-CSR force-constant blocks K (off-diagonal K_ij = -Delta_ij of a bond,
diagonal the negative row sum, so that rigid translations cost no energy).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def block_rows(row_ptr: np.ndarray) -> np.ndarray:
    """Block-row index of every stored block."""
    counts = np.diff(row_ptr)
    return np.repeat(np.arange(counts.shape[0], dtype=np.int64), counts)


def weight_blocks(row_ptr, col_idx, blocks, masses) -> np.ndarray:
    """H blocks: K_ij / sqrt(m_i m_j) on every stored block (eq. intro.2)."""
    rows = block_rows(row_ptr)
    cols = np.asarray(col_idx, dtype=np.int64)
    w = 1.0 / np.sqrt(masses[rows] * masses[cols])
    return blocks * w[:, None, None]


def spring_blocks(row_ptr, col_idx, pairs, unit, k) -> np.ndarray:
    """K on a given block pattern for harmonic springs (eq. intro.1 with the
    pair energy k_p (u_p . (x_j - x_i))^2 / 2): the bond block between i and j
    is -k_p u_p u_p^T, the diagonal block the negative sum of its row's bond
    blocks.  Plain loops over the stored blocks; a block without a spring
    raises."""
    lookup = {(int(i), int(j)): p for p, (i, j) in enumerate(np.asarray(pairs))}
    rows = block_rows(row_ptr)
    K = np.zeros((len(col_idx), 3, 3))
    diag = {}
    for b in range(len(col_idx)):
        i, j = int(rows[b]), int(col_idx[b])
        if i == j:
            diag[i] = b
            continue
        p = lookup[(min(i, j), max(i, j))]
        K[b] = -k[p] * np.outer(unit[p], unit[p])
    for b in range(len(col_idx)):
        i, j = int(rows[b]), int(col_idx[b])
        if i != j:
            K[diag[i]] -= K[b]
    return K


def mapped_blocks(row_ptr, col_idx, hblocks, c: float, e: float) -> np.ndarray:
    """Blocks of H_hat = (H - c I) / e (eq. transf.1): c subtracted on the
    diagonal of every diagonal block, every block divided by e."""
    rows = block_rows(row_ptr)
    out = np.array(hblocks, dtype=np.float64, copy=True)
    diag = rows == np.asarray(col_idx, dtype=np.int64)
    out[diag] -= c * np.eye(3)
    return out / e


def to_bsr(row_ptr, col_idx, hblocks) -> sp.bsr_matrix:
    n_atoms = row_ptr.shape[0] - 1
    return sp.bsr_matrix((np.ascontiguousarray(hblocks), np.asarray(col_idx, dtype=np.int64),
                          np.asarray(row_ptr, dtype=np.int64)),
                         shape=(3 * n_atoms, 3 * n_atoms))


def to_dense(row_ptr, col_idx, hblocks) -> np.ndarray:
    n_atoms = row_ptr.shape[0] - 1
    H = np.zeros((3 * n_atoms, 3 * n_atoms))
    rows = block_rows(row_ptr)
    for b in range(hblocks.shape[0]):
        i, j = rows[b], col_idx[b]
        H[3 * i:3 * i + 3, 3 * j:3 * j + 3] = hblocks[b]
    return H


def glass_H(g):
    """(scipy BSR H, H blocks) of a synthetic glass."""
    hb = weight_blocks(g.row_ptr, g.col_idx, g.blocks, g.masses)
    return to_bsr(g.row_ptr, g.col_idx, hb), hb


def translation_modes(masses: np.ndarray) -> np.ndarray:
    """The three rigid-translation vectors M^{1/2}(1 (x) e_alpha), normalised
    ([n, 3]); they span the null space of H for a periodic spring network."""
    N = masses.shape[0]
    V = np.zeros((3 * N, 3))
    for a in range(3):
        V[a::3, a] = np.sqrt(masses)
    return V / np.linalg.norm(V, axis=0)


def trace_from_springs(pairs, k, masses) -> float:
    """Trace of H from the spring list: each spring adds k u.u (=k) to the
    diagonal blocks of both ends, divided by that end's mass."""
    return float(np.sum(k * (1.0 / masses[pairs[:, 0]] + 1.0 / masses[pairs[:, 1]])))
