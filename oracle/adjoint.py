"""Reverse-mode derivative of the filter application (oracle).

TEST INFRASTRUCTURE ONLY.

The paper has no adjoint; this module defines it from Algorithm 2 by the
chain rule.  Forward: t_0 = X, t_1 = A X, t_{k+1} = 2 A t_k - t_{k-1},
Y = sum_k g_k t_k with A = H_hat = (H - c I)/e (c, e held constant).  For a
loss L with dL/dY = Ybar, the adjoint variables a_k = dL/dt_k satisfy
    a_k = g_k Ybar + 2 A a_{k+1} - a_{k+2}        (k = d .. 1, a_{d+1} = a_{d+2} = 0)
    a_0 = g_0 Ybar +   A a_1     - a_2,
so Xbar = a_0, and
    dL/dA = a_1 t_0^T + sum_{k=1}^{d-1} 2 a_{k+1} t_k^T,   dL/dH = dL/dA / e.
On the stored 3x3 blocks (each block an independent parameter) the gradient
is the corresponding 3x3 slice of dL/dH.

Chain rule through the assembly H_ij = K_ij / sqrt(m_i m_j) (eq. intro.2) of a
spring network (K_ij = K_ji = -k u u^T, K_ii = -sum_j K_ij):
    dL/dk_ij = <u u^T, G_ii/m_i + G_jj/m_j - (G_ij + G_ji)/sqrt(m_i m_j)>,
    dL/dm_i  = -(1/(2 m_i)) [sum_j <G_ij, H_ij> + sum_j <G_ji, H_ji>].
Eigenvalue gradients (Hellmann-Feynman, dlambda/dH = v v^T) use the same
chain rule with G = v v^T on the stored blocks.
"""
from __future__ import annotations

import numpy as np

from .chebyshev import mapped_matvec
from .hessian import block_rows


def forward_terms(H, c, e, coef, X):
    """All recurrence vectors t_0..t_d and Y (small cases only)."""
    A = mapped_matvec(H, c, e)
    d = len(coef) - 1
    ts = [np.array(X, dtype=np.float64)]
    if d >= 1:
        ts.append(A(ts[0]))
    for k in range(2, d + 1):
        ts.append(2.0 * A(ts[k - 1]) - ts[k - 2])
    Y = sum(coef[k] * ts[k] for k in range(d + 1))
    return ts, Y


def adjoint_terms(H, c, e, coef, Ybar):
    """a_0..a_d of the reverse recurrence."""
    A = mapped_matvec(H, c, e)
    d = len(coef) - 1
    a = [None] * (d + 3)
    z = np.zeros_like(Ybar)
    a[d + 1] = z
    a[d + 2] = z
    for k in range(d, 0, -1):
        a[k] = coef[k] * Ybar + 2.0 * A(a[k + 1]) - a[k + 2]
    a[0] = coef[0] * Ybar + (A(a[1]) if d >= 1 else 0.0) - a[2]
    return a[:d + 1]


def filter_vjp_blocks(H, row_ptr, col_idx, c, e, coef, X, Ybar):
    """(Xbar, G) with G[b] = dL/dH on stored block b (3x3)."""
    ts, _ = forward_terms(H, c, e, coef, X)
    a = adjoint_terms(H, c, e, coef, Ybar)
    d = len(coef) - 1
    rows = block_rows(row_ptr)
    cols = np.asarray(col_idx, dtype=np.int64)
    nb = cols.shape[0]
    G = np.zeros((nb, 3, 3))

    def add_outer(w, U, V):
        # w * U V^T restricted to stored blocks: G[b][p][q] += w sum_c U[3i+p, c] V[3j+q, c]
        Ur = U.reshape(-1, 3, U.shape[1])
        Vr = V.reshape(-1, 3, V.shape[1])
        G[:] += w * np.einsum("bpc,bqc->bpq", Ur[rows], Vr[cols])

    if d >= 1:
        add_outer(1.0, a[1], ts[0])
    for k in range(1, d):
        add_outer(2.0, a[k + 1], ts[k])
    return a[0], G / e


def spring_chain_rule(G, hblocks, row_ptr, col_idx, pairs, unit, masses):
    """(dL/dk [P], dL/dm [N]) from block gradients G (untied blocks)."""
    rows = block_rows(row_ptr)
    cols = np.asarray(col_idx, dtype=np.int64)
    N = masses.shape[0]
    index = {}
    for b in range(cols.shape[0]):
        index[(int(rows[b]), int(cols[b]))] = b
    P = pairs.shape[0]
    dk = np.zeros(P)
    for p in range(P):
        i, j = int(pairs[p, 0]), int(pairs[p, 1])
        uu = np.outer(unit[p], unit[p])
        gii, gjj = G[index[(i, i)]], G[index[(j, j)]]
        gij, gji = G[index[(i, j)]], G[index[(j, i)]]
        dk[p] = np.sum(uu * (gii / masses[i] + gjj / masses[j]
                             - (gij + gji) / np.sqrt(masses[i] * masses[j])))
    inner = np.sum(G * hblocks, axis=(1, 2))
    dm = np.zeros(N)
    np.add.at(dm, rows, inner)
    np.add.at(dm, cols, inner)
    dm *= -0.5 / masses
    return dk, dm


def hellmann_feynman_blocks(v, row_ptr, col_idx):
    """G[b] = v_i v_j^T on stored block b = (i, j) for a unit eigenvector v."""
    rows = block_rows(row_ptr)
    cols = np.asarray(col_idx, dtype=np.int64)
    vr = v.reshape(-1, 3)
    return np.einsum("bp,bq->bpq", vr[rows], vr[cols])


def hellmann_feynman_springs(lam, v, pairs, unit, masses):
    """Closed forms: dlam/dk_ij = (u.(w_i - w_j))^2, dlam/dm_i = -lam |v_i|^2 / m_i,
    with w_i = v_i / sqrt(m_i)."""
    vr = v.reshape(-1, 3)
    w = vr / np.sqrt(masses)[:, None]
    du = np.einsum("pc,pc->p", unit, w[pairs[:, 0]] - w[pairs[:, 1]])
    dk = du * du
    dm = -lam * np.sum(vr * vr, axis=1) / masses
    return dk, dm
