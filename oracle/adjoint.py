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


def filter_vjp_block_sample(Hhat, e, coef, X, Ybar, row_ptr, col_idx, blocks):
    """(Xbar, G[blocks]): the sums of filter_vjp_blocks for the listed stored
    blocks only, for sizes where every t_k and a_k cannot be kept: both
    recurrences run in full, but of each vector only the rows of the atoms
    the listed blocks touch are kept.  Hhat(V) returns H_hat V."""
    blocks = np.asarray(blocks, dtype=np.int64)
    bi = block_rows(row_ptr)[blocks]
    bj = np.asarray(col_idx, dtype=np.int64)[blocks]
    atoms = np.unique(np.concatenate([bi, bj]))
    where = {int(a): s for s, a in enumerate(atoms)}
    rows = (3 * atoms[:, None] + np.arange(3)[None, :]).ravel()
    coef = np.asarray(coef, dtype=np.float64)
    d = coef.shape[0] - 1
    # forward: t_0 .. t_{d-1} at the kept rows
    tk = []
    t_prev = np.array(X, dtype=np.float64)
    tk.append(t_prev[rows])
    if d >= 2:
        t_cur = Hhat(t_prev)
        tk.append(t_cur[rows])
        for _ in range(2, d):
            t_prev, t_cur = t_cur, 2.0 * Hhat(t_cur) - t_prev
            tk.append(t_cur[rows])
    # reverse: a_d .. a_1 at the kept rows, then a_0
    ak = [None] * (d + 2)
    a_next2 = np.zeros_like(Ybar)          # a_{k+2}
    a_next = np.zeros_like(Ybar)           # a_{k+1}
    for k in range(d, 0, -1):
        a_k = coef[k] * Ybar + 2.0 * Hhat(a_next) - a_next2
        ak[k] = a_k[rows]
        a_next2, a_next = a_next, a_k
    Xbar = coef[0] * Ybar + (Hhat(a_next) if d >= 1 else 0.0) - a_next2
    G = np.zeros((blocks.shape[0], 3, 3))
    for s in range(blocks.shape[0]):
        ri = slice(3 * where[int(bi[s])], 3 * where[int(bi[s])] + 3)
        rj = slice(3 * where[int(bj[s])], 3 * where[int(bj[s])] + 3)
        if d >= 1:
            G[s] += ak[1][ri] @ tk[0][rj].T
        for k in range(1, d):
            G[s] += 2.0 * (ak[k + 1][ri] @ tk[k][rj].T)
    return Xbar, G / e


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


def spring_loss_central_difference(Hhat, e, coef, X, W, i, j, u, m_i, m_j, h):
    """Central difference [L(k + h) - L(k - h)] / (2 h) of L(k) = <W, p(H_hat) X>
    in the spring constant k of the spring between atoms i and j (unit vector
    u), with c and e held constant; Hhat(V) returns H_hat V = (H V - c V) / e.

    H depends on k through H_ii += k u u^T / m_i, H_jj += k u u^T / m_j,
    H_ij = H_ji -= k u u^T / sqrt(m_i m_j) (eq. intro.2 with K_ij = -k u u^T),
    so H_hat(k +- h) = H_hat +- h E_hat with E_hat = dH/dk / e, which is zero
    outside the rows and columns of atoms i and j.  Subtracting two FP64 losses
    would lose the quotient to cancellation at large n (their rounding, about
    1e-14 |L|, divided by 2h = 2e-6), so the quotient is formed from the two
    recurrences of Algorithm 2 directly: with T+-_k their vectors,
    S_k = (T+_k + T-_k) / 2 and D_k = (T+_k - T-_k) / (2 h) obey
        S_0 = X, D_0 = 0, S_1 = H_hat X, D_1 = E_hat X,
        S_{k+1} = 2 H_hat S_k - S_{k-1} + 2 h^2 E_hat D_k,
        D_{k+1} = 2 H_hat D_k - D_{k-1} + 2 E_hat S_k,
    and the quotient is sum_k g_k <W, D_k>, equal to the two-evaluation
    difference in exact arithmetic.  S and D are advanced side by side as
    one block [S | D]."""
    uu = np.outer(u, u)
    si, sj = slice(3 * i, 3 * i + 3), slice(3 * j, 3 * j + 3)
    mij = np.sqrt(m_i * m_j)

    def Ehat_rows(V):
        """Rows of atoms i and j of E_hat V (its only nonzero rows)."""
        return ((uu @ V[si] / m_i - uu @ V[sj] / mij) / e,
                (uu @ V[sj] / m_j - uu @ V[si] / mij) / e)

    coef = np.asarray(coef, dtype=np.float64)
    d = coef.shape[0] - 1
    if d == 0:
        return 0.0
    q = X.shape[1]
    prev = np.hstack([X, np.zeros_like(X)]).astype(np.float64)      # [S_0 | D_0]
    cur = Hhat(np.hstack([X, np.zeros_like(X)]))                     # [S_1 | D_1]
    cur[:, q:] = 0.0
    ei, ej = Ehat_rows(X)
    cur[si, q:] += ei
    cur[sj, q:] += ej
    quot = coef[1] * float(np.einsum("rc,rc->", W, cur[:, q:]))
    for k in range(1, d):
        es_i, es_j = Ehat_rows(cur[:, :q])          # E_hat S_k
        ed_i, ed_j = Ehat_rows(cur[:, q:])          # E_hat D_k
        nxt = Hhat(cur)
        nxt *= 2.0
        nxt -= prev
        nxt[si, :q] += 2.0 * h * h * ed_i
        nxt[sj, :q] += 2.0 * h * h * ed_j
        nxt[si, q:] += 2.0 * es_i
        nxt[sj, q:] += 2.0 * es_j
        prev, cur = cur, nxt
        quot += coef[k + 1] * float(np.einsum("rc,rc->", W, cur[:, q:]))
    return quot


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
