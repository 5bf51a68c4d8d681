"""Algorithm 2 (oracle): y = p_d(H_hat) x by the three-term recurrence.

TEST INFRASTRUCTURE ONLY.

H_hat = (H - c I) / e is the spectral map of eq. transf.1 (the paper's
half-width d is called e here to keep d for the degree).  The recurrence is
eq. 3-term-recurrence: t_0 = x, t_1 = H_hat x, t_{k+1} = 2 H_hat t_k - t_{k-1};
y accumulates gamma_k t_k (Algorithm 2).  ``coef`` are the (possibly damped)
coefficients of the filter, gamma_0..gamma_d.
"""
from __future__ import annotations

import numpy as np


def mapped_matvec(H, c: float, e: float):
    """Returns a function v -> (H v - c v) / e."""
    def apply(v):
        return (H @ v - c * v) / e
    return apply


def apply_filter(H, c: float, e: float, coef, X: np.ndarray) -> np.ndarray:
    """p_d(H_hat) X for a block X (columns are independent vectors)."""
    Hh = mapped_matvec(H, c, e)
    coef = np.asarray(coef, dtype=np.float64)
    d = coef.shape[0] - 1
    t2 = np.array(X, dtype=np.float64, copy=True)   # t''
    y = coef[0] * t2
    if d >= 1:
        t1 = Hh(t2)                                  # t'
        y = y + coef[1] * t1
        for k in range(2, d + 1):
            t = 2.0 * Hh(t1) - t2
            t2, t1 = t1, t
            y = y + coef[k] * t
    return y


def filter_via_eig(lam, U, c, e, coef, X):
    """Closed form U p(Lambda_hat) U^T X from a full eigendecomposition, with
    T_j(x) = cos(j arccos x) evaluated on the mapped eigenvalues."""
    x = np.clip((lam - c) / e, -1.0, 1.0)
    j = np.arange(len(coef))
    pv = np.cos(np.outer(np.arccos(x), j)) @ np.asarray(coef)
    return U @ (pv[:, None] * (U.T @ X))
