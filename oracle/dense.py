"""The plain definition (oracle): every eigenpair of H in a closed window.

TEST INFRASTRUCTURE ONLY.

Algorithm 1 asks for the eigenpairs (lambda_i, u_i) with lambda_i in the
closed interval (eq. intro.33); their number is the trace of the spectral
projector (eq. intro.5).  For small n this is a dense LAPACK eigendecomposition
followed by selection.
"""
from __future__ import annotations

import numpy as np


def eigh_all(H_dense: np.ndarray):
    return np.linalg.eigh(H_dense)


def window(lam: np.ndarray, U: np.ndarray, lam_lo: float, lam_hi: float):
    sel = (lam >= lam_lo) & (lam <= lam_hi)
    return lam[sel], U[:, sel]


def count_in(lam: np.ndarray, lo: float, hi: float) -> int:
    """mu_[lo,hi] = |sigma(H) cap [lo, hi]| (eq. intro.5)."""
    return int(np.count_nonzero((lam >= lo) & (lam <= hi)))


def sign_fix(U: np.ndarray) -> np.ndarray:
    """Scale each column so that its largest-magnitude entry is positive."""
    U = np.array(U, copy=True)
    idx = np.argmax(np.abs(U), axis=0)
    s = np.sign(U[idx, np.arange(U.shape[1])])
    s[s == 0] = 1.0
    return U * s
