"""Filtered subspace iteration with Rayleigh-Ritz (oracle).

TEST INFRASTRUCTURE ONLY.

Algorithm 4 (Rutishauser's subspace iteration) with the matrix replaced by
the filter pi_k(H_hat) as Sec. 3 prescribes, and Algorithm 1's Rayleigh-Ritz
step on H itself.  Readings of the paper taken here:

* Rayleigh-Ritz is done on H (V^T H V), not by an SVD of the filtered
  operator's triangular factor, because the filter maps distinct eigenvalues
  to equal values (Sec. 2.5) and Algorithm 3 states the residuals on H.
* Orthonormalisation and Rayleigh-Ritz happen after every filter
  application (n_RR = 1).
* Orthonormalisation is Householder QR (LAPACK), deliberately not CholQR.
* Residual rho_i = ||H x_i - theta_i x_i|| / lambda_ub, with lambda_ub the
  same upper bound of ||H|| = lambda_max that defines the spectral map.
* Stop when every Ritz value within delta of the window has rho_i <= tol in
  two consecutive iterations with an unchanged in-window count (so at the
  earliest after the second iteration).
"""
from __future__ import annotations

import numpy as np

from .chebyshev import apply_filter


def rayleigh_ritz(H, X):
    W = H @ X
    S = X.T @ W
    S = 0.5 * (S + S.T)
    theta, Q = np.linalg.eigh(S)
    return theta, X @ Q, W @ Q


def subspace_iteration(H, c, e, coef, X0, lam_lo, lam_hi, lam_ub,
                       tol=1e-12, max_iter=100, delta_rel=1e-6, callback=None):
    X, _ = np.linalg.qr(X0)
    delta = delta_rel * lam_ub
    prev_count = -1
    prev_ok = False
    it = 0
    for it in range(1, max_iter + 1):
        Y = apply_filter(H, c, e, coef, X)
        X, _ = np.linalg.qr(Y)
        theta, X, W = rayleigh_ritz(H, X)
        res = np.linalg.norm(W - X * theta[None, :], axis=0) / lam_ub
        near = (theta >= lam_lo - delta) & (theta <= lam_hi + delta)
        inwin = (theta >= lam_lo) & (theta <= lam_hi)
        cnt = int(np.count_nonzero(inwin))
        if callback is not None:
            callback(it, theta, res)
        ok = bool(np.all(res[near] <= tol))
        if ok and prev_ok and cnt == prev_count:
            break
        prev_ok, prev_count = ok, cnt
    inwin = (theta >= lam_lo) & (theta <= lam_hi)
    return theta[inwin], X[:, inwin], res[inwin], it
