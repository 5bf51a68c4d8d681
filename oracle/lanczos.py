"""Extremal-eigenvalue bounds by a few Lanczos steps (oracle).

TEST INFRASTRUCTURE ONLY.

Algorithm 3 (step 3) estimates lambda_min and lambda_max "using a few Lanczos
steps"; the map of eq. transf.1 needs an upper bound of lambda_max.  Here: m
steps of Lanczos with full re-orthogonalisation (two classical Gram-Schmidt
passes against all previous basis vectors) from a given start vector; the
largest Ritz value theta_max of the tridiagonal matrix, and the bound
lambda_ub = theta_max + |beta_m s_m|, where s_m is the last component of the
corresponding normalised eigenvector of the tridiagonal matrix (the Ritz
residual norm, so an eigenvalue of H lies within it).  H is positive
semi-definite by construction, so lambda_lb = 0.
"""
from __future__ import annotations

import numpy as np


def lanczos_tridiag(H, v0: np.ndarray, m: int = 30):
    n = v0.shape[0]
    V = np.zeros((n, m + 1))
    alpha = np.zeros(m)
    beta = np.zeros(m)
    V[:, 0] = v0 / np.linalg.norm(v0)
    for j in range(m):
        w = H @ V[:, j]
        alpha[j] = V[:, j] @ w
        w = w - alpha[j] * V[:, j]
        if j > 0:
            w = w - beta[j - 1] * V[:, j - 1]
        for _ in range(2):
            w = w - V[:, :j + 1] @ (V[:, :j + 1].T @ w)
        beta[j] = np.linalg.norm(w)
        V[:, j + 1] = w / beta[j]
    return alpha, beta


def lanczos_bounds(H, v0: np.ndarray, m: int = 30):
    """(lambda_lb, lambda_ub, theta_max)."""
    alpha, beta = lanczos_tridiag(H, v0, m)
    T = np.diag(alpha) + np.diag(beta[:-1], 1) + np.diag(beta[:-1], -1)
    theta, S = np.linalg.eigh(T)
    theta_max = theta[-1]
    lam_ub = theta_max + abs(beta[-1] * S[-1, -1])
    return 0.0, float(lam_ub), float(theta_max)
