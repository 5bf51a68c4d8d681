"""Stochastic eigenvalue count (oracle).  TEST INFRASTRUCTURE ONLY.

Sec. 2.4, eq. eigval_count_estimator: mu_[xi,eta] = trace chi_[xi,eta](H)
is estimated by (n/M) sum_l v_l^T psi_k(H_hat) v_l with M unit-norm Gaussian
vectors v_l, psi_k the (damped) truncated Chebyshev series of the
characteristic function, whose coefficients are the Appendix A integral
eq. app.3 over [xi, eta] divided by <T_j, T_j> (eq. cheby-ip.1).
"""
from __future__ import annotations

import numpy as np

from .chebyshev import apply_filter
from .filters import T_norm2, damping, weighted_T_integral


def chi_coefficients(xi, eta, k: int, smoothing="jackson") -> np.ndarray:
    a, b = max(xi, -1.0), min(eta, 1.0)
    gam = np.array([weighted_T_integral(j, a, b) / T_norm2(j) for j in range(k + 1)])
    return damping(smoothing, k) * gam


def count_estimate(H, c, e, xi, eta, V: np.ndarray, k: int = 400, smoothing="jackson") -> float:
    """V: [n, M] Gaussian samples (columns are normalised here)."""
    n, M = V.shape
    Vn = V / np.linalg.norm(V, axis=0)[None, :]
    coef = chi_coefficients(xi, eta, k, smoothing)
    PV = apply_filter(H, c, e, coef, Vn)
    return float(n / M * np.sum(Vn * PV))


def chebyshev_moments(H, c, e, V: np.ndarray, K: int) -> np.ndarray:
    """mu_k = (1/M) sum_l v_l^T T_k(H_hat) v_l, k = 0..K, for the columns of V
    normalised to unit length: the estimator above with psi = T_k, so that
    any window's estimate is n sum_k gamma_k mu_k.  T_k(H_hat) v by the
    three-term recurrence of eq. 3-term-recurrence."""
    n, M = V.shape
    Vn = V / np.linalg.norm(V, axis=0)[None, :]
    mu = np.zeros(K + 1)
    t_prev = Vn
    mu[0] = np.sum(Vn * Vn) / M
    if K >= 1:
        t_cur = (H @ Vn - c * Vn) / e
        mu[1] = np.sum(Vn * t_cur) / M
        for k in range(2, K + 1):
            t_next = 2.0 * (H @ t_cur - c * t_cur) / e - t_prev
            t_prev, t_cur = t_cur, t_next
            mu[k] = np.sum(Vn * t_cur) / M
    return mu


def count_from_moments(mu: np.ndarray, n: int, xi, eta, smoothing="jackson") -> float:
    """Estimated count in the mapped window [xi, eta] from the moments."""
    K = mu.shape[0] - 1
    return float(n * np.dot(chi_coefficients(xi, eta, K, smoothing), mu))
