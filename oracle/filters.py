"""Polynomial filters of the paper, written from their definitions (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* Target ``p`` and its derivative ``q``: Sec. 2.6, eq. fct_f / eq. fct_g.  The
  printed last case "xi - eps < x < 1" is read as "eta + eps < x < 1" (the
  only reading under which p is the C^1 piecewise quadratic the text
  describes and the Fig. 3 values are reproduced).
* Chebyshev coefficients ``gamma_j = <p, T_j> / <T_j, T_j>`` (eq. cheby-ip.2a,
  eq. cheby-ip.1) by the exact integrals of Appendix A (eq. app.1, app.3),
  each quadratic piece clipped to [-1, 1] (end of Sec. 2.6).
* Damping factors: Jackson (eq. jackson_smoothing, alpha_k = pi/(k+2)) and
  Lanczos sigma (eq. lanczos_smoothing, theta_k = pi/(k+1)); eq.
  rho_k_smoothened multiplies them into the coefficients.
* Degree rule (eq. thresh): the smallest k with
  max{pi_k(xi-eps), pi_k(eta+eps)} <= r min{pi_k(xi), pi_k(eta)}, found by
  scanning k = 1, 2, ... (the undamped filter is not monotone in k).  A
  margin end that falls outside [-1, 1] bounds no part of the spectrum, so
  its term is dropped (eq. filter.6 only constrains the spectrum).
* Dirac-delta filter (Sec. 2.5, eq. cheby-delta.1): gamma balanced by
  bisection so that rho_k(xi) = rho_k(eta); its degree is the smallest k with
  rho_k(xi) / rho_k(gamma) <= phi (the tables' "phi", not defined in the
  text; this reading reproduces all their degrees).
"""
from __future__ import annotations

import math

import numpy as np

NONE, JACKSON, LANCZOS = "none", "jackson", "lanczos"


# ----------------------------------------------------------------- targets
def p_target(x, xi, eta, eps):
    """Piecewise-quadratic target p of eq. fct_f (p(xi) = p(eta) = 1)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    m1 = (x >= xi - eps) & (x < xi)
    m2 = (x >= xi) & (x < eta)
    m3 = (x >= eta) & (x < eta + eps)
    out[m1] = (x[m1] - xi + eps) ** 2 / eps ** 2
    out[m2] = 1.0 + ((eta - xi) ** 2 - (2.0 * x[m2] - xi - eta) ** 2) / (2.0 * eps * (eta - xi))
    out[m3] = (x[m3] - eta - eps) ** 2 / eps ** 2
    return out


def q_target(x, xi, eta, eps):
    """Derivative q = p' of eq. fct_g."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    m1 = (x >= xi - eps) & (x < xi)
    m2 = (x >= xi) & (x < eta)
    m3 = (x >= eta) & (x < eta + eps)
    out[m1] = 2.0 / eps ** 2 * (x[m1] - xi + eps)
    out[m2] = 2.0 / (eps * (xi - eta)) * (2.0 * x[m2] - xi - eta)
    out[m3] = 2.0 / eps ** 2 * (x[m3] - eta - eps)
    return out


def pwq_pieces(xi, eta, eps):
    """The three quadratic pieces of p as (a, b, alpha, beta, gamma), with
    p(x) = alpha + beta x + gamma x^2 on [a, b]."""
    lo, hi = xi - eps, eta + eps
    w = eta - xi
    return [
        (lo, xi, lo * lo / eps ** 2, -2.0 * lo / eps ** 2, 1.0 / eps ** 2),
        (xi, eta, 1.0 - 2.0 * xi * eta / (eps * w), 2.0 * (xi + eta) / (eps * w), -2.0 / (eps * w)),
        (eta, hi, hi * hi / eps ** 2, -2.0 * hi / eps ** 2, 1.0 / eps ** 2),
    ]


# --------------------------------------------------- Appendix A integrals
def weighted_T_integral(m: int, a: float, b: float) -> float:
    """eq. app.3: int_a^b T_m(x) / sqrt(1 - x^2) dx for -1 <= a <= b <= 1."""
    ta, tb = math.acos(a), math.acos(b)
    if m == 0:
        return ta - tb
    return (math.sin(m * ta) - math.sin(m * tb)) / m


def pwq_inner_products(xi, eta, eps, d: int) -> np.ndarray:
    """<p, T_j> for j = 0..d, piece by piece, clipped to [-1, 1] (eq. app.1)."""
    out = np.zeros(d + 1)
    for a, b, al, be, ga in pwq_pieces(xi, eta, eps):
        a_c, b_c = max(a, -1.0), min(b, 1.0)
        if not a_c < b_c:
            continue
        I = [weighted_T_integral(m, a_c, b_c) for m in range(d + 3)]
        for j in range(d + 1):
            # x T_j = (T_{j+1} + T_{|j-1|})/2 and x^2 T_j = (T_{j+2} + 2T_j + T_{|j-2|})/4
            out[j] += ((al + ga / 2.0) * I[j]
                       + be / 2.0 * (I[j + 1] + I[abs(j - 1)])
                       + ga / 4.0 * (I[j + 2] + I[abs(j - 2)]))
    return out


def T_norm2(j: int) -> float:
    """eq. cheby-ip.1: <T_j, T_j> = (pi/2)(1 + delta_0j)."""
    return math.pi if j == 0 else math.pi / 2.0


def pwq_coefficients(xi, eta, eps, d: int) -> np.ndarray:
    """Undamped Chebyshev coefficients gamma_0..gamma_d of p (eq. cheby-ip.2a)."""
    ip = pwq_inner_products(xi, eta, eps, d)
    return np.array([ip[j] / T_norm2(j) for j in range(d + 1)])


# ----------------------------------------------------------------- damping
def damping(kind: str, k: int) -> np.ndarray:
    """Smoothing factors g_j^k, j = 0..k."""
    j = np.arange(k + 1, dtype=np.float64)
    if kind == NONE:
        return np.ones(k + 1)
    if kind == JACKSON:
        al = math.pi / (k + 2)
        return (1.0 - j / (k + 2)) * np.cos(j * al) + (1.0 / (k + 2)) * (math.cos(al) / math.sin(al)) * np.sin(j * al)
    if kind == LANCZOS:
        th = math.pi / (k + 1)
        g = np.ones(k + 1)
        g[1:] = np.sin(j[1:] * th) / (j[1:] * th)
        return g
    raise ValueError(kind)


# -------------------------------------------------------------- evaluation
def T_table(x, d: int) -> np.ndarray:
    """T_j(x) = cos(j arccos x) for j = 0..d (Sec. 2.2), rows = j."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    if np.any(np.abs(x) > 1.0):
        raise ValueError("Chebyshev evaluation outside [-1, 1]")
    th = np.arccos(x)
    return np.cos(np.arange(d + 1)[:, None] * th[None, :])


def cheb_eval(coef, x) -> np.ndarray:
    coef = np.asarray(coef, dtype=np.float64)
    return coef @ T_table(x, coef.shape[0] - 1)


def filter_coefficients(xi, eta, eps, d: int, smoothing: str = NONE) -> np.ndarray:
    """Coefficients g_j^d gamma_j of the filter pi_d (eq. rho_k_smoothened)."""
    return damping(smoothing, d) * pwq_coefficients(xi, eta, eps, d)


# ------------------------------------------------------------ degree rule
def _margin_points(xi, eta, eps):
    lo, hi = xi - eps, eta + eps
    return [x for x in (lo, hi) if -1.0 <= x <= 1.0]


def thresh_holds(coef, xi, eta, eps, r) -> bool:
    """eq. thresh for a given coefficient vector."""
    outs = _margin_points(xi, eta, eps)
    vin = cheb_eval(coef, [xi, eta])
    if not outs:
        return True
    vout = cheb_eval(coef, outs)
    return bool(np.max(vout) <= r * np.min(vin))


def degree_rule(xi, eta, eps, r, smoothing=NONE, kmax=20000) -> int:
    """Smallest k >= 1 satisfying eq. thresh (scan k = 1, 2, ...)."""
    gam = pwq_coefficients(xi, eta, eps, kmax)
    outs = _margin_points(xi, eta, eps)
    Tin = T_table([xi, eta], kmax)
    Tout = T_table(outs, kmax) if outs else None
    gin = gam[:, None] * Tin
    gout = gam[:, None] * Tout if outs else None
    for k in range(1, kmax + 1):
        g = damping(smoothing, k)
        vin = g @ gin[: k + 1]
        if not outs:
            return k
        vout = g @ gout[: k + 1]
        if np.max(vout) <= r * np.min(vin):
            return k
    raise RuntimeError("no degree up to kmax satisfies the threshold rule")


def eps_rule(xi, eta, d, r, smoothing=NONE, eps_min=None, eps_max=None, growth=1.01) -> float:
    """Smallest margin eps on a geometric grid (factor ``growth``) for which
    degree d satisfies eq. thresh.  Scans upward from eps_min (default
    (eta - xi)/1000); the first grid point that satisfies the rule is taken."""
    if eps_min is None:
        eps_min = (eta - xi) * 1e-3
    if eps_max is None:
        eps_max = 2.0
    eps = eps_min
    while eps <= eps_max:
        coef = filter_coefficients(xi, eta, eps, d, smoothing)
        if thresh_holds(coef, xi, eta, eps, r):
            return eps
        eps *= growth
    raise RuntimeError("no margin satisfies the threshold rule at this degree")


# ------------------------------------------------------ Dirac-delta filter
def dirac_coefficients(gamma, k: int, smoothing=NONE) -> np.ndarray:
    """eq. cheby-delta.1 with damping: g_j^k T_j(gamma) / <T_j, T_j>."""
    Tg = T_table([gamma], k)[:, 0]
    nrm = np.array([T_norm2(j) for j in range(k + 1)])
    return damping(smoothing, k) * Tg / nrm


def dirac_balance(xi, eta, k: int, smoothing=NONE, iters=200) -> float:
    """gamma in (xi, eta) with rho_k(xi) = rho_k(eta), by bisection."""
    def f(g):
        c = dirac_coefficients(g, k, smoothing)
        v = cheb_eval(c, [xi, eta])
        return v[0] - v[1]
    a, b = xi, eta
    fa = f(a)
    for _ in range(iters):
        mid = 0.5 * (a + b)
        fm = f(mid)
        if fm == 0.0:
            return mid
        if (fm > 0) == (fa > 0):
            a, fa = mid, fm
        else:
            b = mid
    return 0.5 * (a + b)


def dirac_degree(xi, eta, phi, smoothing=NONE, kmax=5000) -> int:
    """Smallest k with rho_k(xi) / rho_k(gamma) <= phi, gamma balanced."""
    for k in range(1, kmax + 1):
        g = dirac_balance(xi, eta, k, smoothing, iters=60)
        c = dirac_coefficients(g, k, smoothing)
        v = cheb_eval(c, [xi, g])
        if v[1] > 0 and v[0] / v[1] <= phi:
            return k
    raise RuntimeError("no Dirac degree up to kmax")


# ------------------------------------------------------------ spectral map
def spectral_map(lam_lb, lam_ub):
    """eq. transf.1: centre c and half-width e (the paper's d) of the bounds."""
    return 0.5 * (lam_ub + lam_lb), 0.5 * (lam_ub - lam_lb)
