"""Pins of the oracle's filter design against values printed in the paper and
against independent quadrature (Sec. 2.3, 2.6, Appendix A, Tables 1-3)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import filters as F

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_filter_values.json")))
SMOOTH = [F.JACKSON, F.LANCZOS, F.NONE]
RVAL = {"0.1": 0.1, "sqrt0.1": math.sqrt(0.1), "quartic0.1": 0.1 ** 0.25}


def test_fig2_target_values():
    g = GOLD["fig2"]
    xi, eta, eps = g["xi"], g["eta"], g["eps"]
    q = F.q_target([xi, eta - 1e-13], xi, eta, eps)
    assert q[0] == pytest.approx(g["q_at_xi"], rel=1e-12)
    assert q[1] == pytest.approx(g["q_at_eta"], rel=1e-9)
    assert F.p_target([(xi + eta) / 2], xi, eta, eps)[0] == pytest.approx(g["p_at_mid"], rel=1e-14)


def test_target_is_c1_symmetric_and_q_is_its_derivative():
    xi, eta, eps = -0.37, -0.21, 0.013
    x = np.linspace(xi - 2 * eps, eta + 2 * eps, 20001)
    p = F.p_target(x, xi, eta, eps)
    # p(xi) = p(eta) = 1, zero outside the margins, symmetric about the midpoint
    assert F.p_target([xi, eta - 1e-15], xi, eta, eps) == pytest.approx([1.0, 1.0], abs=1e-12)
    assert np.all(p[x < xi - eps] == 0) and np.all(p[x >= eta + eps] == 0)
    mid = 0.5 * (xi + eta)
    s = np.linspace(0, 0.5 * (eta - xi) + eps * 0.999, 101)
    np.testing.assert_allclose(F.p_target(mid - s, xi, eta, eps), F.p_target(mid + s, xi, eta, eps), atol=1e-12)
    # q equals the numerical derivative of p everywhere (p is C^1)
    h = 1e-7
    num = (F.p_target(x + h, xi, eta, eps) - F.p_target(x - h, xi, eta, eps)) / (2 * h)
    np.testing.assert_allclose(num, F.q_target(x, xi, eta, eps), atol=2e-3 * (2 / eps))


@pytest.mark.parametrize("xi,eta,eps", [(0.2, 0.3, 0.025), (-0.9, -0.885, 0.002), (-0.995, -0.97, 0.01),
                                        (0.97, 0.99, 0.02)])
def test_coefficients_match_quadrature(xi, eta, eps):
    """Appendix A closed form == trapezoid rule of int_0^pi p(cos t) cos(j t) dt / <T_j,T_j>
    (the cosine substitution of eq. cheby-ip.0); covers pieces clipped at +-1."""
    d = 60
    g = F.pwq_coefficients(xi, eta, eps, d)
    th = np.linspace(0.0, np.pi, 400001)
    pv = F.p_target(np.cos(th), xi, eta, eps)
    for j in range(d + 1):
        ip = np.trapezoid(pv * np.cos(j * th), th)
        assert g[j] == pytest.approx(ip / F.T_norm2(j), abs=2e-8 * max(1.0, np.max(pv)))


def test_weighted_integral_identities():
    # full interval: int T_m / sqrt(1-x^2) = pi delta_m0 (orthogonality against T_0)
    assert F.weighted_T_integral(0, -1.0, 1.0) == pytest.approx(math.pi)
    for m in range(1, 12):
        assert F.weighted_T_integral(m, -1.0, 1.0) == pytest.approx(0.0, abs=1e-14)
    # additivity over a split point
    for m in range(6):
        assert (F.weighted_T_integral(m, -0.3, 0.1) + F.weighted_T_integral(m, 0.1, 0.8)
                == pytest.approx(F.weighted_T_integral(m, -0.3, 0.8), abs=1e-14))


def test_damping_factors():
    for k in (1, 5, 11, 200):
        gj = F.damping(F.JACKSON, k)
        assert gj[0] == pytest.approx(1.0, abs=1e-14)
        # the Jackson factor formula extended to j = k+1 vanishes (alpha_k = pi/(k+2))
        al = math.pi / (k + 2)
        ext = (1 - (k + 1) / (k + 2)) * math.cos((k + 1) * al) + math.cos(al) / math.sin(al) * math.sin((k + 1) * al) / (k + 2)
        assert ext == pytest.approx(0.0, abs=1e-14)
        gl = F.damping(F.LANCZOS, k)
        assert gl[0] == 1.0
        assert gl[k] == pytest.approx(math.sin(k * math.pi / (k + 1)) / (k * math.pi / (k + 1)))
        assert np.all(np.diff(gl) < 0)


def test_jackson_expansion_is_nonnegative():
    """Sec. 2.3: Jackson damping keeps the expansion of a nonnegative function nonnegative."""
    xi, eta, eps = -0.2, 0.2, 0.05
    for k in (11, 40, 150):
        c = F.filter_coefficients(xi, eta, eps, k, F.JACKSON)
        v = F.cheb_eval(c, np.linspace(-1, 1, 4001))
        assert v.min() > -1e-12


def test_fig3_damped_values():
    g = GOLD["fig3"]
    xi, eta, eps, k = g["xi"], g["eta"], g["eps"], g["k"]
    cj = F.filter_coefficients(xi, eta, eps, k, F.JACKSON)
    cl = F.filter_coefficients(xi, eta, eps, k, F.LANCZOS)
    vj = F.cheb_eval(cj, [xi - eps, eta + eps])
    vl = F.cheb_eval(cl, [xi - eps, eta + eps])
    # printed to three significant digits
    assert float(f"{vj[0]:.3g}") == g["jackson_at_xi_minus_eps"]
    assert float(f"{vj[1]:.3g}") == g["jackson_at_eta_plus_eps"]
    assert float(f"{vl[0]:.3g}") == g["lanczos_at_xi_minus_eps"]
    assert float(f"{vl[1]:.3g}") == g["lanczos_at_eta_plus_eps"]


@pytest.mark.parametrize("ti", [0, 1, 2])
def test_table_degrees_piecewise_quadratic(ti):
    t = GOLD["tables"][ti]
    for rkey, degs in t["pwq"].items():
        got = [F.degree_rule(t["xi"], t["eta"], t["eps"], RVAL[rkey], s) for s in SMOOTH]
        assert got == degs, (rkey, got, degs)


@pytest.mark.parametrize("ti", [1, 2])
def test_table_degrees_dirac_full_scan(ti):
    t = GOLD["tables"][ti]
    for phi, degs in t["dirac"].items():
        got = [F.dirac_degree(t["xi"], t["eta"], float(phi), s) for s in SMOOTH]
        assert got == degs, (phi, got, degs)


def test_table1_degrees_dirac_boundary():
    """Table 1's Dirac degrees are large; check the rule flips exactly there."""
    t = GOLD["tables"][0]
    for phi, degs in t["dirac"].items():
        for s, k in zip(SMOOTH, degs):
            def ratio(kk):
                g = F.dirac_balance(t["xi"], t["eta"], kk, s, iters=60)
                v = F.cheb_eval(F.dirac_coefficients(g, kk, s), [t["xi"], g])
                return v[0] / v[1]
            assert ratio(k) <= float(phi) < ratio(k - 1)


def test_spectral_map_worked_example():
    t = GOLD["transf"]
    c, e = F.spectral_map(t["lam_lb"], t["lam_ub"])
    for lo, hi, xlo, xhi in t["windows"]:
        assert (lo - c) / e == pytest.approx(xlo, rel=1e-14)
        assert (hi - c) / e == pytest.approx(xhi, rel=1e-14)


def test_eps_rule_is_smallest_on_grid():
    xi, eta, d, r = -0.98, -0.94, 80, 0.1 ** 0.25
    eps = F.eps_rule(xi, eta, d, r)
    assert F.thresh_holds(F.filter_coefficients(xi, eta, eps, d), xi, eta, eps, r)
    e0 = eps / 1.01
    assert not F.thresh_holds(F.filter_coefficients(xi, eta, e0, d), xi, eta, e0, r)
    # and the degree rule at that eps returns a degree <= d
    assert F.degree_rule(xi, eta, eps, r) <= d
