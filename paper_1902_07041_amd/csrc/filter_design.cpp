// Host-side filter design (Algorithm 3, steps 4 and 6):
//  * spectral map c, e of eq. transf.1 (e is the paper's half-width d);
//  * Chebyshev coefficients of the piecewise-quadratic target p of Sec. 2.6
//    (eq. fct_f) by the exact integrals of Appendix A: each quadratic piece
//    alpha + beta x + gamma x^2 is rewritten in T_0, T_1, T_2 and multiplied
//    into T_j with 2 T_m T_n = T_{m+n} + T_{|m-n|} (eq. app.1); the weighted
//    integrals of T_m over a piece clipped to [-1, 1] are eq. app.3;
//  * damping factors (Jackson eq. jackson_smoothing, Lanczos sigma eq.
//    lanczos_smoothing), multiplied in as in eq. rho_k_smoothened;
//  * the degree / margin rule eq. thresh;
//  * coefficients of the characteristic function for the eigenvalue count
//    (Sec. 2.4).
// Polynomials are evaluated with the three-term recurrence of Sec. 2.2.
#include <cmath>
#include <vector>

#include "internal.h"

namespace pfe {
namespace {

constexpr double kPi = 3.14159265358979323846;

// int_a^b T_m(x) (1 - x^2)^{-1/2} dx, -1 <= a <= b <= 1 (eq. app.3).
double weighted_integral(int m, double a, double b) {
  const double ta = std::acos(a), tb = std::acos(b);
  if (m == 0) return ta - tb;
  return (std::sin(m * ta) - std::sin(m * tb)) / m;
}

// <p, T_j>, j = 0..d, for one quadratic piece on [a, b] (clipped to [-1, 1]).
void add_piece(double a, double b, double al, double be, double ga, int d,
               std::vector<double>& ip) {
  a = std::max(a, -1.0);
  b = std::min(b, 1.0);
  if (!(a < b)) return;
  std::vector<double> I(d + 3);
  for (int m = 0; m <= d + 2; ++m) I[m] = weighted_integral(m, a, b);
  // p = (al + ga/2) T_0 + be T_1 + (ga/2) T_2; times T_j by the product rule
  for (int j = 0; j <= d; ++j) {
    const double t0 = (al + 0.5 * ga) * I[j];
    const double t1 = 0.5 * be * (I[j + 1] + I[std::abs(j - 1)]);
    const double t2 = 0.25 * ga * (I[j + 2] + I[std::abs(j - 2)]);
    ip[j] += t0 + t1 + t2;
  }
}

std::vector<double> pwq_gamma(double xi, double eta, double eps, int d) {
  std::vector<double> ip(d + 1, 0.0);
  const double lo = xi - eps, hi = eta + eps, w = eta - xi;
  // (x - xi + eps)^2 / eps^2 on [xi - eps, xi]
  add_piece(lo, xi, lo * lo / (eps * eps), -2.0 * lo / (eps * eps), 1.0 / (eps * eps), d, ip);
  // 1 + ((eta - xi)^2 - (2x - xi - eta)^2) / (2 eps (eta - xi)) on [xi, eta]
  add_piece(xi, eta, 1.0 - 2.0 * xi * eta / (eps * w), 2.0 * (xi + eta) / (eps * w),
            -2.0 / (eps * w), d, ip);
  // (x - eta - eps)^2 / eps^2 on [eta, eta + eps]
  add_piece(eta, hi, hi * hi / (eps * eps), -2.0 * hi / (eps * eps), 1.0 / (eps * eps), d, ip);
  for (int j = 0; j <= d; ++j) ip[j] /= (j == 0 ? kPi : 0.5 * kPi);   // eq. cheby-ip.1
  return ip;
}

std::vector<double> damping_factors(int kind, int k) {
  std::vector<double> g(k + 1, 1.0);
  if (kind == PFE_SMOOTH_JACKSON) {
    const double al = kPi / (k + 2), cot = std::cos(al) / std::sin(al);
    for (int j = 0; j <= k; ++j)
      g[j] = (1.0 - double(j) / (k + 2)) * std::cos(j * al) + cot * std::sin(j * al) / (k + 2);
  } else if (kind == PFE_SMOOTH_LANCZOS) {
    const double th = kPi / (k + 1);
    for (int j = 1; j <= k; ++j) g[j] = std::sin(j * th) / (j * th);
  }
  return g;
}

// T_0..T_kmax at x by the recurrence.
std::vector<double> cheb_T(double x, int kmax) {
  std::vector<double> T(kmax + 1);
  T[0] = 1.0;
  if (kmax >= 1) T[1] = x;
  for (int j = 2; j <= kmax; ++j) T[j] = 2.0 * x * T[j - 1] - T[j - 2];
  return T;
}

bool thresh_ok(const std::vector<double>& coef, double xi, double eta, double eps, double r) {
  const double lo = xi - eps, hi = eta + eps;
  double vout = -HUGE_VAL;
  bool any = false;
  if (lo >= -1.0) {
    vout = std::max(vout, cheb_value(coef, lo));
    any = true;
  }
  if (hi <= 1.0) {
    vout = std::max(vout, cheb_value(coef, hi));
    any = true;
  }
  if (!any) return true;
  const double vin = std::min(cheb_value(coef, xi), cheb_value(coef, eta));
  return vout <= r * vin;
}

std::vector<double> damped(const std::vector<double>& gam, int smoothing, int k) {
  std::vector<double> g = damping_factors(smoothing, k);
  std::vector<double> c(k + 1);
  for (int j = 0; j <= k; ++j) c[j] = g[j] * gam[j];
  return c;
}

}  // namespace

double cheb_value(const std::vector<double>& coef, double x) {
  double t0 = 1.0, t1 = x, s = coef.empty() ? 0.0 : coef[0];
  if (coef.size() > 1) s += coef[1] * x;
  for (size_t j = 2; j < coef.size(); ++j) {
    const double t2 = 2.0 * x * t1 - t0;
    s += coef[j] * t2;
    t0 = t1;
    t1 = t2;
  }
  return s;
}

std::vector<double> chi_coefficients(double a, double b, int degree, int smoothing) {
  a = std::max(a, -1.0);
  b = std::min(b, 1.0);
  std::vector<double> gam(degree + 1, 0.0);
  if (a < b)
    for (int j = 0; j <= degree; ++j)
      gam[j] = weighted_integral(j, a, b) / (j == 0 ? kPi : 0.5 * kPi);
  return damped(gam, smoothing, degree);
}

Err design_filter(double lam_lo, double lam_hi, double lam_lb, double lam_ub, int degree,
                  double eps, double r, int smoothing, FilterDesign* out) {
  if (!(lam_ub > lam_lb) || !std::isfinite(lam_lb) || !std::isfinite(lam_ub))
    return fail(PFE_EINVAL, "bounds must satisfy lam_lb < lam_ub");
  if (!(lam_hi > lam_lo) || !std::isfinite(lam_lo) || !std::isfinite(lam_hi))
    return fail(PFE_EINVAL, "window must satisfy lam_lo < lam_hi");
  if (smoothing < 0 || smoothing > 2) return fail(PFE_EINVAL, "unknown smoothing");
  if (degree < 0 || eps < 0) return fail(PFE_EINVAL, "degree and eps must be >= 0");
  if (degree == 0 && eps == 0) return fail(PFE_EINVAL, "give a degree, a margin eps, or both");
  if (r == 0) r = std::pow(0.1, 0.25);
  if (!(r > 0 && r < 1)) return fail(PFE_EINVAL, "rate r must lie in (0, 1)");
  const double c = 0.5 * (lam_ub + lam_lb), e = 0.5 * (lam_ub - lam_lb);
  const double xi = (lam_lo - c) / e, eta = (lam_hi - c) / e;
  if (xi < -1.0 || eta > 1.0)
    return fail(PFE_EINVAL, "window must lie inside the spectral bounds");
  FilterDesign f;
  f.c = c;
  f.e = e;
  f.xi = xi;
  f.eta = eta;
  f.r = r;
  f.smoothing = smoothing;
  if (degree > 0 && eps > 0) {
    f.degree = degree;
    f.eps = eps;
  } else if (degree > 0) {
    // smallest eps on the geometric grid eps_min * 1.01^k satisfying eq. thresh
    double ep = (eta - xi) * 1e-3;
    bool found = false;
    while (ep <= 2.0) {
      const std::vector<double> cf = damped(pwq_gamma(xi, eta, ep, degree), smoothing, degree);
      if (thresh_ok(cf, xi, eta, ep, r)) {
        found = true;
        break;
      }
      ep *= 1.01;
    }
    if (!found) return fail(PFE_EINVAL, "no margin satisfies the threshold rule at this degree");
    f.degree = degree;
    f.eps = ep;
  } else {
    // smallest degree k = 1, 2, ... satisfying eq. thresh at eps
    const int kmax = 200000;
    std::vector<double> gam = pwq_gamma(xi, eta, eps, 1024);
    const double pts[4] = {xi, eta, xi - eps, eta + eps};
    int found = 0;
    std::vector<std::vector<double>> T(4);
    int cap = 1024;
    for (int p = 0; p < 4; ++p)
      T[p] = cheb_T(std::min(1.0, std::max(-1.0, pts[p])), cap);
    for (int k = 1; k <= kmax && !found; ++k) {
      if (k > cap) {
        cap *= 2;
        gam = pwq_gamma(xi, eta, eps, cap);
        for (int p = 0; p < 4; ++p) T[p] = cheb_T(std::min(1.0, std::max(-1.0, pts[p])), cap);
      }
      const std::vector<double> g = damping_factors(smoothing, k);
      double v[4] = {0, 0, 0, 0};
      for (int p = 0; p < 4; ++p)
        for (int j = 0; j <= k; ++j) v[p] += g[j] * gam[j] * T[p][j];
      double vout = -HUGE_VAL;
      bool any = false;
      if (pts[2] >= -1.0) {
        vout = std::max(vout, v[2]);
        any = true;
      }
      if (pts[3] <= 1.0) {
        vout = std::max(vout, v[3]);
        any = true;
      }
      if (!any || vout <= r * std::min(v[0], v[1])) found = k;
    }
    if (!found) return fail(PFE_EINVAL, "no degree up to 200000 satisfies the threshold rule");
    f.degree = found;
    f.eps = eps;
  }
  f.coef = damped(pwq_gamma(xi, eta, f.eps, f.degree), smoothing, f.degree);
  *out = std::move(f);
  return ok();
}

// ------------------------------------------------------------- Dirac filter
// rho_k(x) = sum_j g_j T_j(gamma) T_j(x) / <T_j, T_j> (eq. cheby-delta.1 with
// the damping factors g_j of Sec. 2.3), the degree-k stand-in for the Dirac
// distribution at gamma.  gamma in (xi, eta) is balanced so that
// rho_k(xi) = rho_k(eta) (Sec. 2.5), by bisection on rho_k(xi) - rho_k(eta),
// which is positive at gamma = xi and negative at gamma = eta.
std::vector<double> dirac_coef(double gamma, int k, int smoothing) {
  std::vector<double> Tg = cheb_T(std::min(1.0, std::max(-1.0, gamma)), k);
  const std::vector<double> g = damping_factors(smoothing, k);
  std::vector<double> c(k + 1);
  for (int j = 0; j <= k; ++j) c[j] = g[j] * Tg[j] / (j == 0 ? kPi : 0.5 * kPi);
  return c;
}

static double dirac_gamma(double xi, double eta, int k, int smoothing, int iters) {
  auto f = [&](double gm) {
    const std::vector<double> c = dirac_coef(gm, k, smoothing);
    return cheb_value(c, xi) - cheb_value(c, eta);
  };
  double a = xi, b = eta;
  const double fa = f(a);
  for (int it = 0; it < iters; ++it) {
    const double m = 0.5 * (a + b);
    const double fm = f(m);
    if (fm == 0.0) return m;
    if ((fm > 0) == (fa > 0))
      a = m;
    else
      b = m;
  }
  return 0.5 * (a + b);
}

Err design_dirac(double lam_lo, double lam_hi, double lam_lb, double lam_ub, int degree,
                 double phi, int smoothing, DiracDesign* out) {
  if (!(lam_ub > lam_lb) || !std::isfinite(lam_lb) || !std::isfinite(lam_ub))
    return fail(PFE_EINVAL, "bounds must satisfy lam_lb < lam_ub");
  if (!(lam_hi > lam_lo) || !std::isfinite(lam_lo) || !std::isfinite(lam_hi))
    return fail(PFE_EINVAL, "window must satisfy lam_lo < lam_hi");
  if (smoothing < 0 || smoothing > 2) return fail(PFE_EINVAL, "unknown smoothing");
  if (degree < 0) return fail(PFE_EINVAL, "degree must be >= 0");
  if (degree == 0 && !(phi > 0 && phi < 1)) return fail(PFE_EINVAL, "phi must lie in (0, 1)");
  const double c = 0.5 * (lam_ub + lam_lb), e = 0.5 * (lam_ub - lam_lb);
  const double xi = (lam_lo - c) / e, eta = (lam_hi - c) / e;
  if (xi < -1.0 || eta > 1.0) return fail(PFE_EINVAL, "window must lie inside the spectral bounds");
  DiracDesign d;
  d.c = c;
  d.e = e;
  d.xi = xi;
  d.eta = eta;
  d.smoothing = smoothing;
  d.phi = phi;
  int k = degree;
  double gm = 0.5 * (xi + eta);
  if (k == 0) {
    // smallest k with rho_k(xi) / rho_k(gamma) <= phi (Sec. 4.1 tables)
    const int kmax = 20000;
    for (k = 1; k <= kmax; ++k) {
      gm = dirac_gamma(xi, eta, k, smoothing, 60);
      const std::vector<double> cf = dirac_coef(gm, k, smoothing);
      const double top = cheb_value(cf, gm);
      if (top > 0 && cheb_value(cf, xi) / top <= phi) break;
    }
    if (k > kmax) return fail(PFE_EINVAL, "no Dirac degree up to 20000 reaches phi");
  }
  d.degree = k;
  d.gamma = dirac_gamma(xi, eta, k, smoothing, 200);
  d.coef = dirac_coef(d.gamma, k, smoothing);
  d.tau = cheb_value(d.coef, xi);
  d.peak = cheb_value(d.coef, d.gamma);
  *out = std::move(d);
  return ok();
}

}  // namespace pfe
