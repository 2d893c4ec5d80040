// Host-side planning: norm estimate, a priori quadrature bound, parameter
// selection and quadrature rules (Section 3.2-3.3 of Croci & Munoz-Matute).
//
// Everything here is scalar FP64 host code; nothing touches the GPU.
#include <cmath>
#include <cstring>
#include <limits>

#include "phiq.h"
#include "phiq_internal.h"

namespace phiq {

namespace {

constexpr double kAlphaZero = 1e-12;  // below this the integrand is a polynomial

// ---------------------------------------------------------------------------
// Real roots of the monic quartic P(r) = r^4 + a3 r^3 + a2 r^2 + a1 r + 1
// lying in (1, inf).  P' is a cubic; its real roots split (1, inf) into
// intervals on which P is monotone, and each sign change is refined by a
// safeguarded Newton iteration.
// ---------------------------------------------------------------------------
inline double quartic(double r, double a3, double a2, double a1) {
  return (((r + a3) * r + a2) * r + a1) * r + 1.0;
}
inline double dquartic(double r, double a3, double a2, double a1) {
  return ((4.0 * r + 3.0 * a3) * r + 2.0 * a2) * r + a1;
}

// Real roots of c3 x^3 + c2 x^2 + c1 x + c0 (c3 != 0), ascending, Newton-polished.
int cubic_real_roots(double c3, double c2, double c1, double c0, double out[3]) {
  const double b = c2 / c3, c = c1 / c3, d = c0 / c3;
  // depressed cubic x = y - b/3:  y^3 + P y + Q = 0
  const double P = c - b * b / 3.0;
  const double Q = 2.0 * b * b * b / 27.0 - b * c / 3.0 + d;
  const double disc = Q * Q / 4.0 + P * P * P / 27.0;
  int k = 0;
  if (disc > 0) {
    const double s = std::sqrt(disc);
    const double u = std::cbrt(-Q / 2.0 + s), w = std::cbrt(-Q / 2.0 - s);
    out[k++] = u + w - b / 3.0;
  } else if (P == 0.0) {
    out[k++] = -b / 3.0;
  } else {
    const double rr = std::sqrt(-P / 3.0);
    double arg = 3.0 * Q / (2.0 * P * rr);
    arg = std::fmax(-1.0, std::fmin(1.0, arg));
    const double phi = std::acos(arg) / 3.0;
    for (int j = 0; j < 3; ++j) out[k++] = 2.0 * rr * std::cos(phi - 2.0 * M_PI * j / 3.0) - b / 3.0;
  }
  for (int j = 0; j < k; ++j) {  // polish
    double x = out[j];
    for (int it = 0; it < 4; ++it) {
      const double f = ((x + b) * x + c) * x + d;
      const double df = (3.0 * x + 2.0 * b) * x + c;
      if (df == 0.0) break;
      const double dx = f / df;
      x -= dx;
      if (std::fabs(dx) <= 1e-16 * std::fabs(x)) break;
    }
    out[j] = x;
  }
  // ascending
  for (int i = 0; i < k; ++i)
    for (int j = i + 1; j < k; ++j)
      if (out[j] < out[i]) std::swap(out[i], out[j]);
  return k;
}

// Root of the quartic inside [lo, hi] where P changes sign and is monotone.
double refine_root(double lo, double hi, double a3, double a2, double a1) {
  double flo = quartic(lo, a3, a2, a1);
  double x = 0.5 * (lo + hi);
  for (int it = 0; it < 200; ++it) {
    const double f = quartic(x, a3, a2, a1);
    if (f == 0.0) return x;
    if ((f < 0) == (flo < 0)) { lo = x; flo = f; } else { hi = x; }
    const double df = dquartic(x, a3, a2, a1);
    double xn = (df != 0.0) ? x - f / df : 0.5 * (lo + hi);
    if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
    if (std::fabs(xn - x) <= 4e-16 * std::fabs(xn) || hi - lo <= 4e-16 * hi) return xn;
    x = xn;
  }
  return x;
}

int quartic_roots_above_one(double a3, double a2, double a1, double roots[4]) {
  double crit[3];
  const int nc = cubic_real_roots(4.0, 3.0 * a3, 2.0 * a2, a1, crit);
  double pts[5];
  int np = 0;
  pts[np++] = 1.0;
  for (int j = 0; j < nc; ++j)
    if (crit[j] > 1.0) pts[np++] = crit[j];
  // Cauchy bound: every root has |r| < 1 + max |a_i|
  const double top = 2.0 + std::fmax(std::fabs(a3), std::fmax(std::fabs(a2), std::fmax(std::fabs(a1), 1.0)));
  const double last = pts[np - 1];
  pts[np++] = std::fmax(top, 2.0 * last);
  int k = 0;
  for (int j = 0; j + 1 < np; ++j) {
    const double lo = pts[j], hi = pts[j + 1];
    const double flo = quartic(lo, a3, a2, a1), fhi = quartic(hi, a3, a2, a1);
    if (flo == 0.0 && lo > 1.0) { roots[k++] = lo; continue; }
    if ((flo < 0) != (fhi < 0)) roots[k++] = refine_root(lo, hi, a3, a2, a1);
  }
  return k;
}

}  // namespace

// eq. polycoeffs, for the bound on phi_{p+1}
void poly_coeffs(double n, int p, double alpha, phiq_rule rule, double* a3, double* a2, double* a1) {
  if (rule == PHIQ_RULE_CC) {
    *a3 = -4.0 / alpha * (n + 1.0 - p);
    *a1 = 4.0 / alpha * (n - 1.0 + p);
  } else {
    *a3 = -4.0 / alpha * (2.0 * (n + 1.0) - p);
    *a1 = 4.0 / alpha * (2.0 * n + p);
  }
  *a2 = -(2.0 + 8.0 * p / alpha);
}

// log of the Thm 3.2 bound at rho (for phi_{p+1}, (n+1)-node rule).
double log_bound_at(double rho, double n, int p, double alpha, double beta, phiq_rule rule) {
  const double g = (rho + 1.0) * (rho + 1.0) / (2.0 * rho);
  const double logM = p * std::log(g) - (p + 1) * M_LN2 - std::lgamma(p + 1.0) + 0.5 * g * alpha + std::log(beta);
  const double lr = (rule == PHIQ_RULE_CC) ? (1.0 - n) * std::log(rho) : -2.0 * n * std::log(rho);
  return std::log(144.0 / 35.0) + logM + lr - std::log(rho * rho - 1.0);
}

// min over the quartic's real roots > 1 of the bound; +inf if none.
double best_log_bound(double n, int p, double alpha, double beta, phiq_rule rule) {
  double a3, a2, a1;
  poly_coeffs(n, p, alpha, rule, &a3, &a2, &a1);
  double roots[4];
  const int k = quartic_roots_above_one(a3, a2, a1, roots);
  double best = std::numeric_limits<double>::infinity();
  for (int j = 0; j < k; ++j) best = std::fmin(best, log_bound_at(roots[j], n, p, alpha, beta, rule));
  return best;
}

// Algorithm quaderr (log form)
double log_quaderr(double n, int p, double alpha, double beta, phiq_rule rule) {
  double E = -std::numeric_limits<double>::infinity();
  for (int q = 1; q <= p; ++q) E = std::fmax(E, best_log_bound(n, q - 1, alpha, beta, rule));
  return E;
}

// Brent's method (Brent, 1973) for a sign change of f on [a, b].
template <class F>
double brent_root(F&& f, double a, double b, double fa, double fb, double tol) {
  double c = a, fc = fa, d = b - a, e = d;
  for (int it = 0; it < 200; ++it) {
    if ((fb > 0) == (fc > 0)) { c = a; fc = fa; d = b - a; e = d; }
    if (std::fabs(fc) < std::fabs(fb)) { a = b; b = c; c = a; fa = fb; fb = fc; fc = fa; }
    const double tol1 = 2.0 * 2.2e-16 * std::fabs(b) + 0.5 * tol;
    const double xm = 0.5 * (c - b);
    if (std::fabs(xm) <= tol1 || fb == 0.0) return b;
    if (std::fabs(e) >= tol1 && std::fabs(fa) > std::fabs(fb)) {
      double s = fb / fa, pp, qq;
      if (a == c) {
        pp = 2.0 * xm * s;
        qq = 1.0 - s;
      } else {
        const double q0 = fa / fc, r = fb / fc;
        pp = s * (2.0 * xm * q0 * (q0 - r) - (b - a) * (r - 1.0));
        qq = (q0 - 1.0) * (r - 1.0) * (s - 1.0);
      }
      if (pp > 0) qq = -qq;
      pp = std::fabs(pp);
      if (2.0 * pp < std::fmin(3.0 * xm * qq - std::fabs(tol1 * qq), std::fabs(e * qq))) {
        e = d;
        d = pp / qq;
      } else {
        d = xm;
        e = d;
      }
    } else {
      d = xm;
      e = d;
    }
    a = b;
    fa = fb;
    b += (std::fabs(d) > tol1) ? d : (xm > 0 ? tol1 : -tol1);
    fb = f(b);
  }
  return b;
}

// Algorithm quadnodes: the paper's n (rule of n+1 nodes)
int quadnodes(double eps, int p, double alpha, double beta, phiq_rule rule) {
  int n = (rule == PHIQ_RULE_GAUSS) ? 2 : 4;
  const double leps = std::log(eps);
  double E = log_quaderr(n, p, alpha, beta, rule);
  if (E <= leps) return n;
  while (E > leps) {
    if (n > (1 << 24)) return -1;
    n *= 2;
    E = log_quaderr(n, p, alpha, beta, rule);
  }
  auto h = [&](double x) { return log_quaderr(x, p, alpha, beta, rule) - leps; };
  const double a = 0.5 * n, b = n;
  const double root = brent_root(h, a, b, h(a), E - leps, 1e-12);
  return (int)std::ceil(root);
}

// Algorithm setup_quadrature
void setup_quadrature(double eps, int p, double alpha, double beta, phiq_rule rule, double c1,
                      double c2, int d, int* l_out, int* n_out, double* cost_out) {
  if (p == 0) { *l_out = 0; *n_out = -1; *cost_out = 0.0; return; }
  if (alpha <= kAlphaZero) {
    const int m = std::max(1, (p + 1) / 2);
    *l_out = 0; *n_out = m - 1; *cost_out = c1 * d * (m - 1) + c2 * (m - 1);
    return;
  }
  const int lmax = std::max(0, (int)std::ceil(std::log2(alpha)));
  int bl = -1, bn = -1;
  double bc = std::numeric_limits<double>::infinity();
  for (int l = lmax; l >= 0; --l) {
    const double al = std::ldexp(alpha, -l);
    const int n = quadnodes(eps, p, al, beta, rule);
    if (n < 0) break;
    const double C = c1 * d * n + c2 * (n + (double)l * p);
    if (C < bc) { bc = C; bl = l; bn = n; } else break;
  }
  *l_out = bl; *n_out = bn; *cost_out = bc;
}

// Scaling for adaptive Clenshaw-Curtis by the cost Algorithm 2 will have.
// Algorithm 2 runs the nested rules of S_j = 6 2^j + 1 points (j = 0, 1, ...)
// and stops at the first level j >= 1 whose change from level j - 1 is below
// eps, i.e. about one level after the first rule that is accurate: it pays
// S_{j+1} node chains for a rule with S_j nodes.  Whether a 7-point rule is
// accurate or needs 13 decides between 13 and 25 node chains, which costs
// more than a squaring step (p chains).  The prediction uses the CC bound of
// Thm 3.2 at a quarter of the norm: on 3D advection-diffusion draws the bound
// at the full norm predicted the level Algorithm 2 stopped at in 28 of 64
// cases (always one level too late), at a quarter in 60 of 64 (the rest one
// level too late).  A wrong prediction costs time only: the stopping test
// still decides.  l ranges over [l_paper - 1, l_paper + 3] with the paper's
// cost C = c1 d n + c2 (n + l p), n + 1 = the nodes run; ties keep the
// smaller l; if no l is predicted to converge within max_doublings, the
// paper's l.
int cc_scaling(double eps, int p, double alpha, double c1, double c2, int d, int max_doublings, int l_paper) {
  constexpr double kNormFraction = 0.25;
  if (p == 0 || alpha <= kAlphaZero || l_paper < 0) return l_paper;
  const double leps = std::log(eps);
  int bl = l_paper;
  double bc = std::numeric_limits<double>::infinity();
  for (int l = std::max(0, l_paper - 1); l <= l_paper + 3; ++l) {
    const double al = std::ldexp(alpha * kNormFraction, -l);
    int acc = -1;  // first level whose rule the bound accepts
    for (int j = 0; j < max_doublings && acc < 0; ++j)
      if (log_quaderr(6 * (1 << j), p, al, 1.0, PHIQ_RULE_CC) <= leps) acc = j;
    if (acc < 0) continue;
    const int n = 6 << std::max(1, acc + 1);  // the stopping level's rule has n + 1 points
    const double C = c1 * d * n + c2 * (n + (double)l * p);
    if (C < bc) {
      bc = C;
      bl = l;
    }
  }
  return bl;
}

// ---------------------------------------------------------------------------
// Quadrature rules on [0, 1]
// ---------------------------------------------------------------------------
// Gauss-Legendre: Newton on P_m from the Tricomi-type initial guesses,
// weights 2/((1-x^2) P_m'(x)^2), mapped by theta = (1+x)/2, w = omega/2.
namespace {
// P_m(x) and P_{m-1}(x) by the three-term recurrence (m >= 1).
void legendre_pair(int m, double x, double* pm, double* pm1) {
  double a = 1.0, b = x;  // P_0, P_1
  for (int k = 2; k <= m; ++k) {
    const double c = ((2.0 * k - 1.0) * x * b - (k - 1.0) * a) / k;
    a = b;
    b = c;
  }
  *pm = b;
  *pm1 = a;
}
}  // namespace

void gauss_legendre(int m, double* theta, double* w) {
  for (int i = 0; i < (m + 1) / 2; ++i) {
    double x = std::cos(M_PI * (i + 0.75) / (m + 0.5));
    double pm, pm1;
    for (int it = 0; it < 100; ++it) {
      legendre_pair(m, x, &pm, &pm1);
      const double dp = m * (x * pm - pm1) / (x * x - 1.0);
      const double dx = pm / dp;
      x -= dx;
      if (std::fabs(dx) <= 1e-16) break;
    }
    legendre_pair(m, x, &pm, &pm1);
    const double dp = m * (x * pm - pm1) / (x * x - 1.0);
    const double om = 2.0 / ((1.0 - x * x) * dp * dp);
    // x is the (i+1)-th largest root; -x is its mirror image
    theta[m - 1 - i] = 0.5 * (1.0 + x);
    w[m - 1 - i] = 0.5 * om;
    theta[i] = 0.5 * (1.0 - x);
    w[i] = 0.5 * om;
  }
  if (m % 2 == 1) theta[m / 2] = 0.5;
}

// Clenshaw-Curtis with n+1 = m points: interpolate at x_j = cos(j pi/n) by
// sum'' a_k T_k and integrate, int_{-1}^{1} T_k = 2/(1-k^2) (k even), 0 (odd).
void clenshaw_curtis(int m, double* theta, double* w) {
  const int n = m - 1;
  for (int j = 0; j <= n; ++j) {
    double s = 0.0;
    for (int k = 0; k <= n; k += 2) {
      const double mom = 2.0 / (1.0 - (double)k * k);
      const double half = (k == 0 || k == n) ? 0.5 : 1.0;
      s += half * mom * std::cos(M_PI * (double)k * j / n);
    }
    const double endw = (j == 0 || j == n) ? 0.5 : 1.0;
    const double omega = endw * 2.0 / n * s;
    theta[j] = 0.5 * (1.0 + std::cos(M_PI * (double)j / n));
    w[j] = 0.5 * omega;
  }
}

}  // namespace phiq

// ---------------------------------------------------------------------------
// C ABI (host-only part)
// ---------------------------------------------------------------------------
extern "C" {

phiq_status phiq_norm_bound(const phiq_kron_op* op, double t, double* alpha) {
  if (!op || !alpha) return PHIQ_ERR_INVALID_ARG;
  phiq_status st = phiq::validate_op(op);
  if (st != PHIQ_OK) return st;
  if (!std::isfinite(t)) return PHIQ_ERR_NONFINITE;
  *alpha = std::fabs(t) * phiq::sum_infnorms(op);
  return PHIQ_OK;
}

phiq_status phiq_setup_quadrature(double eps, int p, double alpha, double beta, phiq_rule rule,
                                  double c1, double c2, int d, int* l, int* n, double* cost) {
  if (!l || !n || !cost) return PHIQ_ERR_INVALID_ARG;
  if (!std::isfinite(eps) || !std::isfinite(alpha) || !std::isfinite(beta) || !std::isfinite(c1) ||
      !std::isfinite(c2))
    return PHIQ_ERR_NONFINITE;
  if (eps <= 0 || p < 0 || p > PHIQ_MAX_P || alpha < 0 || beta <= 0 || c1 < 0 || c2 < 0 || d < 1 ||
      (rule != PHIQ_RULE_GAUSS && rule != PHIQ_RULE_CC))
    return PHIQ_ERR_INVALID_ARG;
  phiq::setup_quadrature(eps, p, alpha, beta, rule, c1, c2, d, l, n, cost);
  if (*l < 0) return PHIQ_ERR_NOT_CONVERGED;
  return PHIQ_OK;
}

phiq_status phiq_cc_scaling(double eps, int p, double alpha, double c1, double c2, int d, int max_doublings,
                            int* l) {
  if (!l) return PHIQ_ERR_INVALID_ARG;
  if (!std::isfinite(eps) || !std::isfinite(alpha) || !std::isfinite(c1) || !std::isfinite(c2))
    return PHIQ_ERR_NONFINITE;
  if (eps <= 0 || p < 0 || p > PHIQ_MAX_P || alpha < 0 || c1 < 0 || c2 < 0 || d < 1 || max_doublings < 1 ||
      max_doublings > 10)
    return PHIQ_ERR_INVALID_ARG;
  int lp = 0, n = 0;
  double cost = 0.0;
  phiq::setup_quadrature(eps, p, alpha, 1.0, PHIQ_RULE_CC, c1, c2, d, &lp, &n, &cost);
  if (lp < 0) return PHIQ_ERR_NOT_CONVERGED;
  *l = phiq::cc_scaling(eps, p, alpha, c1, c2, d, max_doublings, lp);
  return PHIQ_OK;
}

phiq_status phiq_log_quaderr(double n, int p, double alpha, double beta, phiq_rule rule,
                             double* log_err) {
  if (!log_err) return PHIQ_ERR_INVALID_ARG;
  if (!(alpha > 0) || !(beta > 0) || !(n >= 1) || p < 0 || p > PHIQ_MAX_P ||
      (rule != PHIQ_RULE_GAUSS && rule != PHIQ_RULE_CC))
    return PHIQ_ERR_INVALID_ARG;
  *log_err = phiq::log_quaderr(n, p, alpha, beta, rule);
  return PHIQ_OK;
}

phiq_status phiq_quadnodes(double eps, int p, double alpha, double beta, phiq_rule rule, int* n) {
  if (!n || !(eps > 0) || p < 1 || p > PHIQ_MAX_P || !(alpha > 0) || !(beta > 0)) return PHIQ_ERR_INVALID_ARG;
  if (!std::isfinite(eps) || !std::isfinite(alpha) || !std::isfinite(beta)) return PHIQ_ERR_NONFINITE;
  if (rule != PHIQ_RULE_GAUSS && rule != PHIQ_RULE_CC) return PHIQ_ERR_INVALID_ARG;
  *n = phiq::quadnodes(eps, p, alpha, beta, rule);
  return *n < 0 ? PHIQ_ERR_NOT_CONVERGED : PHIQ_OK;
}

phiq_status phiq_quadrature_rule(phiq_rule rule, int m, double* theta, double* w) {
  if (!theta || !w || m < 1 || m > 100000) return PHIQ_ERR_INVALID_ARG;
  if (rule == PHIQ_RULE_GAUSS) {
    phiq::gauss_legendre(m, theta, w);
  } else if (rule == PHIQ_RULE_CC) {
    if (m < 2) return PHIQ_ERR_INVALID_ARG;
    phiq::clenshaw_curtis(m, theta, w);
  } else {
    return PHIQ_ERR_INVALID_ARG;
  }
  return PHIQ_OK;
}

}  // extern "C"
