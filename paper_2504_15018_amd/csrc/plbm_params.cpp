// Host parameter layer of libplbm (float64): the multiphase unit converter
// and the derivation of the lattice constants from physical properties.
//
//   eqs. (unit), (unit2), Sec. V   C_L = L/L_lat, C_T = C_L^2 nu_l,lat/nu_l,
//                                  C_M = C_L^3 rho_l/rho_l,lat, C_U, C_VF, C_gamma
//   eq. (thickness), Sec. IV       K = p_c/rho_c^3 = (f_xi(rho_I1) - f_xi(rho_I2))^2 / (6 r xi^2)
//   eq. (surface_tension), Sec. IV kappa = sqrt(27/(2 r K)) gamma / (f_gamma(rho_v) - f_gamma(rho_l)),
//                                  f_gamma with rho_v, rho_l as in Appendix B
//   Sec. IV mechanical stability   int_{rho_v}^{rho_l} (p - p_0) psi'/psi^(1+eps) drho = 0
//
// For an equation of state other than the paper's (Peng-Robinson), the
// surface tension follows from the planar equilibrium of the pressure tensor
// eq. (New_Pressure_Tensor) at finite psi (G = -1, lattice units):
//   y(rho) = psi_x^2 = 8 psi^eps int_{rho_v}^{rho} (p - p_0) psi' psi^(-1-eps) drho,
//   gamma / kappa = (1/6) int sqrt(y) psi' drho.
// r = 1 in lattice units throughout.
#include <cmath>
#include <cstring>
#include <functional>
#include <vector>

#include "plbm_host.hpp"

namespace plbm {

namespace {

constexpr double kCs2 = 1.0 / 3.0;

struct Eos {
  int kind;  // EOS_PAPER | EOS_PR
  double K, rv, rl;                 // paper EOS
  double RT, b, aalpha;             // Peng-Robinson
  double p(double r) const {
    if (kind == EOS_PAPER) {
      double s = std::sqrt(r), sv = std::sqrt(rv);
      return K * (2 * r * r * r + (rv - 2 * rl) * r * r + sv * s * (-3 * r * r + 2 * rl * r + rl * rl));
    }
    return r * RT / (1 - b * r) - aalpha * r * r / (1 + 2 * b * r - b * b * r * r);
  }
  double dp(double r) const {
    if (kind == EOS_PAPER) {
      double s = std::sqrt(r), sv = std::sqrt(rv);
      return K * (6 * r * r + 2 * (rv - 2 * rl) * r + sv * (-7.5 * r * s + 3 * rl * s + 0.5 * rl * rl / s));
    }
    double d = 1 - b * r, q = 1 + 2 * b * r - b * b * r * r;
    return RT / (d * d) - aalpha * (2 * r * q - r * r * (2 * b - 2 * b * b * r)) / (q * q);
  }
  // psi^2 = 2 (rho/3 - p) and its derivative
  double R(double r) const { return 2 * (r / 3 - p(r)); }
  double dR(double r) const { return 2 * (1.0 / 3.0 - dp(r)); }
};

// Adaptive Gauss-Kronrod (7, 15) quadrature.
const double kXgk[8] = {0.991455371120812639206854697526329, 0.949107912342758524526189684047851,
                        0.864864423359769072789712788640926, 0.741531185599394439863864773280788,
                        0.586087235467691130294144845693013, 0.405845151377397166906606412076961,
                        0.207784955007898467600689403773245, 0.000000000000000000000000000000000};
const double kWgk[8] = {0.022935322010529224963732008058970, 0.063092092629978553290700663189204,
                        0.104790010322250183839876322541518, 0.140653259715525918745189590510238,
                        0.169004726639267902826583426598550, 0.190350578064785409913256402421014,
                        0.204432940075298892414161999234649, 0.209482141084727828012999174891714};
const double kWg[4] = {0.129484966168869693270611432679082, 0.279705391489276667901467771423780,
                       0.381830050505118944950369775488975, 0.417959183673469387755102040816327};

void gk15(const std::function<double(double)>& f, double a, double b, double* res, double* err) {
  double c = 0.5 * (a + b), h = 0.5 * (b - a);
  double fc = f(c);
  double rk = fc * kWgk[7], rg = fc * kWg[3];
  for (int j = 0; j < 7; ++j) {
    double x = h * kXgk[j];
    double f1 = f(c - x), f2 = f(c + x);
    rk += kWgk[j] * (f1 + f2);
    if (j & 1) rg += kWg[j / 2] * (f1 + f2);
  }
  *res = rk * h;
  *err = std::fabs((rk - rg) * h);
}

double integrate_rec(const std::function<double(double)>& f, double a, double b, double tol, int depth) {
  double r, e;
  gk15(f, a, b, &r, &e);
  if (e <= tol || depth >= 40) return r;
  double m = 0.5 * (a + b);
  return integrate_rec(f, a, m, 0.5 * tol, depth + 1) + integrate_rec(f, m, b, 0.5 * tol, depth + 1);
}

double integrate(const std::function<double(double)>& f, double a, double b, double abstol) {
  return integrate_rec(f, a, b, abstol, 0);
}

// Brent's root finder on a bracketing interval.
bool brent(const std::function<double(double)>& f, double a, double b, double tol, double* root) {
  double fa = f(a), fb = f(b);
  if (fa == 0) { *root = a; return true; }
  if (fb == 0) { *root = b; return true; }
  if ((fa > 0) == (fb > 0)) return false;
  double c = a, fc = fa, d = b - a, e = d;
  for (int it = 0; it < 300; ++it) {
    if ((fb > 0) == (fc > 0)) { c = a; fc = fa; d = b - a; e = d; }
    if (std::fabs(fc) < std::fabs(fb)) { a = b; b = c; c = a; fa = fb; fb = fc; fc = fa; }
    double tol1 = 2 * 2.2e-16 * std::fabs(b) + 0.5 * tol;
    double xm = 0.5 * (c - b);
    if (std::fabs(xm) <= tol1 || fb == 0) { *root = b; return true; }
    if (std::fabs(e) >= tol1 && std::fabs(fa) > std::fabs(fb)) {
      double s = fb / fa, pp, qq;
      if (a == c) {
        pp = 2 * xm * s; qq = 1 - s;
      } else {
        double q0 = fa / fc, r0 = fb / fc;
        pp = s * (2 * xm * q0 * (q0 - r0) - (b - a) * (r0 - 1));
        qq = (q0 - 1) * (r0 - 1) * (s - 1);
      }
      if (pp > 0) qq = -qq; else pp = -pp;
      if (2 * pp < std::fmin(3 * xm * qq - std::fabs(tol1 * qq), std::fabs(e * qq))) { e = d; d = pp / qq; }
      else { d = xm; e = d; }
    } else { d = xm; e = d; }
    a = b; fa = fb;
    b += std::fabs(d) > tol1 ? d : (xm > 0 ? tol1 : -tol1);
    fb = f(b);
  }
  *root = b;
  return true;
}

// Local maximum and minimum of p(rho) on (0, rho_hi): the van der Waals loop.
bool spinodals(const Eos& e, double rho_hi, double* rmax, double* rmin) {
  const int n = 100000;
  double prev = e.dp(rho_hi * 1e-7);
  int found = 0;
  double lo = rho_hi * 1e-7;
  for (int k = 1; k <= n; ++k) {
    double r = rho_hi * (double)k / n;
    double d = e.dp(r);
    if ((prev > 0) != (d > 0)) {
      double root;
      if (!brent([&](double x) { return e.dp(x); }, lo, r, 1e-15, &root)) return false;
      if (found == 0) *rmax = root; else { *rmin = root; return true; }
      ++found;
    }
    prev = d;
    lo = r;
  }
  return false;
}

struct Coex {
  double rv, rl, p0;
};

bool branch_roots(const Eos& e, double p0, double rmax, double rmin, double rho_hi, double* rv, double* rl) {
  auto g = [&](double r) { return e.p(r) - p0; };
  return brent(g, 0.0, rmax, 1e-16, rv) && brent(g, rmin, rho_hi, 1e-15, rl);
}

double stability(const Eos& e, double p0, double rv, double rl, double eps) {
  // (p - p0) psi' / psi^(1+eps) with psi' = R' / (2 psi):  (p - p0) R' / (2 R^(1 + eps/2))
  auto f = [&](double r) {
    double R = e.R(r);
    return (e.p(r) - p0) * e.dR(r) / (2.0 * std::pow(R, 1.0 + 0.5 * eps));
  };
  return integrate(f, rv, rl, 1e-15);
}

bool coexistence(const Eos& e, double eps, double rho_hi, Coex* out) {
  double rmax, rmin;
  if (!spinodals(e, rho_hi, &rmax, &rmin)) return false;
  double phi = e.p(rmax), plo = std::fmax(e.p(rmin), 0.0);
  std::function<double(double)> g = [&](double p0) -> double {
    double rv, rl;
    if (!branch_roots(e, p0, rmax, rmin, rho_hi, &rv, &rl)) return NAN;
    return stability(e, p0, rv, rl, eps);
  };
  // scan a geometric ladder of pressures downward from the top of the loop
  const int n = 32;
  double top = phi * (1 - 1e-9);
  double bot = std::fmax(plo, phi * 1e-8) * (1 + 1e-9);
  double pa = top, ga = g(pa);
  for (int k = 1; k <= n; ++k) {
    double pb = top * std::pow(bot / top, (double)k / n);
    double gb = g(pb);
    if (std::isfinite(ga) && std::isfinite(gb) && (ga > 0) != (gb > 0)) {
      double p0;
      if (!brent(g, pb, pa, 1e-17, &p0)) return false;
      double rv, rl;
      if (!branch_roots(e, p0, rmax, rmin, rho_hi, &rv, &rl)) return false;
      *out = {rv, rl, p0};
      return true;
    }
    pa = pb;
    ga = gb;
  }
  return false;
}

// gamma / kappa at finite psi (see the file header).
double gamma_over_kappa(const Eos& e, const Coex& c, double eps) {
  const int n = 20000;
  // cumulative inner integral on a uniform rho grid (composite trapezoid on a fine grid)
  std::vector<double> rho(n + 1), inner(n + 1, 0.0);
  auto h = [&](double r) {
    double R = e.R(r);
    return (e.p(r) - c.p0) * e.dR(r) / (2.0 * std::pow(R, 1.0 + 0.5 * eps));
  };
  for (int k = 0; k <= n; ++k) rho[k] = c.rv + (c.rl - c.rv) * k / n;
  for (int k = 1; k <= n; ++k) inner[k] = inner[k - 1] + integrate(h, rho[k - 1], rho[k], 1e-18);
  double acc = 0.0;
  for (int k = 1; k <= n; ++k) {
    // Simpson on each cell with the midpoint's inner integral from a half-cell integral
    double ra = rho[k - 1], rb = rho[k], rm = 0.5 * (ra + rb);
    double im = inner[k - 1] + integrate(h, ra, rm, 1e-18);
    auto outer = [&](double r, double in) {
      double R = e.R(r);
      double psi = std::sqrt(R > 0 ? R : 0);
      double y = 8.0 * std::pow(psi, eps) * in;
      return std::sqrt(y > 0 ? y : 0) * e.dR(r) / (2.0 * psi);
    };
    acc += (rb - ra) / 6.0 * (outer(ra, inner[k - 1]) + 4 * outer(rm, im) + outer(rb, inner[k]));
  }
  return acc / 6.0;
}

double f_xi(double r, double rv, double rl) {
  double s = std::sqrt(r), sv = std::sqrt(rv), sl = std::sqrt(rl);
  return std::log(s - sv) / (rl - rv) - std::log(sl - s) / (2 * sl * (sl - sv)) -
         std::log(s + sl) / (2 * sl * (sv + sl));
}

double f_gamma(double r, double rv, double rl) {
  double sv = std::sqrt(rv);
  return r * r / 4 - rl * r / 2 - sv * r * std::sqrt(r) / 3 + sv * rl * std::sqrt(r);
}

void pr_constants(double T_over_Tc, double omega, double* a, double* b, double* R, double* T, double* alpha) {
  *a = 2.0 / 49.0;
  *b = 2.0 / 21.0;
  *R = 1.0;
  double Tc = 0.0778 * (*a) / (0.45724 * (*b) * (*R));
  *T = T_over_Tc * Tc;
  double m = 0.37464 + 1.54226 * omega - 0.26992 * omega * omega;
  double q = 1 + m * (1 - std::sqrt(T_over_Tc));
  *alpha = q * q;
}

Eos eos_of(const plbm_lattice_params& p) {
  Eos e{};
  e.kind = p.eos;
  e.K = p.K;
  e.rv = p.eos_rho_v;
  e.rl = p.eos_rho_l;
  e.RT = p.pr_R * p.pr_T;
  e.b = p.pr_b;
  e.aalpha = p.pr_a * p.pr_alpha;
  return e;
}

double rho_hi_of(const plbm_lattice_params& p) { return p.eos == EOS_PAPER ? 3.0 * p.eos_rho_l : 0.999 / p.pr_b; }

void set_bf(plbm_lattice_params* o, const double* bf, double scale) {
  for (int a = 0; a < 3; ++a) o->body_force[a] = bf ? bf[a] / scale : 0.0;
}

}  // namespace

double params_K_from_width(double xi, double rv, double rl) {
  double r1 = rv + 0.33 * (rl - rv), r2 = rv + 0.67 * (rl - rv);
  double d = f_xi(r1, rv, rl) - f_xi(r2, rv, rl);
  return d * d / (6.0 * xi * xi);
}

double params_kappa_from_gamma(double gamma, double K, double rv, double rl) {
  return std::sqrt(27.0 / (2.0 * K)) * gamma / (f_gamma(rv, rv, rl) - f_gamma(rl, rv, rl));
}

int params_paper_lattice(double rv, double rl, double xi, double eps, double kappa, double tau_v, double tau_l,
                         const double* bf, plbm_lattice_params* o) {
  if (!(rv > 0) || !(rl > rv) || !(xi > 0) || !(tau_v > 0.5) || !(tau_l > 0.5))
    return set_error(PLBM_E_INVALID, "paper EOS: need 0 < rho_v < rho_l, xi > 0, tau > 1/2");
  std::memset(o, 0, sizeof(*o));
  o->eos = EOS_PAPER;
  o->K = params_K_from_width(xi, rv, rl);
  o->eos_rho_v = rv;
  o->eos_rho_l = rl;
  o->epsilon = eps > 0 ? eps : 2.0;
  o->kappa = kappa;
  o->G = -1.0;
  o->tau_v = tau_v;
  o->tau_l = tau_l;
  set_bf(o, bf, 1.0);
  Coex c;
  if (!coexistence(eos_of(*o), o->epsilon, rho_hi_of(*o), &c))
    return set_error(PLBM_E_NOCONVERGE, "paper EOS: mechanical-stability coexistence not found");
  o->rho_v = c.rv;
  o->rho_l = c.rl;
  return PLBM_OK;
}

int params_pr_lattice(double T_over_Tc, double omega, double eps, double kappa, double tau_v, double tau_l,
                      const double* bf, plbm_lattice_params* o) {
  if (!(T_over_Tc > 0 && T_over_Tc < 1) || !(tau_v > 0.5) || !(tau_l > 0.5))
    return set_error(PLBM_E_INVALID, "Peng-Robinson: need 0 < T/Tc < 1 and tau > 1/2");
  std::memset(o, 0, sizeof(*o));
  o->eos = EOS_PR;
  pr_constants(T_over_Tc, omega, &o->pr_a, &o->pr_b, &o->pr_R, &o->pr_T, &o->pr_alpha);
  o->epsilon = eps > 0 ? eps : 2.0;
  o->kappa = kappa;
  o->G = -1.0;
  o->tau_v = tau_v;
  o->tau_l = tau_l;
  set_bf(o, bf, 1.0);
  Coex c;
  if (!coexistence(eos_of(*o), o->epsilon, rho_hi_of(*o), &c))
    return set_error(PLBM_E_NOCONVERGE, "Peng-Robinson: mechanical-stability coexistence not found");
  o->rho_v = c.rv;
  o->rho_l = c.rl;
  return PLBM_OK;
}

int params_resolve(const plbm_phys_params* ph, const plbm_lattice_map* mp, plbm_lattice_params* o) {
  if (!ph || !mp || !o) return set_error(PLBM_E_INVALID, "null argument");
  if (!(ph->L > 0) || !(mp->L_lat > 0) || !(mp->tau_l > 0.5) || !(ph->nu_l > 0) || !(ph->nu_v > 0) ||
      !(ph->rho_l > 0) || !(ph->rho_v > 0) || !(ph->rho_v < ph->rho_l))
    return set_error(PLBM_E_INVALID, "need L, L_lat, nu_v, nu_l > 0, 0 < rho_v < rho_l, tau_l > 1/2");
  const double rho_l_lat_in = mp->rho_l_lat > 0 ? mp->rho_l_lat : 1.187;
  const double eps = ph->epsilon > 0 ? ph->epsilon : 2.0;
  const double C_L = ph->L / mp->L_lat;
  const double nu_l_lat = kCs2 * (mp->tau_l - 0.5);
  const double C_T = C_L * C_L * nu_l_lat / ph->nu_l;
  const double nu_v_lat = ph->nu_v * C_T / (C_L * C_L);
  const double tau_v = nu_v_lat / kCs2 + 0.5;
  int st;
  double rho_l_lat = rho_l_lat_in;
  double C_M = C_L * C_L * C_L * ph->rho_l / rho_l_lat;
  double C_VF = C_M / (C_L * C_L * C_T * C_T);
  double bf[3];
  for (int a = 0; a < 3; ++a) bf[a] = ph->body_force[a] / C_VF;
  if (ph->eos == EOS_PAPER) {
    if (!(ph->xi > 0)) return set_error(PLBM_E_INVALID, "paper EOS: need xi > 0");
    const double C_rho = C_M / (C_L * C_L * C_L);
    const double rv = ph->rho_v / C_rho, rl = ph->rho_l / C_rho;
    st = params_paper_lattice(rv, rl, ph->xi / C_L, eps, 1.0, tau_v, mp->tau_l, bf, o);
    if (st) return st;
    const double C_gamma = C_M / (C_T * C_T);
    if (ph->gamma > 0) {
      o->gamma_lat = ph->gamma / C_gamma;
      o->kappa = params_kappa_from_gamma(o->gamma_lat, o->K, rv, rl);
    }
  } else if (ph->eos == EOS_PR) {
    st = params_pr_lattice(ph->T_over_Tc, ph->omega, eps, 1.0, tau_v, mp->tau_l, bf, o);
    if (st) return st;
    if (mp->rho_l_lat <= 0) {
      // the lattice liquid density is the EOS's own coexistence liquid density
      rho_l_lat = o->rho_l;
      C_M = C_L * C_L * C_L * ph->rho_l / rho_l_lat;
      C_VF = C_M / (C_L * C_L * C_T * C_T);
      for (int a = 0; a < 3; ++a) o->body_force[a] = ph->body_force[a] / C_VF;
    }
    const double C_gamma = C_M / (C_T * C_T);
    if (ph->gamma > 0) {
      o->gamma_lat = ph->gamma / C_gamma;
      Coex c{o->rho_v, o->rho_l, eos_of(*o).p(o->rho_v)};
      o->kappa = o->gamma_lat / gamma_over_kappa(eos_of(*o), c, eps);
    }
  } else {
    return set_error(PLBM_E_INVALID, "unknown EOS");
  }
  o->C_L = C_L;
  o->C_T = C_T;
  o->C_M = C_M;
  o->C_U = C_L / C_T;
  o->C_VF = C_M / (C_L * C_L * C_T * C_T);
  o->C_gamma = C_M / (C_T * C_T);
  o->C_p = C_M / (C_L * C_T * C_T);
  o->Re = ph->U_phys > 0 ? ph->U_phys * ph->L / ph->nu_l : 0.0;
  return PLBM_OK;
}

double params_gamma_over_kappa(const plbm_lattice_params* p) {
  Eos e = eos_of(*p);
  Coex c{p->rho_v, p->rho_l, e.p(p->rho_v)};
  return gamma_over_kappa(e, c, p->epsilon);
}

}  // namespace plbm
