// Host-side double-precision physics and buffer layout of libcola.
//
// * background: flat LCDM, E(a) = sqrt(Om a^-3 + 1 - Om), d tau = da/(a^3 E) (Sec. 2);
// * time grid: a_i uniform in a from a_ini to 1; kick/drift intervals in tau by
//   Gauss-Legendre quadrature;
// * initial spectrum: Eisenstein & Hu (1998) no-wiggle transfer function, normalised to
//   sigma8 by Gauss-Legendre quadrature in ln k over 1e-5 < k < 1e2 h/Mpc;
// * PM-force scalars of the models at a given a (Secs. 5-6).

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "internal.h"

namespace cola {

static constexpr double kH0c = 1.0 / 2997.92458;

// ------------------------------------------------------------------ Gauss-Legendre
// Nodes/weights on [-1, 1] by Newton iteration on P_n (Golub-Welsch is not needed at n = 16).
struct GL {
  std::vector<double> x, w;
  explicit GL(int n) : x(n), w(n) {
    for (int i = 0; i < n; ++i) {
      double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
      for (int it = 0; it < 100; ++it) {
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
          const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        const double dp = n * (z * p1 - p0) / (z * z - 1.0);
        const double dz = p1 / dp;
        z -= dz;
        if (std::fabs(dz) < 1e-16) break;
      }
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      const double dp = n * (z * p1 - p0) / (z * z - 1.0);
      x[i] = z;
      w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
  }
};

static const GL& gl16() {
  static GL g(16);
  return g;
}

template <class F>
static double integrate(F f, double lo, double hi, int panels) {
  const GL& g = gl16();
  double tot = 0.0;
  const double h = (hi - lo) / panels;
  for (int p = 0; p < panels; ++p) {
    const double a = lo + p * h, m = a + 0.5 * h;
    double s = 0.0;
    for (size_t i = 0; i < g.x.size(); ++i) s += g.w[i] * f(m + 0.5 * h * g.x[i]);
    tot += 0.5 * h * s;
  }
  return tot;
}

// ------------------------------------------------------------------ background
double Cosmo::E(double a) const { return std::sqrt(om / (a * a * a) + ol); }

double tau_between(const Cosmo& c, double a0, double a1) {
  if (a1 == a0) return 0.0;
  // d tau = d ln a / (a^2 E)
  return integrate([&](double lna) {
    const double a = std::exp(lna);
    return 1.0 / (a * a * c.E(a));
  }, std::log(a0), std::log(a1), 16);
}

double a_of_step(const cola_params& p, int i) {
  const double ai = 1.0 / (1.0 + p.z_init);
  return ai + i * (1.0 - ai) / p.n_steps;
}

// ------------------------------------------------------------------ initial spectrum
double eh_transfer(const cola_params& p, double k) {
  const double theta = p.t_cmb / 2.7;
  const double omh2 = p.omega_m * p.h * p.h, obh2 = p.omega_b * p.h * p.h;
  const double fb = p.omega_b / p.omega_m;
  const double s = 44.5 * std::log(9.83 / omh2) / std::sqrt(1.0 + 10.0 * std::pow(obh2, 0.75));
  const double alpha = 1.0 - 0.328 * std::log(431.0 * omh2) * fb + 0.38 * std::log(22.3 * omh2) * fb * fb;
  const double ks = 0.43 * k * p.h * s;
  const double gam = p.omega_m * p.h * (alpha + (1.0 - alpha) / (1.0 + ks * ks * ks * ks));
  const double q = k * theta * theta / gam;
  const double L0 = std::log(2.0 * M_E + 1.8 * q);
  const double C0 = 14.2 + 731.0 / (1.0 + 62.5 * q);
  return L0 / (L0 + C0 * q * q);
}

double sigma8_norm(const cola_params& p) {
  auto f = [&](double lnk) {
    const double k = std::exp(lnk);
    const double x = 8.0 * k;
    const double W = x > 1e-4 ? 3.0 * (std::sin(x) - x * std::cos(x)) / (x * x * x) : 1.0 - x * x / 10.0;
    const double T = eh_transfer(p, k);
    return k * k * k * std::pow(k, p.n_s) * T * T * W * W / (2.0 * M_PI * M_PI);
  };
  const double I = integrate(f, std::log(1e-5), std::log(1e2), 4000);
  return p.sigma8 * p.sigma8 / I;
}

// ------------------------------------------------------------------ general {m, beta} tables
// Natural cubic spline through (x_i, y_i): second derivatives M with M_0 = M_{n-1} = 0 from
// the tridiagonal continuity equations, by the Thomas algorithm.
static void natural_spline(int n, const double* x, const double* y, double* M) {
  std::vector<double> c(n, 0.0), d(n, 0.0);
  M[0] = M[n - 1] = 0.0;
  for (int i = 1; i < n - 1; ++i) {
    const double h0 = x[i] - x[i - 1], h1 = x[i + 1] - x[i];
    const double a = h0, b = 2.0 * (h0 + h1), cc = h1;
    const double r = 6.0 * ((y[i + 1] - y[i]) / h1 - (y[i] - y[i - 1]) / h0);
    const double den = b - a * (i > 1 ? c[i - 1] : 0.0);
    c[i] = cc / den;
    d[i] = (r - a * (i > 1 ? d[i - 1] : 0.0)) / den;
  }
  for (int i = n - 2; i >= 1; --i) M[i] = d[i] - c[i] * (i + 1 < n - 1 ? M[i + 1] : 0.0);
}

MBSpline mb_spline(const cola_params& p) {
  MBSpline s{};
  if (p.model != COLA_MBETA) return s;
  s.n = p.mb_n;
  for (int i = 0; i < s.n; ++i) {
    s.x[i] = p.mb_lna[i];
    s.yb[i] = p.mb_beta[i];
    s.ym[i] = std::log(p.mb_m2[i]);
  }
  natural_spline(s.n, s.x, s.yb, s.Mb);
  natural_spline(s.n, s.x, s.ym, s.Mm);
  return s;
}

// Phi_crit(a) of App. C, (9 Om / (2 beta(a))) int_{a_0}^{a} beta / ((m^2/H0^2) a'^4) da',
// by Gauss-Legendre panels of width <= 0.01 in ln a' (the integrand there is
// beta / ((m^2/H0^2) a'^3))
static double mb_phi_crit(const cola_params& p, const MBSpline& s, double a) {
  const double l0 = s.x[0], l1 = std::log(a);
  if (!(l1 > l0)) return 0.0;
  const int panels = std::max(1, (int)std::ceil((l1 - l0) / 0.01));
  const double I = integrate([&](double lna) {
    const double x = std::exp(lna);
    double b, m2, dm2;
    mb_eval(s, x, b, m2, dm2);
    return b / (m2 * x * x * x);
  }, l0, l1, panels);
  double b, m2, dm2;
  mb_eval(s, a, b, m2, dm2);
  return 4.5 * p.omega_m / b * I;
}

// ------------------------------------------------------------------ model scalars
StepScalars step_scalars(const cola_params& p, double a) {
  StepScalars s{};
  const double om = p.omega_m, ol = 1.0 - om;
  const double E = std::sqrt(om / (a * a * a) + ol);
  s.a = a;
  s.kappa = (float)(1.5 * om * a);
  s.fifth = (p.model == COLA_FR_HS1 || p.model == COLA_NDGP || p.model == COLA_SYMMETRON ||
             p.model == COLA_MBETA || p.model == COLA_KMOUFLAGE) ? 1 : 0;
  s.screen = s.fifth && p.screening;
  if (p.model == COLA_FR_HS1) {
    const double X = om / (a * a * a) + 4.0 * ol, Y = om + 4.0 * ol;
    const double r = X / Y;
    s.a2m2 = (float)(a * a * kH0c * kH0c * Y * r * r * r / (2.0 * p.fr0_abs));
    s.coupling = (float)(1.0 / 3.0);
    const double fR = p.fr0_abs * (Y / X) * (Y / X);
    s.cham_thr = (float)(1.5 * fR * a * a / (kH0c * kH0c));
  } else if (p.model == COLA_SYMMETRON) {
    // App. C: C = 2 beta^2, a^2 m^2, and the potential threshold Phi_crit a^2/(H0/c)^2 on
    // the code potential; before a_* the coupling is zero and the force Newtonian
    const double as = p.sym_astar / a;
    const double sv = a > p.sym_astar ? 1.0 - as * as * as : 0.0;
    s.a2m2 = (float)(a * a * kH0c * kH0c * p.sym_mass * p.sym_mass * sv);
    s.coupling = (float)(2.0 * p.sym_beta * p.sym_beta * sv);
    const double phi_crit = 3.0 * om / (p.sym_astar * p.sym_astar * p.sym_astar * p.sym_mass * p.sym_mass);
    s.cham_thr = (float)(phi_crit * a * a / (kH0c * kH0c));
  } else if (p.model == COLA_MBETA) {
    // App. C: C = 2 beta^2, a^2 m^2, and the threshold Phi_crit a^2/(H0/c)^2 on the code
    // potential with Phi_crit from the App. C integral
    const MBSpline sp = mb_spline(p);
    double b, m2, dm2;
    mb_eval(sp, a, b, m2, dm2);
    s.a2m2 = (float)(a * a * kH0c * kH0c * m2);
    s.coupling = (float)(2.0 * b * b);
    s.cham_thr = (float)(mb_phi_crit(p, sp, a) * a * a / (kH0c * kH0c));
  } else if (p.model == COLA_KMOUFLAGE) {   // App. B: massless, C = 2 beta^2
    s.coupling = (float)(2.0 * p.km_beta * p.km_beta);
  } else if (p.model == COLA_NDGP) {
    const double oma = om / (a * a * a) / (E * E);
    const double beta = 1.0 + 2.0 * p.rc_h0 * E * (1.0 - 0.5 * oma);
    s.beta = (float)beta;
    s.coupling = (float)(1.0 / (3.0 * beta));
    const double a3 = (p.readings & COLA_READ_X_NO_A3) ? 1.0 : a * a * a;
    s.vx_pref = (float)(8.0 * p.rc_h0 * p.rc_h0 * om / (9.0 * beta * beta * a3));
    s.vx_off = (p.readings & COLA_READ_X_TOTAL_DENSITY) ? s.vx_pref : 0.f;
  }
  return s;
}

PMScalars pm_scalars(const cola_params& p, double a) {
  const StepScalars sc = step_scalars(p, a);
  PMScalars s{};
  s.g_n = -sc.kappa;
  s.g_5 = sc.fifth ? -sc.coupling * sc.kappa : 0.f;
  s.a2m2 = sc.a2m2;
  s.sop_g_n = 0.f;
  s.thr = sc.cham_thr;
  s.vx = sc.vx_pref;
  s.vx0 = sc.vx_off;
  s.cn = 0.f;
  s.c5 = 1.f;
  s.screen = sc.screen;
  s.potential = (p.model == COLA_FR_HS1 || p.model == COLA_SYMMETRON || p.model == COLA_MBETA) ? 1 : 0;
  s.gradient = p.model == COLA_KMOUFLAGE ? 1 : 0;
  {
    const double f = p.km_lambda * kH0c * kH0c / (a * a);
    s.km_r = s.gradient ? (float)(f * f) : 0.f;
  }
  if (s.screen) {
    if (s.potential) {
      s.sop_g_n = -sc.kappa;
    } else {   // one source: (rho - 1)(g_n + g_5 eps) over k^2
      s.cn = s.g_n;
      s.c5 = s.g_5;
      s.g_n = 1.f;
      s.g_5 = 0.f;
      s.a2m2 = 0.f;
    }
  }
  return s;
}

void step_times(const cola_params& p, int i, double out[4]) {
  const Cosmo cz{p.omega_m, 1.0 - p.omega_m};
  const double ai = a_of_step(p, i), an = a_of_step(p, i + 1);
  const double a_lo = (i == 0) ? ai : 0.5 * (a_of_step(p, i - 1) + ai);
  const double a_hi = 0.5 * (ai + an);
  out[0] = ai;
  out[1] = an;
  out[2] = tau_between(cz, a_lo, a_hi);
  out[3] = tau_between(cz, ai, an);
}

StepDev step_dev(const cola_params& p, const Layout& L, int i) {
  double tm[4];
  step_times(p, i, tm);
  const double ai = tm[0];
  const PMScalars m = pm_scalars(p, ai);
  StepDev d{};
  d.g_n = m.g_n;
  d.g_5 = m.g_5;
  d.a2m2 = m.a2m2;
  d.sop_g_n = m.sop_g_n;
  d.thr = m.thr;
  d.vx = m.vx;
  d.vx0 = m.vx0;
  d.cn = m.cn;
  d.c5 = m.c5;
  d.km_r = m.km_r;
  d.dtk = (float)tm[2];
  d.dtd = (float)tm[3];
  d.slice0 = (int64_t)i * L.n_k * 6;
  d.slice1 = (int64_t)(i + 1) * L.n_k * 6;
  return d;
}

// ------------------------------------------------------------------ validation / layout
static bool is_2a3b(int n) {
  if (n < 2 || n % 2) return false;
  while (n % 2 == 0) n /= 2;
  if (n % 3 == 0) n /= 3;
  return n == 1;
}

void validate(const cola_params& p) {
  auto bad = [](const char* m) { throw Error{COLA_E_ARG, m}; };
  if (!(p.omega_m > 0 && p.omega_m <= 1)) bad("omega_m must be in (0, 1]");
  if (!(p.omega_b >= 0 && p.omega_b < p.omega_m)) bad("omega_b must be in [0, omega_m)");
  if (!(p.h > 0) || !(p.sigma8 > 0) || !(p.t_cmb > 0)) bad("h, sigma8 and t_cmb must be > 0");
  if (!std::isfinite(p.n_s)) bad("n_s must be finite");
  if (p.model < 0 || p.model > 5)
    bad("model must be 0 (LCDM), 1 (f(R)), 2 (nDGP), 3 (symmetron), 4 (tabulated {m, beta}) or "
        "5 (k-Mouflage)");
  if (p.model == COLA_KMOUFLAGE &&
      !(p.km_beta >= 0 && p.km_k0 > 0 && p.km_m >= 2 && p.km_m <= 8 && p.km_lambda >= 0 &&
        p.km_x0 >= 0 && std::isfinite(p.km_xn) && std::isfinite(p.km_beta) &&
        std::isfinite(p.km_k0) && std::isfinite(p.km_lambda) && std::isfinite(p.km_x0)))
    bad("k-Mouflage needs km_beta >= 0, km_k0 > 0, 2 <= km_m <= 8, km_lambda >= 0, km_x0 >= 0");
  if (p.model == COLA_MBETA) {
    if (p.mb_n < 4 || p.mb_n > COLA_MBETA_MAX_KNOTS) bad("mb_n must be in [4, COLA_MBETA_MAX_KNOTS]");
    for (int i = 0; i < p.mb_n; ++i) {
      if (!std::isfinite(p.mb_lna[i]) || !std::isfinite(p.mb_beta[i]) || !std::isfinite(p.mb_m2[i]))
        bad("mb tables must be finite");
      if (i > 0 && !(p.mb_lna[i] > p.mb_lna[i - 1])) bad("mb_lna must be strictly ascending");
      if (!(p.mb_beta[i] >= 0) || !(p.mb_m2[i] > 0)) bad("mb_beta must be >= 0 and mb_m2 > 0");
    }
    if (!(p.mb_lna[0] <= -std::log1p(p.z_init) + 1e-12) || !(p.mb_lna[p.mb_n - 1] >= 0))
      bad("mb_lna must span [ln a_ini, 0]");
  }
  if (p.model == COLA_SYMMETRON &&
      !(p.sym_beta >= 0 && p.sym_mass > 0 && p.sym_astar > 0 && p.sym_astar < 1))
    bad("symmetron needs sym_beta >= 0, sym_mass > 0, 0 < sym_astar < 1");
  if (p.model == COLA_FR_HS1 && !(p.fr0_abs > 0)) bad("fr0_abs must be > 0 for f(R)");
  if (p.model == COLA_NDGP && !(p.rc_h0 > 0)) bad("rc_h0 must be > 0 for nDGP");
  if (p.screening < 0 || p.screening > 1) bad("screening must be 0 or 1");
  if (p.filter < 0 || p.filter > 2) bad("filter must be 0, 1 or 2");
  if (!(p.r_smooth >= 0)) bad("r_smooth must be >= 0");
  if (p.growth_mode < 0 || p.growth_mode > 1) bad("growth_mode must be 0 or 1");
  if (!is_2a3b(p.np1d) || !is_2a3b(p.nmesh1d)) bad("np1d and nmesh1d must be of the form 2^a 3^b, b <= 1");
  if (p.np1d < 8 || p.np1d > 1024) bad("np1d must be in [8, 1024]");
  if (p.nmesh1d < p.np1d || p.nmesh1d > 2048) bad("nmesh1d must be in [np1d, 2048]");
  if (p.nmesh1d % p.np1d) bad("nmesh1d must be a multiple of np1d");
  if (p.nmesh1d > 4 * p.np1d) bad("nmesh1d must be at most 4 np1d");
  if (!fft_size_supported(p.np1d) || !fft_size_supported(p.nmesh1d)) bad("FFT size not supported");
  if (!(p.box > 0) || !(p.z_init > 0)) bad("box and z_init must be > 0");
  if (p.n_steps < 1 || p.n_steps > 4096) bad("n_steps must be in [1, 4096]");
  if (p.readings & ~COLA_READ_ALL) bad("readings has unknown bits");
}

Layout make_layout(const cola_params& p) {
  validate(p);
  Layout L{};
  L.np = p.np1d;
  L.nm = p.nmesh1d;
  L.box = p.box;
  L.inv_cell = (float)(p.nmesh1d / p.box);
  L.N = (int64_t)L.np * L.np * L.np;
  L.M = (int64_t)L.nm * L.nm * L.nm;
  L.pitch_p = half_pitch(L.np);
  L.pitch_m = half_pitch(L.nm);
  L.plane_p = plane_stride(L.np);
  L.plane_m = plane_stride(L.nm);
  L.pgrid_elems = (size_t)L.np * L.plane_p;
  L.mesh_elems = (size_t)L.nm * L.plane_m;
  L.kdep = ((p.model == COLA_FR_HS1 || p.model == COLA_SYMMETRON || p.model == COLA_MBETA) &&
            p.growth_mode == 0);
  L.n_k = L.kdep ? 3 * (int64_t)(L.np / 2) * (L.np / 2) + 1 : 1;
  L.n_steps = p.n_steps;
  size_t o = 0;
  L.off_growth = o;
  o = align_up(o + (size_t)(p.n_steps + 1) * L.n_k * 6 * sizeof(double));
  L.off_ref = o;
  o = align_up(o + 6 * sizeof(double));
  L.off_tw_m = o;
  o = align_up(o + (size_t)L.nm * sizeof(float2));
  L.off_tw_p = o;
  o = align_up(o + (size_t)L.np * sizeof(float2));
  L.off_scratch = o;
  L.scratch_bytes = pk_scratch_bytes(L, 2048) + align_up(2048 * (sizeof(float4) + 8));
  o = align_up(o + L.scratch_bytes);
  L.off_lpt_coef = o;
  o = align_up(o + (L.kdep ? 2 * (size_t)L.n_k * sizeof(float2) : 0));
  L.off_steps = o;
  o = align_up(o + (size_t)p.n_steps * sizeof(StepDev));
  L.off_ctr = o;
  o = align_up(o + sizeof(int));
  L.tables_bytes = o;
  const size_t mesh_bytes = align_up(L.mesh_elems * sizeof(float2));
  const size_t pfield_bytes = align_up(L.pgrid_elems * sizeof(float2));
  o = 0;
  for (int i = 0; i < 6; ++i) {
    L.off_mesh[i] = o;
    o += mesh_bytes;
  }
  {
    const size_t l3 = align_up((size_t)3 * L.N * sizeof(float));
    const size_t need = 3 * pfield_bytes + 2 * l3;
    size_t q = 0;
    if (L.kdep) {
      if (need <= 3 * mesh_bytes) {
        q = L.off_mesh[0];
      } else {
        q = o;
        o += need;
      }
    }
    for (int i = 0; i < 3; ++i) L.off_lptw[i] = q + i * pfield_bytes;
    L.off_lpp3 = q + 3 * pfield_bytes;
    L.off_dlt3 = L.off_lpp3 + l3;
  }
  L.tile = (L.nm % 16 == 0 && L.nm / 16 >= 2) ? 16 : (L.nm % 8 == 0 && L.nm / 8 >= 2) ? 8 : 4;
  L.nt1 = L.nm / L.tile;
  L.ntiles = (int64_t)L.nt1 * L.nt1 * L.nt1;
  L.off_bins = o;
  o += bins_bytes(L.ntiles);
  const size_t entries_bytes = align_up((size_t)L.N * 12);   // one 12-byte CIC record per particle
  // k-Mouflage deposits a second time while the Newtonian force mesh (over slots 3-5) is
  // still needed, so its records get their own area
  if (entries_bytes <= mesh_bytes && p.model != COLA_KMOUFLAGE) {
    L.off_entries = L.off_mesh[5];   // dead before the force mesh is written
  } else {
    L.off_entries = o;
    o += entries_bytes;
  }
  L.work_bytes = o;
  L.disp_bytes = align_up((size_t)3 * L.N * sizeof(float));
  L.lpt_bytes = L.kdep ? 2 * pfield_bytes : 2 * L.disp_bytes;
  return L;
}

}  // namespace cola
