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

// ------------------------------------------------------------------ model scalars
StepScalars step_scalars(const cola_params& p, double a) {
  StepScalars s{};
  const double om = p.omega_m, ol = 1.0 - om;
  const double E = std::sqrt(om / (a * a * a) + ol);
  s.a = a;
  s.kappa = (float)(1.5 * om * a);
  s.fifth = (p.model == COLA_FR_HS1 || p.model == COLA_NDGP || p.model == COLA_SYMMETRON) ? 1 : 0;
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
  s.potential = (p.model == COLA_FR_HS1 || p.model == COLA_SYMMETRON) ? 1 : 0;
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

StepDev step_dev(const cola_params& p, const Layout& L, int i) {
  const Cosmo cz{p.omega_m, 1.0 - p.omega_m};
  const double ai = a_of_step(p, i), an = a_of_step(p, i + 1);
  const double a_lo = (i == 0) ? ai : 0.5 * (a_of_step(p, i - 1) + ai);
  const double a_hi = 0.5 * (ai + an);
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
  d.dtk = (float)tau_between(cz, a_lo, a_hi);
  d.dtd = (float)tau_between(cz, ai, an);
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
  if (p.model < 0 || p.model > 3) bad("model must be 0 (LCDM), 1 (f(R)), 2 (nDGP) or 3 (symmetron)");
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
  L.kdep = ((p.model == COLA_FR_HS1 || p.model == COLA_SYMMETRON) && p.growth_mode == 0);
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
  for (int i = 0; i < 6; ++i) {
    L.off_pfield[i] = o;
    if (L.kdep) o += pfield_bytes;
  }
  L.tile = (L.nm % 16 == 0 && L.nm / 16 >= 2) ? 16 : (L.nm % 8 == 0 && L.nm / 8 >= 2) ? 8 : 4;
  L.nt1 = L.nm / L.tile;
  L.ntiles = (int64_t)L.nt1 * L.nt1 * L.nt1;
  L.off_bins = o;
  o += bins_bytes(L.ntiles);
  const size_t entries_bytes = align_up((size_t)L.N * sizeof(float4));
  if (entries_bytes <= mesh_bytes) {
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
