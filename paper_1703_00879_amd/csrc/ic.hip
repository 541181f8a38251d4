// Growth factors (FP64) and the Gaussian initial conditions.
//
// Growth (Secs. 3.1, 4.1, 4.2, App. B): per Fourier mode,
//   D1'' = kappa mu(k,a) D1,
//   D2'' = kappa mu D2 - kappa mu D1^2 [1 + 2 a^4 H^2 gamma_2(k, k/sqrt2, k/sqrt2, a)/(kappa mu)],
// primes d/dtau, kappa = 1.5 Omega_m a, with the Einstein-de Sitter growing-mode values at
// a_ini (D1 = 1, D1' = a^2 E, D2 = -3/7, D2' = -(6/7) a^2 E).  One thread integrates one
// integer |nu|^2 of the particle grid (k = 2 pi |nu| / L) with classical fourth-order
// Runge-Kutta in ln a (steps <= 1e-3), stopping exactly on every a_i of the time grid.
// This is the only double-precision arithmetic on the device.
//
// Initial field: counter-based SplitMix64 white noise (Steele, Lea & Flood 2014) with a
// Box-Muller transform, scaled in Fourier space by sqrt(N P_ini(k) / L^3), where P_ini is
// the Eisenstein-Hu no-wiggle spectrum normalised to sigma8 at z = 0 and divided by the
// square of the LCDM growth factor D1(a = 1) of the same ODE.

#include <algorithm>
#include <cmath>

#include "internal.h"

namespace cola {

constexpr double kH0c = 1.0 / 2997.92458;   // H0/c in h/Mpc

struct GrowthDev {
  double om, fr0, rc, a_ini, kf;
  double sb, sm, sa;  // symmetron beta_*, m_*/H0, a_*
  double kb, kk0, kx0, kxn;   // k-Mouflage beta, K0, X(a) = kx0 a^kxn
  int km;                     // k-Mouflage exponent m
  int model;          // effective model for the growth (LCDM when growth_mode = 1)
  int kdep;           // table indexed by |nu|^2
  int n_steps;
  int64_t n_k;
};

__device__ __forceinline__ double dE(double a, double om) { return sqrt(om / (a * a * a) + 1.0 - om); }

// One classical fourth-order Runge-Kutta step of length h in ln a.
template <int NV, class Rhs>
__device__ __forceinline__ void rk4_step(double* y, double lna, double h, const Rhs& rhs) {
  double k1[NV], k2[NV], k3[NV], k4[NV], yt[NV];
  rhs(lna, y, k1);
  for (int c = 0; c < NV; ++c) yt[c] = y[c] + 0.5 * h * k1[c];
  rhs(lna + 0.5 * h, yt, k2);
  for (int c = 0; c < NV; ++c) yt[c] = y[c] + 0.5 * h * k2[c];
  rhs(lna + 0.5 * h, yt, k3);
  for (int c = 0; c < NV; ++c) yt[c] = y[c] + h * k3[c];
  rhs(lna + h, yt, k4);
  for (int c = 0; c < NV; ++c) y[c] += h / 6.0 * (k1[c] + 2.0 * k2[c] + 2.0 * k3[c] + k4[c]);
}

// RK4 in ln a from lna to le in equal steps <= 1e-3.
template <int NV, class Rhs>
__device__ __forceinline__ void rk4_segment(double* y, double& lna, double le, const Rhs& rhs) {
  const int nsub = (int)ceil((le - lna) / 1e-3);
  if (nsub <= 0) return;
  const double h = (le - lna) / nsub;
  for (int s = 0; s < nsub; ++s) {
    rk4_step<NV>(y, lna, h, rhs);
    lna = (s + 1 == nsub) ? le : lna + h;
  }
}

// RK4 from lna to l1 for a right-hand side that switches on at l_kink (the symmetron at
// a_*; -1e300 for the other models).  A step boundary falls exactly on l_kink.  Just after
// it the symmetron's gamma_2 term has a peak whose width in ln a scales as
// (k / (a_* m_*))^2, far below 1e-3 for the fundamental mode of a large box; the steps
// there start at 1e-10 and grow geometrically (h = 1e-10 + 0.02 (ln a - l_kink)) until
// they reach the 1e-3 of the rest of the integration.
template <int NV, class Rhs>
__device__ __forceinline__ void rk4_to(double* y, double& lna, double l1, double l_kink, const Rhs& rhs) {
  if (lna < l_kink && l_kink < l1) rk4_segment<NV>(y, lna, l_kink, rhs);
  if (lna >= l_kink) {
    while (lna < l1) {
      const double h = 1e-10 + 0.02 * (lna - l_kink);
      if (h >= 1e-3) break;
      if (h >= l1 - lna) {
        rk4_step<NV>(y, lna, l1 - lna, rhs);
        lna = l1;
      } else {
        rk4_step<NV>(y, lna, h, rhs);
        lna += h;
      }
    }
  }
  rk4_segment<NV>(y, lna, l1, rhs);
}

// RK4 from lna to l1 (as rk4_to) with a step boundary on every knot of a tabulated
// {m, beta} model in between: the splines' third derivatives jump there, which a step
// across a knot would integrate at lower order.
template <int NV, class Rhs>
__device__ __forceinline__ void rk4_to_knots(double* y, double& lna, double l1, double l_kink,
                                             const GrowthDev& g, const MBSpline& mb, const Rhs& rhs) {
  if (g.model == COLA_MBETA) {
    for (int j = 0; j < mb.n; ++j)
      if (mb.x[j] > lna && mb.x[j] < l1) rk4_to<NV>(y, lna, mb.x[j], l_kink, rhs);
  }
  rk4_to<NV>(y, lna, l1, l_kink, rhs);
}

__device__ __forceinline__ double growth_kink(const GrowthDev& g) {
  return g.model == COLA_SYMMETRON ? log(g.sa) : -1e300;
}

// mu(k, a) of the model (Secs. 5.1, 5.2, App. C)
__device__ __forceinline__ double growth_mu(const GrowthDev& g, const MBSpline& mb, double k, double a) {
  if (g.model == COLA_FR_HS1) {
    const double ol = 1.0 - g.om;
    const double X = g.om / (a * a * a) + 4.0 * ol, Y = g.om + 4.0 * ol;
    const double r = X / Y;
    const double a2m2 = a * a * kH0c * kH0c * Y * r * r * r / (2.0 * g.fr0);
    return 1.0 + k * k / (3.0 * (k * k + a2m2));
  }
  if (g.model == COLA_NDGP) {
    const double E = dE(a, g.om);
    const double oma = g.om / (a * a * a) / (E * E);
    return 1.0 + 1.0 / (3.0 * (1.0 + 2.0 * g.rc * E * (1.0 - 0.5 * oma)));
  }
  if (g.model == COLA_KMOUFLAGE) {   // App. B: 1 + 2 beta^2 / P_X(X(a)), P_X = 1 + m K0 X^(m-1)
    const double X = g.kx0 * pow(a, g.kxn);
    return 1.0 + 2.0 * g.kb * g.kb / (1.0 + g.km * g.kk0 * pow(X, (double)(g.km - 1)));
  }
  if (g.model == COLA_MBETA) {   // App. C: 1 + 2 beta^2 k^2/(k^2 + a^2 m^2), tabulated
    double b, m2, dm2;
    mb_eval(mb, a, b, m2, dm2);
    const double a2m2 = a * a * kH0c * kH0c * m2;
    return 1.0 + 2.0 * b * b * k * k / (k * k + a2m2);
  }
  if (g.model == COLA_SYMMETRON) {   // App. C: 1 + 2 beta^2 k^2/(k^2 + a^2 m^2)
    if (a <= g.sa) return 1.0;
    const double r = g.sa / a, s = 1.0 - r * r * r;
    const double a2m2 = a * a * kH0c * kH0c * g.sm * g.sm * s;
    return 1.0 + 2.0 * g.sb * g.sb * s * k * k / (k * k + a2m2);
  }
  return 1.0;
}

// 2 a^4 H^2 gamma_2^E(k, k1, k2, a) (Secs. 5.1, 5.2); c2 = cos^2 theta
__device__ __forceinline__ double gamma2E_term(const GrowthDev& g, const MBSpline& mb, double k, double k1,
                                               double k2, double c2, double a) {
  const double E = dE(a, g.om);
  const double a6 = (a * a * a) * (a * a * a);
  double g2 = 0.0;
  if (g.model == COLA_FR_HS1) {
    const double ol = 1.0 - g.om;
    const double X = g.om / (a * a * a) + 4.0 * ol, Y = g.om + 4.0 * ol;
    const double c0 = X * X * X / (2.0 * g.fr0 * Y * Y);
    const double ah = a * kH0c;
    const double P = k * k / (ah * ah) + c0, P1 = k1 * k1 / (ah * ah) + c0, P2 = k2 * k2 / (ah * ah) + c0;
    const double kah = k / (ah * E);
    g2 = -9.0 * g.om * g.om / (48.0 * a6 * g.fr0 * g.fr0) * kah * kah * (X * X * X * X * X) / (Y * Y * Y * Y)
         / (P * P1 * P2);
  } else if (g.model == COLA_NDGP) {
    const double oma = g.om / (a * a * a) / (E * E);
    const double beta = 1.0 + 2.0 * g.rc * E * (1.0 - 0.5 * oma);
    g2 = -(g.rc * g.rc * g.om * g.om) / (6.0 * E * E * beta * beta * beta * a6) * (1.0 - c2);
  } else if (g.model == COLA_MBETA) {
    // App. C with the tabulated beta, m^2/H0^2 and d(m^2/H0^2)/da
    double b, m2, dm2;
    mb_eval(mb, a, b, m2, dm2);
    const double ah = a * kH0c;
    const double P = k * k / (ah * ah) + m2, P1 = k1 * k1 / (ah * ah) + m2, P2 = k2 * k2 / (ah * ah) + m2;
    const double H = E * kH0c;
    g2 = m2 * dm2 * b * b * g.om / (2.0 * P * P1 * P2) * k * k / (a * a * a * a * H * H);
  } else if (g.model == COLA_SYMMETRON && a > g.sa) {
    // App. C: m^2 (dm^2/da) beta^2 Om / (2 H0^4 Pi Pi Pi) k^2/(a^4 H^2), Pi(q) = (q/(aH0))^2 + m^2/H0^2
    const double r = g.sa / a, s = 1.0 - r * r * r;
    const double m2 = g.sm * g.sm * s, dm2 = g.sm * g.sm * 3.0 * g.sa * g.sa * g.sa / (a * a * a * a);
    const double ah = a * kH0c;
    const double P = k * k / (ah * ah) + m2, P1 = k1 * k1 / (ah * ah) + m2, P2 = k2 * k2 / (ah * ah) + m2;
    const double H = E * kH0c;
    g2 = m2 * dm2 * g.sb * g.sb * s * g.om / (2.0 * P * P1 * P2) * k * k / (a * a * a * a * H * H);
  }
  return 2.0 * a * a * a * a * E * E * g2;
}

// mu(k, a) and 2 a^4 H^2 gamma_2(k, k/sqrt2, k/sqrt2, a) for the growth equations
__device__ __forceinline__ void growth_model(const GrowthDev& g, const MBSpline& mb, double k, double a,
                                             double& mu, double& g2term) {
  const double E = dE(a, g.om);
  if (g.model == COLA_FR_HS1) {
    const double ol = 1.0 - g.om;
    const double X = g.om / (a * a * a) + 4.0 * ol, Y = g.om + 4.0 * ol;
    const double r = X / Y;
    const double a2m2 = a * a * kH0c * kH0c * Y * r * r * r / (2.0 * g.fr0);
    const double k2 = k * k;
    mu = 1.0 + k2 / (3.0 * (k2 + a2m2));
    // gamma_2^E (Sec. 5.1) at k1 = k2 = k/sqrt2
    const double c0 = X * X * X / (2.0 * g.fr0 * Y * Y);
    const double ah = a * kH0c;
    const double Pk = k2 / (ah * ah) + c0;
    const double Ph = 0.5 * k2 / (ah * ah) + c0;
    const double kah = k / (ah * E);
    const double X5Y4 = (X * X * X * X * X) / (Y * Y * Y * Y);
    const double g2 = -9.0 * g.om * g.om / (48.0 * ((a * a * a) * (a * a * a)) * g.fr0 * g.fr0) * kah * kah * X5Y4
                      / (Pk * Ph * Ph);
    g2term = 2.0 * a * a * a * a * E * E * g2;
  } else if (g.model == COLA_NDGP) {
    const double oma = g.om / (a * a * a) / (E * E);
    const double beta = 1.0 + 2.0 * g.rc * E * (1.0 - 0.5 * oma);
    mu = 1.0 + 1.0 / (3.0 * beta);
    const double g2 = -(g.rc * g.rc * g.om * g.om) / (6.0 * E * E * beta * beta * beta * ((a * a * a) * (a * a * a)));
    g2term = 2.0 * a * a * a * a * E * E * g2;
  } else if (g.model == COLA_KMOUFLAGE) {   // gamma_2 = 0
    mu = growth_mu(g, mb, k, a);
    g2term = 0.0;
  } else if (g.model == COLA_SYMMETRON || g.model == COLA_MBETA) {
    mu = growth_mu(g, mb, k, a);
    g2term = gamma2E_term(g, mb, k, k * M_SQRT1_2, k * M_SQRT1_2, 0.0, a);
  } else {
    mu = 1.0;
    g2term = 0.0;
  }
}

// d y / d ln a for y = (D1, D1', D2, D2'), ' = d/dtau; d/dln a = (a^2 E)^-1 d/dtau.
// HALF (the COLA_READ_D2_HALF_K reading): y also carries (D1, D1') at k/sqrt2, and the D2
// source takes that D1 squared in place of D1(k)^2.
template <bool HALF>
__device__ __forceinline__ void growth_rhs(const GrowthDev& g, const MBSpline& mb, double k, double lna,
                                           const double* y, double* dy) {
  const double a = exp(lna);
  double mu, g2t;
  growth_model(g, mb, k, a, mu, g2t);
  const double kap = 1.5 * g.om * a;
  const double f = 1.0 / (a * a * dE(a, g.om));
  const double ds = HALF ? y[4] : y[0];
  dy[0] = y[1] * f;
  dy[1] = kap * mu * y[0] * f;
  dy[2] = y[3] * f;
  dy[3] = (kap * mu * y[2] - kap * mu * ds * ds - g2t * ds * ds) * f;
  if constexpr (HALF) {
    dy[4] = y[5] * f;
    dy[5] = kap * growth_mu(g, mb, k * M_SQRT1_2, a) * y[4] * f;
  }
}

template <bool HALF>
__device__ __forceinline__ void store_slice(const GrowthDev& g, const MBSpline& mb, double k, double a,
                                            const double* y, double* out) {
  double mu, g2t;
  growth_model(g, mb, k, a, mu, g2t);
  const double kap = 1.5 * g.om * a;
  const double ds = HALF ? y[4] : y[0];
  out[0] = y[0];
  out[1] = y[1];
  out[2] = kap * mu * y[0];
  out[3] = y[2];
  out[4] = y[3];
  out[5] = kap * mu * y[2] - kap * mu * ds * ds - g2t * ds * ds;
}

template <bool HALF>
__global__ void __launch_bounds__(64) k_growth_ode(GrowthDev g, MBSpline mb, double* __restrict__ table,
                                                   double* __restrict__ ref) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t > g.n_k) return;
  GrowthDev gg = g;
  double k;
  if (t == g.n_k) {   // LCDM reference for the initial spectrum: D1(a = 1), mu = 1
    gg.model = COLA_LCDM;
    k = 0.0;
  } else {
    k = g.kdep ? g.kf * sqrt((double)t) : 0.0;
  }
  const double ai = g.a_ini;
  const double g0 = ai * ai * dE(ai, g.om);
  constexpr int NV = HALF ? 6 : 4;
  double y[NV];
  y[0] = 1.0;
  y[1] = g0;
  y[2] = -3.0 / 7.0;
  y[3] = -6.0 / 7.0 * g0;
  if constexpr (HALF) {
    y[4] = 1.0;
    y[5] = g0;
  }
  double lna = log(ai);
  const int nsl = (t == g.n_k) ? 1 : g.n_steps + 1;
  for (int i = 0; i < nsl; ++i) {
    const double a_target = (t == g.n_k) ? 1.0 : ai + i * (1.0 - ai) / g.n_steps;
    const double l1 = log(a_target);
    rk4_to_knots<NV>(y, lna, l1, growth_kink(gg), gg, mb,
                     [&](double l, const double* yy, double* dy) { growth_rhs<HALF>(gg, mb, k, l, yy, dy); });
    if (t == g.n_k)
      store_slice<HALF>(gg, mb, k, a_target, y, ref);
    else
      store_slice<HALF>(gg, mb, k, a_target, y, table + ((int64_t)i * g.n_k + t) * 6);
  }
}

void launch_growth_ode(const cola_params& p, const Layout& L, double* table, double* ref,
                       hipStream_t s) {
  ProfScope ps("growth_ode", s);
  GrowthDev g;
  g.om = p.omega_m;
  g.fr0 = p.fr0_abs;
  g.rc = p.rc_h0;
  g.a_ini = 1.0 / (1.0 + p.z_init);
  g.kf = 2.0 * M_PI / p.box;
  g.model = (p.growth_mode == 1) ? COLA_LCDM : p.model;
  g.sb = p.sym_beta;
  g.sm = p.sym_mass;
  g.sa = p.sym_astar;
  g.kb = p.km_beta;
  g.kk0 = p.km_k0;
  g.kx0 = p.km_x0;
  g.kxn = p.km_xn;
  g.km = p.km_m;
  g.kdep = L.kdep ? 1 : 0;
  g.n_steps = p.n_steps;
  g.n_k = L.n_k;
  const int64_t threads = L.n_k + 1;
  const MBSpline mb = mb_spline(p);
  if (p.readings & COLA_READ_D2_HALF_K)
    hipLaunchKernelGGL(k_growth_ode<true>, dim3((unsigned)((threads + 63) / 64)), dim3(64), 0, s, g,
                       mb, table, ref);
  else
    hipLaunchKernelGGL(k_growth_ode<false>, dim3((unsigned)((threads + 63) / 64)), dim3(64), 0, s, g,
                       mb, table, ref);
  COLA_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ per-step LPT coefficients
__global__ void k_lpt_coef(const double* __restrict__ table, int64_t slice0, int64_t slice1,
                           const StepDev* __restrict__ steps, const int* __restrict__ ctr,
                           int64_t n_k, float2* __restrict__ coef) {
  if (steps) {
    slice0 = steps[*ctr].slice0;
    slice1 = steps[*ctr].slice1;
  }
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n_k;
       k += (int64_t)gridDim.x * blockDim.x) {
    const double* t0 = table + slice0 + 6 * k;
    const double* t1 = table + slice1 + 6 * k;
    coef[k] = make_float2((float)t0[2], (float)t0[5]);
    coef[n_k + k] = make_float2((float)(t1[0] - t0[0]), (float)(t1[3] - t0[3]));
  }
}

void launch_lpt_coef(const Layout& L, const double* table, int64_t slice0, int64_t slice1,
                     const StepDev* steps, const int* ctr, float2* coef, hipStream_t s) {
  ProfScope ps("lpt_coef", s);
  const unsigned g = (unsigned)std::min<int64_t>((L.n_k + 255) / 256, 4096);
  hipLaunchKernelGGL(k_lpt_coef, dim3(g), dim3(256), 0, s, table, slice0, slice1, steps, ctr,
                     L.n_k, coef);
  COLA_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ triangle growth
// Exact second-order growth of a Fourier triangle k = k1 + k2 (Sec. 4.2) beside the
// approximation the path uses, D2_hat(k)(1 - cos^2 theta), for checking it (Fig. 1):
//   D2'' = kappa mu(k) D2 - kappa mu(k) D1(k1) D1(k2)
//          [1 - (2 mu(k1) - mu(k))/mu(k) cos^2 theta + 2 a^4 H^2 gamma_2/(kappa mu(k))],
//   gamma_2 = gamma_2^E(k, k1, k2) + (3/2) Omega_m(a) [mu(k) - mu(k1)] k1.k2/k2^2  (Sec. 4),
// with D2 = -(3/7)(1 - cos^2 theta), D2' = -(6/7)(1 - cos^2 theta) a^2 E at a_ini; the
// terms that single out k1 are taken as printed.  Same integrator as k_growth_ode.

// y = (D1(k1), D1'(k1), D1(k2), D1'(k2), D1(k), D1'(k), D2, D2', D2_hat, D2_hat')
struct Triangle {
  double k, k1, k2, c, c2;
};

__device__ __forceinline__ void triangle_rhs(const GrowthDev& g, const MBSpline& mb, const Triangle& t,
                                             double lna, const double* y, double* dy) {
  const double a = exp(lna);
  const double E = dE(a, g.om);
  const double kap = 1.5 * g.om * a;
  const double f = 1.0 / (a * a * E);
  const double mu = growth_mu(g, mb, t.k, a), mu1 = growth_mu(g, mb, t.k1, a), mu2 = growth_mu(g, mb, t.k2, a);
  const double oma = g.om / (a * a * a) / (E * E);
  const double g2t = gamma2E_term(g, mb, t.k, t.k1, t.k2, t.c2, a)
                     + 2.0 * a * a * a * a * E * E * 1.5 * oma * (mu - mu1) * (t.k1 / t.k2) * t.c;
  const double src = 1.0 - (2.0 * mu1 - mu) / mu * t.c2 + g2t / (kap * mu);
  double muh, g2h;
  growth_model(g, mb, t.k, a, muh, g2h);   // the approximate equation at k
  dy[0] = y[1] * f;
  dy[1] = kap * mu1 * y[0] * f;
  dy[2] = y[3] * f;
  dy[3] = kap * mu2 * y[2] * f;
  dy[4] = y[5] * f;
  dy[5] = kap * mu * y[4] * f;
  dy[6] = y[7] * f;
  dy[7] = (kap * mu * y[6] - kap * mu * y[0] * y[2] * src) * f;
  dy[8] = y[9] * f;
  dy[9] = (kap * muh * y[8] - kap * muh * y[4] * y[4] - g2h * y[4] * y[4]) * f;
}

__global__ void __launch_bounds__(64) k_growth_triangle(GrowthDev g, MBSpline mb, int n, const double* __restrict__ tri, double a_end,
                                  double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  Triangle t;
  t.k = tri[3 * i];
  t.k1 = tri[3 * i + 1];
  t.k2 = tri[3 * i + 2];
  const double tol = 1e-12 * (t.k1 + t.k2);
  if (!(t.k1 > 0.0 && t.k2 > 0.0 && t.k >= fabs(t.k1 - t.k2) - tol && t.k <= t.k1 + t.k2 + tol)) {
    out[2 * i] = out[2 * i + 1] = __builtin_nan("");
    return;
  }
  t.c = fmin(1.0, fmax(-1.0, (t.k * t.k - t.k1 * t.k1 - t.k2 * t.k2) / (2.0 * t.k1 * t.k2)));
  t.c2 = t.c * t.c;
  const double ai = g.a_ini;
  const double g0 = ai * ai * dE(ai, g.om);
  const double s2 = 1.0 - t.c2;
  double y[10] = {1.0, g0, 1.0, g0, 1.0, g0, -3.0 / 7.0 * s2, -6.0 / 7.0 * s2 * g0, -3.0 / 7.0,
                  -6.0 / 7.0 * g0};
  double lna = log(ai);
  rk4_to_knots<10>(y, lna, log(a_end), growth_kink(g), g, mb,
                   [&](double l, const double* yy, double* dy) { triangle_rhs(g, mb, t, l, yy, dy); });
  out[2 * i] = y[6];
  out[2 * i + 1] = y[8] * s2;
}

void launch_growth_triangles(const cola_params& p, int n, const double* tri, double a, double* out,
                             hipStream_t s) {
  ProfScope ps("growth_triangles", s);
  GrowthDev g{};
  g.om = p.omega_m;
  g.fr0 = p.fr0_abs;
  g.rc = p.rc_h0;
  g.a_ini = 1.0 / (1.0 + p.z_init);
  g.model = (p.growth_mode == 1) ? COLA_LCDM : p.model;
  g.sb = p.sym_beta;
  g.sm = p.sym_mass;
  g.sa = p.sym_astar;
  g.kb = p.km_beta;
  g.kk0 = p.km_k0;
  g.kx0 = p.km_x0;
  g.kxn = p.km_xn;
  g.km = p.km_m;
  const MBSpline mb = mb_spline(p);
  hipLaunchKernelGGL(k_growth_triangle, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, g, mb, n, tri,
                     a, out);
  COLA_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ white noise
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ float unit_open(uint64_t z) {   // ((z >> 11) + 1/2) 2^-53 in (0,1)
  return ((float)(z >> 11) + 0.5f) * 0x1p-53f;
}

__global__ void k_noise(uint64_t seed, int n, int rpitch, int64_t rplane, float* __restrict__ padded,
                        float* __restrict__ flat) {
  const int64_t total = (int64_t)n * n * n;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < total;
       j += (int64_t)gridDim.x * blockDim.x) {
    const float u0 = unit_open(splitmix64(seed, 2 * (uint64_t)j));
    const float u1 = unit_open(splitmix64(seed, 2 * (uint64_t)j + 1));
    const float g = sqrtf(-2.f * logf(u0)) * cospif(2.f * u1);
    if (padded) {
      const int64_t r = j / n;
      padded[(r / n) * rplane + (r % n) * rpitch + (j - r * n)] = g;
    }
    if (flat) flat[j] = g;
  }
}

void launch_noise(const cola_params& p, int n, int pitch, int64_t plane, float* padded, float* flat,
                  hipStream_t s) {
  ProfScope ps("noise", s);
  const int64_t total = (int64_t)n * n * n;
  const unsigned g = (unsigned)std::min<int64_t>((total + 255) / 256, 1 << 20);
  hipLaunchKernelGGL(k_noise, dim3(g), dim3(256), 0, s, p.seed, n, 2 * pitch, 2 * plane, padded,
                     flat);
  COLA_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ delta_k -> phi1_k
struct EHDev {
  float A;        // sigma8 normalisation of k^ns T^2
  float ns, th2, omh, alpha, kfac;   // kfac = 0.43 s h (s in Mpc)
};

__device__ __forceinline__ float eh_T(const EHDev& e, float k) {
  const float kk = e.kfac * k;
  const float k4 = (kk * kk) * (kk * kk);
  const float gam = e.omh * (e.alpha + (1.f - e.alpha) / (1.f + k4));
  const float q = k * e.th2 / gam;
  const float L0 = logf(2.f * 2.718281828459045f + 1.8f * q);
  const float C0 = 14.2f + 731.f / (1.f + 62.5f * q);
  return L0 / (L0 + C0 * q * q);
}

// phi1_k = W_k sqrt(N P_ini(k) / L^3) / k^2 ; zero at k = 0 and in row padding
__global__ void k_ic_phi1(const float2* __restrict__ wk, float2* __restrict__ phi1, int n, int pitch,
                          int64_t plane, float kf, float norm, EHDev eh,
                          const double* __restrict__ ref) {
  const float d1 = (float)ref[0];
  const float inv_d1sq = 1.f / (d1 * d1);
  const int h = n / 2;
  const int64_t total = (int64_t)n * n * pitch;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int iz = (int)(e % pitch);
    const int64_t r = e / pitch;
    const int iy = (int)(r % n), ix = (int)(r / n);
    const int nx = ix < h ? ix : ix - n, ny = iy < h ? iy : iy - n;
    const int n2 = nx * nx + ny * ny + iz * iz;
    const int64_t idx = ix * plane + (int64_t)iy * pitch + iz;
    float2 out = make_float2(0.f, 0.f);
    if (iz <= h && n2 > 0) {
      const float k2 = kf * kf * (float)n2;
      const float k = sqrtf(k2);
      const float T = eh_T(eh, k);
      const float P = eh.A * powf(k, eh.ns) * T * T * inv_d1sq;
      const float amp = sqrtf(norm * P) / k2;
      const float2 w = wk[idx];
      out = make_float2(amp * w.x, amp * w.y);
    }
    phi1[idx] = out;
  }
}

void launch_ic_phi1(const cola_params& p, const Layout& L, const float2* wk, float2* phi1,
                    double A_norm, const double* ref, hipStream_t s) {
  ProfScope ps("ic_phi1", s);
  EHDev e;
  const double omh2 = p.omega_m * p.h * p.h, obh2 = p.omega_b * p.h * p.h;
  const double fb = p.omega_b / p.omega_m;
  const double sh = 44.5 * std::log(9.83 / omh2) / std::sqrt(1.0 + 10.0 * std::pow(obh2, 0.75));
  e.A = (float)A_norm;
  e.ns = (float)p.n_s;
  const double th = p.t_cmb / 2.7;
  e.th2 = (float)(th * th);
  e.omh = (float)(p.omega_m * p.h);
  e.alpha = (float)(1.0 - 0.328 * std::log(431.0 * omh2) * fb + 0.38 * std::log(22.3 * omh2) * fb * fb);
  e.kfac = (float)(0.43 * sh * p.h);
  const double N = (double)L.N;
  const float norm = (float)(N / (p.box * p.box * p.box));
  const int64_t total = (int64_t)L.np * L.np * L.pitch_p;
  const unsigned g = (unsigned)std::min<int64_t>((total + 255) / 256, 1 << 20);
  hipLaunchKernelGGL(k_ic_phi1, dim3(g), dim3(256), 0, s, wk, phi1, L.np, L.pitch_p, L.plane_p,
                     (float)(2.0 * M_PI / p.box), norm, e, ref);
  COLA_LAUNCH_CHECK();
}

}  // namespace cola
