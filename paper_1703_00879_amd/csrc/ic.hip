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
  int model;          // effective model for the growth (LCDM when growth_mode = 1)
  int kdep;           // table indexed by |nu|^2
  int n_steps;
  int64_t n_k;
};

__device__ __forceinline__ double dE(double a, double om) { return sqrt(om / (a * a * a) + 1.0 - om); }

// mu(k, a) and 2 a^4 H^2 gamma_2(k, k/sqrt2, k/sqrt2, a) for the growth equations
__device__ __forceinline__ void growth_model(const GrowthDev& g, double k, double a, double& mu,
                                             double& g2term) {
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
  } else {
    mu = 1.0;
    g2term = 0.0;
  }
}

// d y / d ln a for y = (D1, D1', D2, D2'), ' = d/dtau; d/dln a = (a^2 E)^-1 d/dtau
__device__ __forceinline__ void growth_rhs(const GrowthDev& g, double k, double lna, const double y[4],
                                           double dy[4]) {
  const double a = exp(lna);
  double mu, g2t;
  growth_model(g, k, a, mu, g2t);
  const double kap = 1.5 * g.om * a;
  const double f = 1.0 / (a * a * dE(a, g.om));
  dy[0] = y[1] * f;
  dy[1] = kap * mu * y[0] * f;
  dy[2] = y[3] * f;
  dy[3] = (kap * mu * y[2] - kap * mu * y[0] * y[0] - g2t * y[0] * y[0]) * f;
}

__device__ __forceinline__ void store_slice(const GrowthDev& g, double k, double a, const double y[4],
                                            double* out) {
  double mu, g2t;
  growth_model(g, k, a, mu, g2t);
  const double kap = 1.5 * g.om * a;
  out[0] = y[0];
  out[1] = y[1];
  out[2] = kap * mu * y[0];
  out[3] = y[2];
  out[4] = y[3];
  out[5] = kap * mu * y[2] - kap * mu * y[0] * y[0] - g2t * y[0] * y[0];
}

__global__ void k_growth_ode(GrowthDev g, double* __restrict__ table, double* __restrict__ ref) {
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
  double y[4] = {1.0, g0, -3.0 / 7.0, -6.0 / 7.0 * g0};
  double lna = log(ai);
  const int nsl = (t == g.n_k) ? 1 : g.n_steps + 1;
  for (int i = 0; i < nsl; ++i) {
    const double a_target = (t == g.n_k) ? 1.0 : ai + i * (1.0 - ai) / g.n_steps;
    const double l1 = log(a_target);
    const int nsub = (int)ceil((l1 - lna) / 1e-3);
    if (nsub > 0) {
      const double h = (l1 - lna) / nsub;
      for (int s = 0; s < nsub; ++s) {
        double k1[4], k2[4], k3[4], k4[4], yt[4];
        growth_rhs(gg, k, lna, y, k1);
        for (int c = 0; c < 4; ++c) yt[c] = y[c] + 0.5 * h * k1[c];
        growth_rhs(gg, k, lna + 0.5 * h, yt, k2);
        for (int c = 0; c < 4; ++c) yt[c] = y[c] + 0.5 * h * k2[c];
        growth_rhs(gg, k, lna + 0.5 * h, yt, k3);
        for (int c = 0; c < 4; ++c) yt[c] = y[c] + h * k3[c];
        growth_rhs(gg, k, lna + h, yt, k4);
        for (int c = 0; c < 4; ++c) y[c] += h / 6.0 * (k1[c] + 2.0 * k2[c] + 2.0 * k3[c] + k4[c]);
        lna = (s + 1 == nsub) ? l1 : lna + h;
      }
    }
    if (t == g.n_k)
      store_slice(gg, k, a_target, y, ref);
    else
      store_slice(gg, k, a_target, y, table + ((int64_t)i * g.n_k + t) * 6);
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
  g.kdep = L.kdep ? 1 : 0;
  g.n_steps = p.n_steps;
  g.n_k = L.n_k;
  const int64_t threads = L.n_k + 1;
  hipLaunchKernelGGL(k_growth_ode, dim3((unsigned)((threads + 63) / 64)), dim3(64), 0, s, g, table,
                     ref);
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

__device__ __forceinline__ double growth_mu(const GrowthDev& g, double k, double a) {
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
  return 1.0;
}

// 2 a^4 H^2 gamma_2^E(k, k1, k2, a) (Secs. 5.1, 5.2); c2 = cos^2 theta
__device__ __forceinline__ double gamma2E_term(const GrowthDev& g, double k, double k1, double k2,
                                               double c2, double a) {
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
  }
  return 2.0 * a * a * a * a * E * E * g2;
}

// y = (D1(k1), D1'(k1), D1(k2), D1'(k2), D1(k), D1'(k), D2, D2', D2_hat, D2_hat')
struct Triangle {
  double k, k1, k2, c, c2;
};

__device__ __forceinline__ void triangle_rhs(const GrowthDev& g, const Triangle& t, double lna,
                                             const double y[10], double dy[10]) {
  const double a = exp(lna);
  const double E = dE(a, g.om);
  const double kap = 1.5 * g.om * a;
  const double f = 1.0 / (a * a * E);
  const double mu = growth_mu(g, t.k, a), mu1 = growth_mu(g, t.k1, a), mu2 = growth_mu(g, t.k2, a);
  const double oma = g.om / (a * a * a) / (E * E);
  const double g2t = gamma2E_term(g, t.k, t.k1, t.k2, t.c2, a)
                     + 2.0 * a * a * a * a * E * E * 1.5 * oma * (mu - mu1) * (t.k1 / t.k2) * t.c;
  const double src = 1.0 - (2.0 * mu1 - mu) / mu * t.c2 + g2t / (kap * mu);
  double muh, g2h;
  growth_model(g, t.k, a, muh, g2h);   // the approximate equation at k
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

__global__ void k_growth_triangle(GrowthDev g, int n, const double* __restrict__ tri, double a_end,
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
  const double l1 = log(a_end);
  const int nsub = (int)ceil((l1 - lna) / 1e-3);
  if (nsub > 0) {
    const double h = (l1 - lna) / nsub;
    for (int s = 0; s < nsub; ++s) {
      double k1[10], k2[10], k3[10], k4[10], yt[10];
      triangle_rhs(g, t, lna, y, k1);
      for (int c = 0; c < 10; ++c) yt[c] = y[c] + 0.5 * h * k1[c];
      triangle_rhs(g, t, lna + 0.5 * h, yt, k2);
      for (int c = 0; c < 10; ++c) yt[c] = y[c] + 0.5 * h * k2[c];
      triangle_rhs(g, t, lna + 0.5 * h, yt, k3);
      for (int c = 0; c < 10; ++c) yt[c] = y[c] + h * k3[c];
      triangle_rhs(g, t, lna + h, yt, k4);
      for (int c = 0; c < 10; ++c) y[c] += h / 6.0 * (k1[c] + 2.0 * k2[c] + 2.0 * k3[c] + k4[c]);
      lna = (s + 1 == nsub) ? l1 : lna + h;
    }
  }
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
  hipLaunchKernelGGL(k_growth_triangle, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, g, n, tri, a,
                     out);
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
