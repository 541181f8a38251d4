// Fourier-space operators applied to half-complex fields, evaluated per mode.
//
// Layout: element (ix, iy, iz) of an n^3 half-complex field sits at
// (ix * n + iy) * pitch + iz; nu_x = ix (ix < n/2) or ix - n, likewise nu_y, nu_z = iz
// (0 .. n/2; iz > n/2 is row padding and evaluates to 0); k = kf * nu, kf = 2 pi / L.
// An odd factor i k_c is zero on the Nyquist plane of axis c; a mixed factor k_i k_j
// (i != j) is zero on the Nyquist plane of either axis; the k = 0 mode of every Green's
// function is zero.  These keep every inverse transform Hermitian.
#pragma once

#include "internal.h"

namespace cola {

// Hardware reciprocal, square root and base-2 exponential (each within about 1 ulp): the
// correctly rounded library forms expand to ten or more instructions apiece, which the
// per-mode operators and the screening factors cannot afford in issue-limited passes.
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float fast_exp(float x) {
  return __builtin_amdgcn_exp2f(x * 1.44269504088896340736f);
}

__device__ __forceinline__ float smooth_window(float k2R2, int filter) {
  if (filter == 0) return fast_exp(-0.5f * k2R2);             // Gaussian
  if (filter == 2) return k2R2 <= 1.f ? 1.f : 0.f;            // sharp-k, k R <= 1
  // spherical top-hat 3 (sin x - x cos x)/x^3; its Taylor series below x = 1/2, where
  // the closed form cancels in single precision
  if (k2R2 < 0.25f) return 1.f - k2R2 * (0.1f - k2R2 * (1.f / 280.f - k2R2 * (1.f / 15120.f)));
  const float x = sqrtf(k2R2);
  float s, c;
  sincosf(x, &s, &c);
  return 3.f * (s - x * c) / (x * x * x);
}

// Value of operator KIND at mode (ix, iy, iz) given the raw source values a (and b).
template <int KIND>
__device__ __forceinline__ float2 kspace_apply(const KOp& op, int ix, int iy, int iz, float2 a,
                                               float2 b) {
  const int n = op.n, h = n >> 1;
  if (iz > h) return make_float2(0.f, 0.f);
  const int nx = ix < h ? ix : ix - n;
  const int ny = iy < h ? iy : iy - n;
  const int nz = iz;
  const int n2 = nx * nx + ny * ny + nz * nz;
  // component selection by value (no captured or dynamically indexed locals, which the
  // compiler would otherwise keep in private scratch memory)
  const int ic = op.comp == 0 ? ix : (op.comp == 1 ? iy : iz);
  const int jc = op.comp2 == 0 ? ix : (op.comp2 == 1 ? iy : iz);
  const bool nyq_c = ic == h, nyq_c2 = jc == h;
  const float k_c = op.kf * (float)(op.comp == 0 ? nx : (op.comp == 1 ? ny : nz));
  const float k_c2 = op.kf * (float)(op.comp2 == 0 ? nx : (op.comp2 == 1 ? ny : nz));
  if constexpr (KIND == K_COPY) {
    return make_float2(op.scale * a.x, op.scale * a.y);
  } else if constexpr (KIND == K_FORCE) {
    if (n2 == 0 || nyq_c) return make_float2(0.f, 0.f);
    const float k2 = op.kf * op.kf * (float)n2;
    const float gn = op.g_n * fast_rcp(k2), g5 = op.g_5 * fast_rcp(k2 + op.a2m2);
    const float2 g = make_float2(gn * a.x + g5 * b.x, gn * a.y + g5 * b.y);
    const float f = k_c * op.scale;   // -i k_c g
    return make_float2(f * g.y, -f * g.x);
  } else if constexpr (KIND == K_POT) {
    if (n2 == 0) return make_float2(0.f, 0.f);
    const float k2 = op.kf * op.kf * (float)n2;
    const float f = op.g_n * fast_rcp(k2) * op.scale;
    return make_float2(f * a.x, f * a.y);
  } else if constexpr (KIND == K_SMOOTH) {
    if (n2 == 0) return make_float2(0.f, 0.f);
    const float k2 = op.kf * op.kf * (float)n2;
    const float f = smooth_window(k2 * op.r_smooth * op.r_smooth, op.filter) * op.scale;
    return make_float2(f * a.x, f * a.y);
  } else if constexpr (KIND == K_LPT) {
    if (n2 == 0 || nyq_c) return make_float2(0.f, 0.f);
    float x1, x2;
    const int64_t e = (int64_t)(op.kdep ? n2 : 0) * 6;
    const double* t0 = op.table + op.tab_slice0 + e;
    const double* t1 = op.table + op.tab_slice1 + e;
    if (op.coef) {                   // the step's FP32 pairs: one 8-byte read per mode
      const float2 cf = op.coef[op.kdep ? n2 : 0];
      x1 = cf.x;
      x2 = cf.y;
    } else if (op.lpt_mode == 0) {   // second derivatives at slice 0
      x1 = (float)t0[2];
      x2 = (float)t0[5];
    } else if (op.lpt_mode == 1) {   // D(slice 1) - D(slice 0)
      x1 = (float)(t1[0] - t0[0]);
      x2 = (float)(t1[3] - t0[3]);
    } else {                         // D(slice 0)
      x1 = (float)t0[0];
      x2 = (float)t0[3];
    }
    const float2 g = make_float2(x1 * a.x + x2 * b.x, x1 * a.y + x2 * b.y);
    const float f = k_c * op.scale;   // +i k_c g
    return make_float2(-f * g.y, f * g.x);
  } else if constexpr (KIND == K_HESS) {
    if (op.comp != op.comp2 && (nyq_c || nyq_c2)) return make_float2(0.f, 0.f);
    const float f = -k_c * k_c2 * op.scale;
    return make_float2(f * a.x, f * a.y);
  } else if constexpr (KIND == K_GRAD) {
    if (nyq_c) return make_float2(0.f, 0.f);
    const float f = k_c * op.scale;
    return make_float2(-f * a.y, f * a.x);
  } else {
    return make_float2(0.f, 0.f);
  }
}

// Sources an operator reads (a always; b for K_FORCE with a screened source and K_LPT).
template <int KIND>
__device__ __forceinline__ bool kspace_uses_b(const KOp& op) {
  return (KIND == K_LPT) || (KIND == K_FORCE && op.b != nullptr);
}

template <int KIND>
__device__ __forceinline__ float2 kspace_eval(const KOp& op, int ix, int iy, int iz, int64_t idx) {
  const float2 a = op.a[idx];
  const float2 b = kspace_uses_b<KIND>(op) ? op.b[idx] : a;
  return kspace_apply<KIND>(op, ix, iy, iz, a, b);
}

// Potential part of the force operator: [g_n/k^2 a + g_5/(k^2 + a2m2) b] * scale
// (zero at k = 0 and in row padding).
__device__ __forceinline__ float2 green_force(const KOp& op, int ix, int iy, int iz, float2 a, float2 b) {
  const int n = op.n, h = n >> 1;
  if (iz > h) return make_float2(0.f, 0.f);
  const int nx = ix < h ? ix : ix - n, ny = iy < h ? iy : iy - n;
  const int n2 = nx * nx + ny * ny + iz * iz;
  if (n2 == 0) return make_float2(0.f, 0.f);
  const float k2 = op.kf * op.kf * (float)n2;
  const float gn = op.g_n * fast_rcp(k2) * op.scale, g5 = op.g_5 * fast_rcp(k2 + op.a2m2) * op.scale;
  return make_float2(gn * a.x + g5 * b.x, gn * a.y + g5 * b.y);
}

// -i k_comp g, zero on the Nyquist plane of axis comp.
__device__ __forceinline__ float2 grad_minus_i(const KOp& op, int ix, int iy, int iz, int comp, float2 g) {
  const int n = op.n, h = n >> 1;
  const int ic = comp == 0 ? ix : (comp == 1 ? iy : iz);
  if (ic == h) return make_float2(0.f, 0.f);
  const int nu = comp == 2 ? ic : (ic < h ? ic : ic - n);
  const float k = op.kf * (float)nu;
  return make_float2(k * g.y, -k * g.x);
}

}  // namespace cola
