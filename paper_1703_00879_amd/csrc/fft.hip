// Stockham 3D real FFT for gfx950.
//
// A 3D transform of an n^3 mesh is three passes over HBM:
//   Z pass  (contiguous rows): real rows of n floats <-> half-complex rows of n/2 + 1
//           values, via an n/2-point complex transform of (x_even + i x_odd) and the
//           usual split/merge twiddle step;
//   Y pass  (stride = pitch):  length-n complex transforms over tiles of B contiguous
//           columns, one x-plane at a time;
//   X pass  (stride = n*pitch): length-n complex transforms over tiles of B contiguous
//           (y, z) columns.
// Each work-group stages its tile in LDS as [element][column] so that a wavefront reads
// B consecutive columns (128 B) per element -- global loads and stores are fully
// coalesced in every pass -- and runs the radix-8/4/3/2 Stockham stages in LDS with the
// butterfly operands held in registers across each stage's barrier.  The inverse
// transform's X pass can evaluate a k-space operator while loading (Poisson/fifth-force
// Green's function and gradient, smoothing window, LPT growth factors), so the k-space
// multiply costs no pass of its own.
//
// Conventions: forward e^{-i k x}, inverse e^{+i k x}, both unnormalised.  Twiddles come
// from a table exp(-2 pi i t / n) built on the host in double precision.

#include "internal.h"
#include "kspace.h"

namespace cola {

// ------------------------------------------------------------------ complex helpers
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
// multiply by DIR * i  (DIR = -1: -i, DIR = +1: +i)
template <int DIR>
__device__ __forceinline__ float2 mul_i(float2 a) {
  return DIR < 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
}

// ------------------------------------------------------------------ small DFTs
template <int R, int DIR>
struct Dft;

template <int DIR>
struct Dft<2, DIR> {
  static __device__ __forceinline__ void run(float2* v) {
    float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <int DIR>
struct Dft<3, DIR> {
  static __device__ __forceinline__ void run(float2* v) {
    const float h = 0.86602540378443864676f;  // sqrt(3)/2
    float2 t = cadd(v[1], v[2]);
    float2 d = csub(v[1], v[2]);
    float2 m = make_float2(v[0].x - 0.5f * t.x, v[0].y - 0.5f * t.y);
    float2 s = mul_i<DIR>(make_float2(h * d.x, h * d.y));
    v[0] = cadd(v[0], t);
    v[1] = cadd(m, s);
    v[2] = csub(m, s);
  }
};

template <int DIR>
struct Dft<4, DIR> {
  static __device__ __forceinline__ void run(float2* v) {
    float2 t0 = cadd(v[0], v[2]);
    float2 t1 = csub(v[0], v[2]);
    float2 t2 = cadd(v[1], v[3]);
    float2 t3 = mul_i<DIR>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  }
};

template <int DIR>
struct Dft<8, DIR> {
  static __device__ __forceinline__ void run(float2* v) {
    const float c = 0.70710678118654752440f;
    float2 e[4] = {v[0], v[2], v[4], v[6]};
    float2 o[4] = {v[1], v[3], v[5], v[7]};
    Dft<4, DIR>::run(e);
    Dft<4, DIR>::run(o);
    // o[k] *= w8^k, w8 = exp(DIR * 2 pi i / 8)
    o[1] = make_float2(c * (o[1].x - DIR * o[1].y), c * (o[1].y + DIR * o[1].x));
    o[2] = mul_i<DIR>(o[2]);
    o[3] = make_float2(c * (-o[3].x - DIR * o[3].y), c * (-o[3].y + DIR * o[3].x));
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[k] = cadd(e[k], o[k]);
      v[k + 4] = csub(e[k], o[k]);
    }
  }
};

// ------------------------------------------------------------------ plans
// Radix plan and per-thread element count E for each supported transform length.
template <int N>
struct Plan;
#define COLA_PLAN(N_, E_, NST_, ...)                              \
  template <>                                                     \
  struct Plan<N_> {                                               \
    static constexpr int E = E_;                                  \
    static constexpr int nst = NST_;                              \
    static constexpr int rad[NST_] = {__VA_ARGS__};               \
  };
COLA_PLAN(4, 4, 1, 4)
COLA_PLAN(6, 6, 2, 2, 3)
COLA_PLAN(8, 8, 1, 8)
COLA_PLAN(12, 12, 2, 4, 3)
COLA_PLAN(16, 16, 2, 4, 4)
COLA_PLAN(24, 24, 2, 8, 3)
COLA_PLAN(32, 8, 2, 8, 4)
COLA_PLAN(48, 24, 3, 8, 2, 3)
COLA_PLAN(64, 8, 2, 8, 8)
COLA_PLAN(96, 24, 3, 8, 4, 3)
COLA_PLAN(128, 8, 3, 8, 4, 4)
COLA_PLAN(192, 24, 3, 8, 8, 3)
COLA_PLAN(256, 8, 3, 8, 8, 4)
COLA_PLAN(384, 24, 4, 8, 4, 4, 3)
COLA_PLAN(512, 8, 3, 8, 8, 8)
COLA_PLAN(768, 24, 4, 8, 8, 4, 3)
COLA_PLAN(1024, 16, 4, 8, 8, 4, 4)
COLA_PLAN(1536, 24, 4, 8, 8, 8, 3)
COLA_PLAN(2048, 16, 4, 8, 8, 8, 4)
#undef COLA_PLAN

// One Stockham stage of radix R on B transforms of length N held in LDS as
// lds[j * LS + c] (element j of transform c).  Butterfly b = tid + i*T maps to
// column c = b % B (fastest, so lanes touch consecutive LDS words) and index j = b / B.
// All operands are read into registers before the barrier, so the stage is in place.
// Twiddles: tw[t * TWS] = exp(-2 pi i t / N).
template <int N, int R, int NS, int DIR, int E, int B, int LS, int TWS>
__device__ __forceinline__ void stockham_stage(float2* lds, int tid, int T, const float2* __restrict__ tw) {
  constexpr int NB = E / R;
  float2 v[NB][R];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = tid + i * T;
    const int c = b % B, j = b / B;
#pragma unroll
    for (int r = 0; r < R; ++r) v[i][r] = lds[(j + r * (N / R)) * LS + c];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = tid + i * T;
    const int c = b % B, j = b / B;
    const int k = j % NS;
    if (NS > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        float2 w = tw[(r * k * (N / (NS * R))) * TWS];
        if (DIR > 0) w.y = -w.y;
        v[i][r] = cmul(v[i][r], w);
      }
    }
    Dft<R, DIR>::run(v[i]);
    const int idxD = (j / NS) * NS * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) lds[(idxD + r * NS) * LS + c] = v[i][r];
  }
  __syncthreads();
}

template <int N, int DIR, int E, int B, int LS, int TWS, int S, int NS>
struct Stages {
  static __device__ __forceinline__ void run(float2* lds, int tid, int T, const float2* tw) {
    if constexpr (S < Plan<N>::nst) {
      constexpr int R = Plan<N>::rad[S];
      stockham_stage<N, R, NS, DIR, E, B, LS, TWS>(lds, tid, T, tw);
      Stages<N, DIR, E, B, LS, TWS, S + 1, NS * R>::run(lds, tid, T, tw);
    }
  }
};

template <int N, int DIR, int E, int B, int LS, int TWS>
__device__ __forceinline__ void lds_fft(float2* lds, int tid, int T, const float2* tw) {
  Stages<N, DIR, E, B, LS, TWS, 0, 1>::run(lds, tid, T, tw);
}

// ------------------------------------------------------------------ column passes
// Columns per tile for the strided passes (128 B per element row when B = 16).
template <int N>
struct ColCfg {
  static constexpr int E = Plan<N>::E;
  static constexpr int B = (N * 16 * 8 <= 131072 && N * 16 / E <= 1024) ? 16 : 8;
  static constexpr int T = N * B / E;
};

// Strided pass: tile t covers columns [col0, col0 + B) of block t / tilesPerBlock,
// element j of column c at base + j * elemStride + c.
template <int N, int DIR, int KIND>
__global__ void __launch_bounds__(ColCfg<N>::T)
k_fft_col(float2* __restrict__ data, int64_t elemStride, int64_t tilesPerBlock,
          int64_t blockStride, const float2* __restrict__ tw, KOp op) {
  constexpr int B = ColCfg<N>::B, E = ColCfg<N>::E, T = ColCfg<N>::T;
  __shared__ float2 lds[N * B];
  const int tid = threadIdx.x;
  const int64_t tile = blockIdx.x;
  const int64_t colInBlock = (tile % tilesPerBlock) * B;
  const int64_t base = (tile / tilesPerBlock) * blockStride + colInBlock;
#pragma unroll 4
  for (int e = tid; e < N * B; e += T) {
    const int c = e % B, j = e / B;
    const int64_t idx = base + j * elemStride + c;
    float2 v;
    if constexpr (KIND == K_COPY) {
      v = (op.a ? op.a : data)[idx];
    } else {
      // X pass of an inverse transform: element j is nu_x, column (y, z)
      const int64_t col = colInBlock + c;
      v = kspace_eval<KIND>(op, j, (int)(col / op.pitch), (int)(col % op.pitch), idx);
    }
    lds[j * B + c] = v;
  }
  __syncthreads();
  lds_fft<N, DIR, E, B, B, 1>(lds, tid, T, tw);
#pragma unroll 4
  for (int e = tid; e < N * B; e += T) {
    const int c = e % B, j = e / B;
    data[base + j * elemStride + c] = lds[j * B + c];
  }
}

// ------------------------------------------------------------------ row passes
constexpr int pow2_floor(int x) { return x >= 2 ? 2 * pow2_floor(x / 2) : 1; }

template <int NC>
struct RowCfg {
  static constexpr int E = Plan<NC>::E;
  static constexpr int B0 = pow2_floor(2048 / NC);
  static constexpr int B = B0 < 1 ? 1 : (B0 > 64 ? 64 : B0);
  static constexpr int T = NC * B / E;
  static constexpr int LS = B + 1;   // odd LDS stride: transposed row loads stay conflict-light
};

// Forward Z pass: real rows of n = 2 NC floats (pitch 2*pitch floats) -> half-complex rows
// of NC + 1 values (pitch `pitch`).  Twiddles tw[t] = exp(-2 pi i t / n).
template <int NC>
__global__ void __launch_bounds__(RowCfg<NC>::T)
k_fft_r2c_row(const float* __restrict__ in, float2* __restrict__ out, int64_t nrows, int pitch,
              const float2* __restrict__ tw) {
  constexpr int B = RowCfg<NC>::B, E = RowCfg<NC>::E, T = RowCfg<NC>::T, LS = RowCfg<NC>::LS;
  __shared__ float2 lds[NC * LS];
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * B;
  for (int e = tid; e < NC * B; e += T) {
    const int c = e / NC, m = e % NC;
    float2 v = make_float2(0.f, 0.f);
    if (r0 + c < nrows) v = reinterpret_cast<const float2*>(in + (r0 + c) * (int64_t)(2 * pitch))[m];
    lds[m * LS + c] = v;
  }
  __syncthreads();
  lds_fft<NC, -1, E, B, LS, 2>(lds, tid, T, tw);
  // X_k = (Z_k + conj Z_{NC-k})/2 - (i/2) w^k (Z_k - conj Z_{NC-k}),  w = exp(-2 pi i / n)
  for (int e = tid; e < (NC + 1) * B; e += T) {
    const int c = e / (NC + 1), k = e % (NC + 1);
    if (r0 + c >= nrows) continue;
    const float2 zk = lds[(k == NC ? 0 : k) * LS + c];
    const float2 zc = cconj(lds[(k == 0 ? 0 : NC - k) * LS + c]);
    const float2 ev = make_float2(0.5f * (zk.x + zc.x), 0.5f * (zk.y + zc.y));
    const float2 od = make_float2(0.5f * (zk.x - zc.x), 0.5f * (zk.y - zc.y));
    const float2 w = (k == NC) ? make_float2(-1.f, 0.f) : tw[k];
    const float2 t = cmul(w, od);          // w^k (Z_k - conj Z_{NC-k}) / 2
    out[(r0 + c) * (int64_t)pitch + k] = make_float2(ev.x + t.y, ev.y - t.x);   // ev - i t
  }
}

// Inverse Z pass: half-complex rows (NC + 1 values) -> real rows of n = 2 NC floats,
// unnormalised.  Z_k = (X_k + conj X_{NC-k}) + i w^{-k} (X_k - conj X_{NC-k}),
// then z = IDFT_NC(Z) gives (x_even + i x_odd) * n/... (unnormalised length-n inverse).
template <int NC>
__global__ void __launch_bounds__(RowCfg<NC>::T)
k_fft_c2r_row(const float2* __restrict__ in, float* __restrict__ out, int64_t nrows, int pitch,
              const float2* __restrict__ tw) {
  constexpr int B = RowCfg<NC>::B, E = RowCfg<NC>::E, T = RowCfg<NC>::T, LS = RowCfg<NC>::LS;
  __shared__ float2 lds[NC * LS];
  __shared__ float2 xin[(NC + 1) * B];
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * B;
  for (int e = tid; e < (NC + 1) * B; e += T) {
    const int c = e / (NC + 1), k = e % (NC + 1);
    float2 v = make_float2(0.f, 0.f);
    if (r0 + c < nrows) v = in[(r0 + c) * (int64_t)pitch + k];
    xin[c * (NC + 1) + k] = v;
  }
  __syncthreads();
  for (int e = tid; e < NC * B; e += T) {
    const int c = e / NC, k = e % NC;
    const float2 xk = xin[c * (NC + 1) + k];
    const float2 xc = cconj(xin[c * (NC + 1) + NC - k]);
    const float2 s = cadd(xk, xc);
    const float2 d = csub(xk, xc);
    const float2 w = cconj(tw[k]);           // exp(+2 pi i k / n)
    const float2 t = cmul(w, d);
    lds[k * LS + c] = make_float2(s.x - t.y, s.y + t.x);   // s + i t
  }
  __syncthreads();
  lds_fft<NC, +1, E, B, LS, 2>(lds, tid, T, tw);
  for (int e = tid; e < NC * B; e += T) {
    const int c = e / NC, m = e % NC;
    if (r0 + c >= nrows) continue;
    reinterpret_cast<float2*>(out + (r0 + c) * (int64_t)(2 * pitch))[m] = lds[m * LS + c];
  }
}

// ------------------------------------------------------------------ dispatch
bool fft_size_supported(int n) {
  switch (n) {
    case 8: case 12: case 16: case 24: case 32: case 48: case 64: case 96: case 128:
    case 192: case 256: case 384: case 512: case 768: case 1024: case 1536: case 2048:
      return true;
    default:
      return false;
  }
}

template <int N, int DIR, int KIND>
static void col_pass(float2* data, int64_t elemStride, int64_t tiles, int64_t tilesPerBlock,
                     int64_t blockStride, const float2* tw, const KOp& op, hipStream_t s,
                     const char* name) {
  ProfScope ps(name, s);
  hipLaunchKernelGGL((k_fft_col<N, DIR, KIND>), dim3((unsigned)tiles), dim3(ColCfg<N>::T), 0, s,
                     data, elemStride, tilesPerBlock, blockStride, tw, op);
  COLA_LAUNCH_CHECK();
}

template <int N>
static void r2c_impl(const FFTPlan& pl, const float* in, float2* out, hipStream_t s) {
  const int n = pl.n, P = pl.pitch;
  const int64_t rows = (int64_t)n * n;
  {
    ProfScope ps("fft_r2c_z", s);
    constexpr int B = RowCfg<N / 2>::B;
    hipLaunchKernelGGL((k_fft_r2c_row<N / 2>), dim3((unsigned)((rows + B - 1) / B)),
                       dim3(RowCfg<N / 2>::T), 0, s, in, out, rows, P, pl.tw);
    COLA_LAUNCH_CHECK();
  }
  KOp op;
  constexpr int B = ColCfg<N>::B;
  // Y pass: per x-plane, tiles of B z-columns, element stride = pitch
  col_pass<N, -1, K_COPY>(out, P, (int64_t)n * (P / B), P / B, (int64_t)n * P, pl.tw, op, s,
                          "fft_y_fwd");
  // X pass: tiles of B (y, z) columns, element stride = n * pitch
  col_pass<N, -1, K_COPY>(out, (int64_t)n * P, (int64_t)n * P / B, (int64_t)n * P / B, 0, pl.tw, op,
                          s, "fft_x_fwd");
}

template <int N>
static void c2r_impl(const FFTPlan& pl, int kind, const KOp& op_in, float2* data, float* out,
                     hipStream_t s) {
  const int n = pl.n, P = pl.pitch;
  const int64_t rows = (int64_t)n * n;
  constexpr int B = ColCfg<N>::B;
  KOp op = op_in;
  op.n = n;
  op.pitch = P;
  const int64_t xtiles = (int64_t)n * P / B;
  switch (kind) {
    case K_COPY: col_pass<N, 1, K_COPY>(data, (int64_t)n * P, xtiles, xtiles, 0, pl.tw, op, s, "fft_x_inv"); break;
    case K_FORCE: col_pass<N, 1, K_FORCE>(data, (int64_t)n * P, xtiles, xtiles, 0, pl.tw, op, s, "fft_x_inv_force"); break;
    case K_POT: col_pass<N, 1, K_POT>(data, (int64_t)n * P, xtiles, xtiles, 0, pl.tw, op, s, "fft_x_inv_pot"); break;
    case K_SMOOTH: col_pass<N, 1, K_SMOOTH>(data, (int64_t)n * P, xtiles, xtiles, 0, pl.tw, op, s, "fft_x_inv_smooth"); break;
    case K_LPT: col_pass<N, 1, K_LPT>(data, (int64_t)n * P, xtiles, xtiles, 0, pl.tw, op, s, "fft_x_inv_lpt"); break;
    case K_HESS: col_pass<N, 1, K_HESS>(data, (int64_t)n * P, xtiles, xtiles, 0, pl.tw, op, s, "fft_x_inv_hess"); break;
    case K_GRAD: col_pass<N, 1, K_GRAD>(data, (int64_t)n * P, xtiles, xtiles, 0, pl.tw, op, s, "fft_x_inv_grad"); break;
    default: throw Error{COLA_E_ARG, "unknown k-space operator"};
  }
  KOp none;
  col_pass<N, 1, K_COPY>(data, P, (int64_t)n * (P / B), P / B, (int64_t)n * P, pl.tw, none, s,
                         "fft_y_inv");
  {
    ProfScope ps("fft_c2r_z", s);
    constexpr int BR = RowCfg<N / 2>::B;
    hipLaunchKernelGGL((k_fft_c2r_row<N / 2>), dim3((unsigned)((rows + BR - 1) / BR)),
                       dim3(RowCfg<N / 2>::T), 0, s, data, out, rows, P, pl.tw);
    COLA_LAUNCH_CHECK();
  }
}

void fft_r2c(const FFTPlan& pl, const float* in, float2* out, hipStream_t s) {
  switch (pl.n) {
#define CASE(N_) case N_: r2c_impl<N_>(pl, in, out, s); return;
    CASE(8) CASE(12) CASE(16) CASE(24) CASE(32) CASE(48) CASE(64) CASE(96) CASE(128)
    CASE(192) CASE(256) CASE(384) CASE(512) CASE(768) CASE(1024) CASE(1536) CASE(2048)
#undef CASE
    default: throw Error{COLA_E_UNSUPPORTED, "FFT size not supported"};
  }
}

void fft_c2r(const FFTPlan& pl, int kind, const KOp& op, float2* data, float* out, hipStream_t s) {
  switch (pl.n) {
#define CASE(N_) case N_: c2r_impl<N_>(pl, kind, op, data, out, s); return;
    CASE(8) CASE(12) CASE(16) CASE(24) CASE(32) CASE(48) CASE(64) CASE(96) CASE(128)
    CASE(192) CASE(256) CASE(384) CASE(512) CASE(768) CASE(1024) CASE(1536) CASE(2048)
#undef CASE
    default: throw Error{COLA_E_UNSUPPORTED, "FFT size not supported"};
  }
}

}  // namespace cola
