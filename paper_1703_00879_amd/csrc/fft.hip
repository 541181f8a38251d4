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

#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <type_traits>

#include "internal.h"
#include "kspace.h"

namespace cola {

// Element offsets: 32-bit while a whole mesh of n^3 half-complex values (with padding)
// stays below 2^32 elements (n <= 1536), so addresses are one register plus a scalar base.
template <int N>
using Off = typename std::conditional<(N <= 1536), uint32_t, uint64_t>::type;

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

// Streaming loads and stores that bypass cache retention (nontemporal): for passes whose
// every element is touched once, so that what the caches hold is the pass's own spill and
// twiddle traffic rather than data that will not be read again.
typedef float nfloat2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 load_stream(const float2* p) {
  const nfloat2 v = __builtin_nontemporal_load(reinterpret_cast<const nfloat2*>(p));
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ void store_stream(float2* p, float2 v) {
  nfloat2 w;
  w.x = v.x;
  w.y = v.y;
  __builtin_nontemporal_store(w, reinterpret_cast<nfloat2*>(p));
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
COLA_PLAN(2048, 32, 4, 8, 8, 8, 4)   // 32 per thread: 512 threads per 8-column tile
// Plans of the row passes: the column plans, except that the lengths with a factor 3 take
// radices 4, 2 and 3 only, so that 12 elements per thread divide by every radix instead of
// 24 (a row pass holds its next block's rows in registers besides the butterflies).
template <int N>
struct RowPlan : Plan<N> {};
#define COLA_ROW_PLAN(N_, E_, NST_, ...)                          \
  template <>                                                     \
  struct RowPlan<N_> {                                            \
    static constexpr int E = E_;                                  \
    static constexpr int nst = NST_;                              \
    static constexpr int rad[NST_] = {__VA_ARGS__};               \
  };
COLA_ROW_PLAN(24, 12, 3, 4, 2, 3)
COLA_ROW_PLAN(48, 12, 3, 4, 4, 3)
COLA_ROW_PLAN(96, 12, 4, 4, 4, 2, 3)
COLA_ROW_PLAN(192, 12, 4, 4, 4, 4, 3)
COLA_ROW_PLAN(384, 12, 5, 4, 4, 4, 2, 3)
COLA_ROW_PLAN(768, 12, 5, 4, 4, 4, 4, 3)
#undef COLA_ROW_PLAN
#undef COLA_PLAN
// First and last radix equal: a transform's last stage can hand its outputs to the next
// transform's first stage in registers (kStoreIR).
template <int N>
constexpr bool kHandOff = Plan<N>::rad[0] == Plan<N>::rad[Plan<N>::nst - 1];

// Twiddle of operand r of butterfly k in the Stockham stage with NS = product of the
// earlier radices.  TWS > 0: from the full table, tw[t * TWS] = exp(-2 pi i t / N) (the
// column passes, whose lanes share few k).  TWS == 0: from a per-stage table, entry
// (NS - 1) + k (R - 1) + (r - 1) (built by fill_stage_twiddles), so that the lanes of a
// row pass, which take consecutive k, read consecutive LDS words instead of words a
// multiple of the bank count apart.  Both hold the same values.
template <int N, int R, int NS, int TWS>
__device__ __forceinline__ float2 stage_twiddle(const float2* __restrict__ tw, int k, int r) {
  if constexpr (TWS == 0)
    return tw[(NS - 1) + k * (R - 1) + (r - 1)];
  else
    return tw[(r * k * (N / (NS * R))) * TWS];
}

// Per-stage twiddle table of the N-point plan (N - 1 entries, stage after stage, the
// entries of a stage ordered by butterfly k then operand r) from the full table of a
// transform of length N * S (src[t] = exp(-2 pi i t / (N S))).
template <int N, class P = Plan<N>>
__device__ __forceinline__ void fill_stage_twiddles(float2* tw, const float2* __restrict__ src,
                                                    int S, int tid, int T) {
  for (int e = tid; e < N - 1; e += T) {
    int rest = e, ns = 1, t = 0;
#pragma unroll
    for (int st = 0; st < P::nst; ++st) {
      const int R = P::rad[st];
      const int cnt = ns * (R - 1);
      if (rest >= 0 && rest < cnt) t = (rest % (R - 1) + 1) * (rest / (R - 1)) * (N / (ns * R));
      rest -= cnt;
      ns *= R;
    }
    tw[e] = src[t * S];
  }
}

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
        float2 w = stage_twiddle<N, R, NS, TWS>(tw, k, r);
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

template <int N, int DIR, int E, int B, int LS, int TWS, int S, int NS, class P>
struct Stages {
  static __device__ __forceinline__ void run(float2* lds, int tid, int T, const float2* tw) {
    if constexpr (S < P::nst) {
      constexpr int R = P::rad[S];
      stockham_stage<N, R, NS, DIR, E, B, LS, TWS>(lds, tid, T, tw);
      Stages<N, DIR, E, B, LS, TWS, S + 1, NS * R, P>::run(lds, tid, T, tw);
    }
  }
};

template <int N, int DIR, int E, int B, int LS, int TWS, class P = Plan<N>>
__device__ __forceinline__ void lds_fft(float2* lds, int tid, int T, const float2* tw) {
  Stages<N, DIR, E, B, LS, TWS, 0, 1, P>::run(lds, tid, T, tw);
}

// Stockham transform of B columns whose first stage reads its operands through
// `load(i, r, j, c)` (operand r of the thread's butterfly i, element j of column c) and
// whose last stage writes through `store(j, c, v)`; only the middle stages go through LDS.
// Each thread issues all of its E loads before it uses any of them, so a work-group keeps
// its whole tile in flight.  FL says whether `load` reads the LDS tile (kFirstFromLds) or
// `store` writes it (kLastToLds), so that the stage in question separates its reads from
// its in-place writes by a barrier; after a kLastToLds transform the caller must
// synchronise before reading the tile.
constexpr int kFirstFromLds = 1, kLastToLds = 2;
// kStoreIR: the last stage calls store(j, c, v, i, r), naming the butterfly i and operand r
// that produced the value.  The last stage's (i, r) -> element map equals the first
// stage's when both have the same radix, so a following transform can take its first
// operands from registers filled by this store.
constexpr int kStoreIR = 4;

template <int N, int DIR, int E, int B, int LS, int TWS, int S, int NS, int FL = 0,
          class P = Plan<N>>
struct GStages {
  template <class Load, class Store>
  static __device__ __forceinline__ void run(float2* lds, int tid, int T, const float2* tw,
                                             Load& load, Store& store) {
    constexpr int nst = P::nst;
    if constexpr (S < nst) {
      constexpr int R = P::rad[S];
      constexpr int NB = E / R;
      float2 v[NB][R];
      constexpr bool reads_lds = S > 0 || (FL & kFirstFromLds);
      constexpr bool writes_lds = S + 1 < nst || (FL & kLastToLds);
      if constexpr (S == 0) {
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          const int b = tid + i * T;
          const int c = b % B, j = b / B;
#pragma unroll
          for (int r = 0; r < R; ++r) v[i][r] = load(i, r, j + r * (N / R), c);
        }
      } else {
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          const int b = tid + i * T;
          const int c = b % B, j = b / B;
#pragma unroll
          for (int r = 0; r < R; ++r) v[i][r] = lds[(j + r * (N / R)) * LS + c];
        }
      }
      if constexpr (reads_lds && writes_lds) __syncthreads();   // all reads before the in-place writes
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        const int b = tid + i * T;
        const int c = b % B, j = b / B;
        const int k = j % NS;
        if (NS > 1) {
#pragma unroll
          for (int r = 1; r < R; ++r) {
            float2 w = stage_twiddle<N, R, NS, TWS>(tw, k, r);
            if (DIR > 0) w.y = -w.y;
            v[i][r] = cmul(v[i][r], w);
          }
        }
        Dft<R, DIR>::run(v[i]);
        const int idxD = (j / NS) * NS * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if constexpr (S + 1 == nst) {
            if constexpr ((FL & kStoreIR) != 0)
              store(idxD + r * NS, c, v[i][r], i, r);
            else
              store(idxD + r * NS, c, v[i][r]);
          } else {
            lds[(idxD + r * NS) * LS + c] = v[i][r];
          }
        }
      }
      if constexpr (S + 1 < nst) {
        __syncthreads();
        GStages<N, DIR, E, B, LS, TWS, S + 1, NS * R, FL, P>::run(lds, tid, T, tw, load, store);
      }
    }
  }
};

// ------------------------------------------------------------------ column passes
// Columns per tile for the strided passes: as many as a 128 KB LDS tile holds, up to 16
// (a 128-byte row segment per element, so every load and store moves whole cache lines),
// one work-group per CU with the plan's own elements per thread; 1536- and 2048-point
// columns go 8 to a tile (64-byte row segments).
template <int N>
struct ColCfg {
  static constexpr int E = Plan<N>::E;
  static constexpr int B0 = 131072 / (8 * N);
  static constexpr int B = B0 >= 16 ? 16 : (B0 >= 8 ? 8 : 4);
  static constexpr int T = N * B / E;
  static_assert(T <= 1024, "column tile needs too many threads");
};

// Strided pass: tile t covers columns [col0, col0 + B) of block t / tilesPerBlock, element
// j of column c at base + j * elemStride + c.  The twiddles are staged in LDS so that no
// butterfly stage waits on the global-load queue.
// Columns per tile of the X passes (element stride one x-plane): these run faster with
// more work-groups per CU, so 512- and 1024-point columns go 8 to a tile (two or four
// work-groups per CU) where the Y passes take 16.
template <int N>
struct XCfg {
  static constexpr int B = (N == 512 || N == 1024) ? 8 : ColCfg<N>::B;
};

template <int N, int DIR, int KIND, int BB = ColCfg<N>::B>
__global__ void __launch_bounds__(N * BB / ColCfg<N>::E)
k_fft_col(float2* __restrict__ data, int64_t elemStride, int64_t tilesPerBlock,
          int64_t blockStride, int64_t ntiles, const float2* __restrict__ tw_g, KOp op) {
  constexpr int B = BB, E = ColCfg<N>::E, T = N * BB / E;
  __shared__ float2 lds[N * B];
  __shared__ float2 tw[N];
  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += T) tw[i] = tw_g[i];   // first read after stage 0's barrier
  using O = Off<N>;
  const unsigned tile = xcd_block(blockIdx.x, gridDim.x);   // neighbouring tiles share an L2
  const unsigned tpb = (unsigned)tilesPerBlock;
  const O colInBlock = (O)(tile % tpb) * B;
  const O base = (O)(tile / tpb) * (O)blockStride + colInBlock;
  const O es = (O)elemStride;
  const float2* src = (KIND == K_COPY && op.a) ? op.a : data;
  static_assert(T % B == 0, "a thread's butterflies must share one column");
  // X pass of an inverse transform: element j is nu_x; the thread's (y, z) column
  const int col = (int)colInBlock + tid % B;
  const int iy = KIND == K_COPY ? 0 : col / op.pitch, iz = KIND == K_COPY ? 0 : col % op.pitch;
  auto load = [&](int, int, int j, int c) -> float2 {
    const O idx = base + (O)j * es + c;
    if constexpr (KIND == K_COPY)
      return src[idx];
    else
      return kspace_eval<KIND>(op, j, iy, iz, idx);
  };
  auto store = [&](int j, int c, float2 v) { data[base + (O)j * es + c] = v; };
  GStages<N, DIR, E, B, B, 1, 0, 1>::run(lds, tid, T, tw, load, store);
}

// X pass of a forward transform fused with the X pass of the inverse transform through a
// k-space operator: the forward result (delta_k), multiplied by the operator (smoothing
// window or Newtonian potential), is transformed back through the same LDS tile into
// `out`, and with KEEP also written back in place.  One read and one or two writes of the
// field instead of two reads and two writes.
// Tile of the forward-operator-inverse X pass: the X-pass tile (for 1024-point columns 8
// to a 64 KB tile, two work-groups per CU, 25 % faster than one 16-column tile per CU).
// Elements per thread of the fused kernels that keep a column (or the Green's function)
// in registers across two transforms of a tile.  With 16 elements a 2048-point tile of 8
// columns needs 1024 threads, whose 128-register budget per lane spilled 150-180 bytes per
// lane to scratch memory (through the L2 to HBM); 32 elements per thread on 512 threads
// get 256 registers and spill 0-64 bytes, and measured 12-30 % faster (the 2048-point plan
// now takes 32 for every column pass; the plain Y passes gained 2.5 %).  At 1024 points
// the larger E spilled more and ran slower, so there the plan's E stays.  Each butterfly
// is computed the same way whatever E is.
template <int N, int B>
struct FusedCfg {
  static constexpr int E = (N >= 2048 && N * B / ColCfg<N>::E >= 1024) ? 2 * ColCfg<N>::E
                                                                      : ColCfg<N>::E;
  static constexpr int T = N * B / E;
};

template <int N>
struct OpCfg {
  static constexpr int B = XCfg<N>::B;
  static constexpr int E = FusedCfg<N, B>::E;
  static constexpr int T = FusedCfg<N, B>::T;
};

template <int N, int KIND, bool KEEP>
__global__ void __launch_bounds__(OpCfg<N>::T)
k_fft_col_fwd_op(float2* __restrict__ data, float2* __restrict__ out, int64_t elemStride,
                 const float2* __restrict__ tw_g, KOp op) {
  constexpr int B = OpCfg<N>::B, E = OpCfg<N>::E, T = OpCfg<N>::T;
  if (op.steps) op.g_n = op.steps[*op.step_ctr].sop_g_n;
  static_assert(T % B == 0, "a thread's butterflies must share one column");
  __shared__ float2 lds[N * B];
  __shared__ float2 tw[N];
  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += T) tw[i] = tw_g[i];
  using O = Off<N>;
  const O base = (O)xcd_block(blockIdx.x, gridDim.x) * B, es = (O)elemStride;
  const int col = (int)base + tid % B;   // (y, z) column of every element this thread touches
  const int iy = col / op.pitch, iz = col % op.pitch;
  auto load = [&](int, int, int j, int c) -> float2 { return data[base + (O)j * es + c]; };
  auto store2 = [&](int j, int c, float2 v) { out[base + (O)j * es + c] = v; };
  if constexpr (kHandOff<N>) {
    // the operator is applied in the forward transform's last stage and the inverse
    // starts from those registers
    constexpr int R0 = Plan<N>::rad[0], NB0 = E / R0;
    float2 hv[NB0][R0];
    auto store = [&](int j, int c, float2 v, int i, int r) {
      if (KEEP) data[base + (O)j * es + c] = v;
      hv[i][r] = kspace_apply<KIND>(op, j, iy, iz, v, v);
    };
    GStages<N, -1, E, B, B, 1, 0, 1, kStoreIR>::run(lds, tid, T, tw, load, store);
    __syncthreads();   // every thread has read its last operands out of the tile
    auto load2 = [&](int i, int r, int, int) -> float2 { return hv[i][r]; };
    GStages<N, +1, E, B, B, 1, 0, 1>::run(lds, tid, T, tw, load2, store2);
  } else {
    auto store = [&](int j, int c, float2 v) {
      if (KEEP) data[base + (O)j * es + c] = v;
      lds[j * B + c] = kspace_apply<KIND>(op, j, iy, iz, v, v);
    };
    GStages<N, -1, E, B, B, 1, 0, 1, kLastToLds>::run(lds, tid, T, tw, load, store);
    __syncthreads();
    auto load2 = [&](int, int, int j, int c) -> float2 { return lds[j * B + c]; };
    GStages<N, +1, E, B, B, 1, 0, 1, kFirstFromLds>::run(lds, tid, T, tw, load2, store2);
  }
}

// X pass of the forward transform of the (screened) source fused with the X passes of the
// inverse force transforms.  The forward X transform of `src` gives S_k in the LDS tile;
// the Green's function g = [g_n/k^2 delta_k + g_5/(k^2 + a^2 m^2) S_k] / M is formed once
// per element (delta_k read from dk, or S_k itself when dk is null) and kept in registers.
// F_c = IFFT[-i k_c g]: along an X column k_y and k_z are constants, so they commute with
// the X transform and only two X transforms are needed, G0 = X^-1[-i k_x g] into o0 and
// G = X^-1[g] into o1; the Y pass forms the y and z components from G.  The outputs may
// alias dk and src: every read of a column precedes the first write to it.  The column
// data is touched once, so it streams past the caches and leaves the L2 to the register
// spills of the two inverse transforms.
template <int N, bool DK>
__global__ void __launch_bounds__((FusedCfg<N, ColCfg<N>::B>::T))
k_fft_col_fwd_force(const float2* dk, const float2* src, float2* o0, float2* o1,
                    int64_t elemStride, const float2* __restrict__ tw_g, KOp op) {
  constexpr int B = ColCfg<N>::B, E = FusedCfg<N, B>::E, T = FusedCfg<N, B>::T;
  if (op.steps) {
    const StepDev& sd = op.steps[*op.step_ctr];
    op.g_n = op.step_newton ? sd.cn : sd.g_n;
    op.g_5 = op.step_newton ? 0.f : sd.g_5;
    op.a2m2 = op.step_newton ? 0.f : sd.a2m2;
  }
  constexpr int R0 = Plan<N>::rad[0], NB0 = E / R0;
  static_assert(T % B == 0, "a thread's butterflies must share one column");
  __shared__ float2 lds[N * B];
  __shared__ float2 tw[N];
  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += T) tw[i] = tw_g[i];
  using O = Off<N>;
  const O base = (O)xcd_block(blockIdx.x, gridDim.x) * B, es = (O)elemStride;   // X pass
  const int c0 = tid % B;
  const int col = (int)base + c0;
  const int iy = col / op.pitch, iz = col % op.pitch;
  float2 g[NB0][R0];
  if constexpr (DK) {
    // delta_k of the thread's elements, loaded with S's (same element map as the first
    // stage) so that both reads are in flight together; g takes them until the Green's
    // function replaces them
#pragma unroll
    for (int i = 0; i < NB0; ++i) {
      const int j = (tid + i * T) / B;
#pragma unroll
      for (int r = 0; r < R0; ++r) g[i][r] = load_stream(dk + base + (O)(j + r * (N / R0)) * es + c0);
    }
  }
  auto load = [&](int, int, int j, int c) -> float2 { return load_stream(src + base + (O)j * es + c); };
  if constexpr (!DK && kHandOff<N>) {
    // one source: g is formed in the forward transform's last stage, in registers
    auto store = [&](int jj, int, float2 v, int i, int r) { g[i][r] = green_force(op, jj, iy, iz, v, v); };
    GStages<N, -1, E, B, B, 1, 0, 1, kStoreIR>::run(lds, tid, T, tw, load, store);
  } else {
    auto store = [&](int j, int c, float2 v) { lds[j * B + c] = v; };
    GStages<N, -1, E, B, B, 1, 0, 1, kLastToLds>::run(lds, tid, T, tw, load, store);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NB0; ++i) {
      const int j = (tid + i * T) / B;
#pragma unroll
      for (int r = 0; r < R0; ++r) {
        const int jj = j + r * (N / R0);
        const float2 sv = lds[jj * B + c0];
        const float2 dv = DK ? g[i][r] : sv;
        g[i][r] = green_force(op, jj, iy, iz, dv, sv);
      }
    }
  }
  __syncthreads();   // the tile is reused by the inverse transforms
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    float2* out = t == 0 ? o0 : o1;
    auto load = [&](int i, int r, int jj, int) -> float2 {
      return t == 0 ? grad_minus_i(op, jj, iy, iz, 0, g[i][r]) : g[i][r];
    };
    auto store = [&](int j, int c, float2 v) { store_stream(out + base + (O)j * es + c, v); };
    GStages<N, +1, E, B, B, 1, 0, 1>::run(lds, tid, T, tw, load, store);
    __syncthreads();   // the second transform reuses the LDS tile
  }
}

// Inverse Y pass of G = X^-1[g] giving two force components at once: F_y needs the Y
// transform of -i k_y G (k_y varies along the column) and F_z = -i k_z Y^-1[G] (k_z is
// the column's constant).  The column is loaded once and kept in registers for both
// transforms; outA (F_y, may alias data) and outB (F_z) take the results.  Tile t covers
// columns [col0, col0 + B) of x-plane t / tilesPerBlock, as in k_fft_col.
template <int N>
__global__ void __launch_bounds__((FusedCfg<N, ColCfg<N>::B>::T))
k_fft_col_inv_yz(const float2* data, float2* outA, float2* __restrict__ outB, int64_t elemStride,
                 int64_t tilesPerBlock, int64_t blockStride, const float2* __restrict__ tw_g,
                 KOp op) {
  constexpr int B = ColCfg<N>::B, E = FusedCfg<N, B>::E, T = FusedCfg<N, B>::T;
  constexpr int R0 = Plan<N>::rad[0], NB0 = E / R0;
  static_assert(T % B == 0, "a thread's butterflies must share one column");
  __shared__ float2 lds[N * B];
  __shared__ float2 tw[N];
  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += T) tw[i] = tw_g[i];
  using O = Off<N>;
  const unsigned tile = xcd_block(blockIdx.x, gridDim.x);
  const unsigned tpb = (unsigned)tilesPerBlock;
  const O colInBlock = (O)(tile % tpb) * B;
  const O base = (O)(tile / tpb) * (O)blockStride + colInBlock;
  const O es = (O)elemStride;
  const int c0 = tid % B;
  const int iz = (int)colInBlock + c0;   // Y pass: the column is z
  float2 gv[NB0][R0];
#pragma unroll
  for (int i = 0; i < NB0; ++i) {
    const int j = (tid + i * T) / B;
#pragma unroll
    for (int r = 0; r < R0; ++r) gv[i][r] = data[base + (O)(j + r * (N / R0)) * es + c0];
  }
  {
    auto load = [&](int i, int r, int jj, int) -> float2 {
      return grad_minus_i(op, 0, jj, iz, 1, gv[i][r]);
    };
    auto store = [&](int j, int c, float2 v) { outA[base + (O)j * es + c] = v; };
    GStages<N, +1, E, B, B, 1, 0, 1>::run(lds, tid, T, tw, load, store);
  }
  __syncthreads();   // the second transform reuses the LDS tile
  {
    auto load = [&](int i, int r, int, int) -> float2 { return gv[i][r]; };
    auto store = [&](int j, int c, float2 v) {
      outB[base + (O)j * es + c] = grad_minus_i(op, 0, j, iz, 2, v);
    };
    GStages<N, +1, E, B, B, 1, 0, 1>::run(lds, tid, T, tw, load, store);
  }
}

// Inverse X pass of a scale-dependent LPT term (App. A): the displacement-like field
// IDFT[i k (c1 phi1_k + c2 phi2_k)], c1 and c2 the step's FP32 growth coefficients of
// |nu|^2 (one 8-byte table read per mode).  A = -(c1 phi1_k + c2 phi2_k) / N is formed in
// registers from one read of each potential, and two X transforms go out through the LDS
// tile, as in k_fft_col_fwd_force: G0 = X^-1[-i k_x A] (= X^-1[i k_x (c1 phi1 + c2 phi2)]/N)
// into o0 and G = X^-1[A] into o1, from which the Y passes of the force transforms give
// the three components.  Columns past z = n/2 (row padding) get zeros.
template <int N>
struct LptXCfg {
  static constexpr int B = XCfg<N>::B;
  static constexpr int E = FusedCfg<N, B>::E;
  static constexpr int T = FusedCfg<N, B>::T;
};

// At 1024 points two work-groups (72 KB of LDS each) share a CU when the kernel keeps to
// 128 registers (it needs about 134 left to itself): 5 % faster.
template <int N>
__global__ void __launch_bounds__(LptXCfg<N>::T)
__attribute__((amdgpu_waves_per_eu(N == 1024 ? 4 : 1)))
k_fft_col_lpt(const float2* __restrict__ phi1, const float2* __restrict__ phi2,
              float2* __restrict__ o0, float2* __restrict__ o1, int64_t elemStride,
              const float2* __restrict__ tw_g, KOp op) {
  constexpr int B = LptXCfg<N>::B, E = LptXCfg<N>::E, T = LptXCfg<N>::T;
  constexpr int R0 = Plan<N>::rad[0], NB0 = E / R0;
  static_assert(T % B == 0, "a thread's butterflies must share one column");
  __shared__ float2 lds[N * B];
  __shared__ float2 tw[N];
  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += T) tw[i] = tw_g[i];   // first read after stage 0's barrier
  using O = Off<N>;
  const O base = (O)xcd_block(blockIdx.x, gridDim.x) * B, es = (O)elemStride;
  const int c0 = tid % B;
  const int col = (int)base + c0;
  const int iy = col / op.pitch, iz = col % op.pitch;
  const int n = op.n, h = n >> 1;
  const int ny = iy < h ? iy : iy - n;
  const int n2yz = ny * ny + iz * iz;
  const float ms = -op.scale;
  float2 g[NB0][R0];
#pragma unroll
  for (int i = 0; i < NB0; ++i) {
    const int j = (tid + i * T) / B;
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      const int jj = j + r * (N / R0);
      const O idx = base + (O)jj * es + c0;
      const float2 a = load_stream(phi1 + idx), b = load_stream(phi2 + idx);
      const int nx = jj < h ? jj : jj - n;
      const int n2 = nx * nx + n2yz;
      g[i][r] = make_float2(0.f, 0.f);
      if (iz <= h && n2 != 0) {
        const float2 cf = op.coef[n2];
        g[i][r] = make_float2(ms * (cf.x * a.x + cf.y * b.x), ms * (cf.x * a.y + cf.y * b.y));
      }
    }
  }
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    float2* out = t == 0 ? o0 : o1;
    auto load = [&](int i, int r, int jj, int) -> float2 {
      return t == 0 ? grad_minus_i(op, jj, iy, iz, 0, g[i][r]) : g[i][r];
    };
    auto store = [&](int j, int c, float2 v) { store_stream(out + base + (O)j * es + c, v); };
    GStages<N, +1, E, B, B, 1, 0, 1>::run(lds, tid, T, tw, load, store);
    __syncthreads();   // the second transform reuses the LDS tile
  }
}

// ------------------------------------------------------------------ row passes
constexpr int pow2_floor(int x) { return x >= 2 ? 2 * pow2_floor(x / 2) : 1; }

// Rows of 1024 complex values (2048-point real rows) take 8 elements per thread, half the
// plan's 16: twice the threads per row tile, which measured 10-35 % faster row passes.
template <int NC>
constexpr int kRowE = NC == 1024 ? 8 : RowPlan<NC>::E;

// Row block blk of a row pass: rows r0 = blk B .. r0 + B - 1 of a mesh of nrows rows, kN
// to a plane, `pitch` elements apart within a plane and `plane` elements apart between
// planes.  The row count is whole planes (nrows = kN x planes), so when B divides kN a
// block is complete and lies within one plane: a row's offset is one multiply-add from
// the block's, with no division and no bounds test per element.
template <int kN, int B, class O>
struct RowBlock {
  O r0, base;
  int64_t nrows, plane;
  int pitch;
  __device__ __forceinline__ RowBlock(int64_t blk, int64_t nrows_, int pitch_, int64_t plane_)
      : r0((O)blk * B), nrows(nrows_), plane(plane_), pitch(pitch_) {
    base = (r0 / kN) * (O)plane + (r0 % kN) * (O)pitch;
  }
  __device__ __forceinline__ bool valid(int c) const {
    if constexpr (kN % B == 0)
      return true;
    else
      return r0 + c < (O)nrows;
  }
  __device__ __forceinline__ O off(int c) const {
    if constexpr (kN % B == 0) {
      return base + (O)(c * pitch);
    } else {
      const O r = r0 + c;
      return (r / kN) * (O)plane + (r % kN) * (O)pitch;
    }
  }
};

// LDS twiddles of a row pass (rows of n = 2 NC reals): tw[k] = exp(-2 pi i k / n) for the
// split steps, k < NC, then the per-stage table of the NC-point transform at tw + NC.
template <int NC>
__device__ __forceinline__ void row_twiddles(float2* tw, const float2* __restrict__ tw_g, int tid,
                                             int T) {
  for (int i = tid; i < NC; i += T) tw[i] = tw_g[i];
  fill_stage_twiddles<NC, RowPlan<NC>>(tw + NC, tw_g, 2, tid, T);
}

// Row-pass tiles: rows of 1024 complex values go one to a work-group with an unpadded
// tile (a single row has no transposed accesses to pad against), shorter rows as many as
// fill 32 KB with a padded stride.  The row kernels loop over row blocks and load the next
// block's rows while transforming the current ones; kPersist says whether they run as a
// persistent grid (as many work-groups as fit the device at once) or one work-group per
// block.  At 1024 the persistent one-row form measured 2-45 % faster, depending on the
// pass, than four-row tiles one work-group per block, and the persistent grid took
// 7-20 % off the multi-row passes of 96-384-point rows (the ensemble and serving
// meshes); at 512 the multi-row tiles one work-group per block were the faster ones.
template <int NC>
struct RowCfg {
  static constexpr int E = kRowE<NC>;
  static constexpr int B0 = pow2_floor(4096 / NC);
  static constexpr int B = NC >= 1024 ? 1 : (B0 < 1 ? 1 : (B0 > 64 ? 64 : B0));
  static constexpr bool kPersist = NC != 512;
  static constexpr int T = NC * B / E;
  // odd LDS stride: transposed row loads stay conflict-light; one row needs no padding
  static constexpr int LS = B == 1 ? 1 : B + 1;
};

// Split step of an inverse real transform: B rows of NC + 1 half-complex values X_k give
//   Z_k = (X_k + conj X_{NC-k}) + i exp(+2 pi i k / n) (X_k - conj X_{NC-k}),  k < NC,
// the input of the NC-point inverse transform of (x_even + i x_odd), at tile[k * LS + c].
// Each of TT threads holds NP pairs (X_k, X_{NC-k}), 1 <= k < NC/2, read straight from the
// rows: every value is loaded once and both Z_k and Z_{NC-k} follow from the pair, so the
// tile needs no mirror exchange.  The pair k = 0 is (X_0, X_NC) together with the
// self-mirrored X_{NC/2}.  load() issues the reads (row(c) gives row c, or null past the
// last row); store() needs the twiddles exp(-2 pi i t / n) in LDS.
template <int NC, int NP>
struct InvSplit {
  static constexpr int H = NC / 2;
  float2 xa[NP], xb[NP], xm[NP];
  template <class Row>
  __device__ __forceinline__ void load(int t, int TT, const Row& row) {
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const int e = t + i * TT, c = e / H, k = e % H;
      xa[i] = xb[i] = xm[i] = make_float2(0.f, 0.f);
      const float2* rp = row(c);
      if (rp) {
        xa[i] = rp[k];
        xb[i] = rp[k == 0 ? NC : NC - k];
        if (k == 0) xm[i] = rp[H];
      }
    }
  }
  __device__ __forceinline__ void store(int t, int TT, const float2* tw, float2* tile, int LS) const {
    auto z = [&](float2 xk, float2 xc, int k) {   // xc = conj X_{NC-k}
      const float2 sm = cadd(xk, xc);
      const float2 d = csub(xk, xc);
      const float2 u = cmul(cconj(tw[k]), d);   // exp(+2 pi i k / n) d
      return make_float2(sm.x - u.y, sm.y + u.x);   // sm + i u
    };
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const int e = t + i * TT, c = e / H, k = e % H;
      tile[k * LS + c] = z(xa[i], cconj(xb[i]), k);
      if (k == 0)
        tile[H * LS + c] = z(xm[i], cconj(xm[i]), H);
      else
        tile[(NC - k) * LS + c] = z(xb[i], cconj(xa[i]), NC - k);
    }
  }
};

// Split step of a forward real transform: B rows held in LDS as Z (the NC-point transform
// of x_even + i x_odd, lds[k * LS + c]) give the NC + 1 half-complex values
//   X_k = (Z_k + conj Z_{NC-k})/2 - (i/2) w^k (Z_k - conj Z_{NC-k}),  w = exp(-2 pi i / n),
// handed to store(c, k, X_k).  Thread tid takes elements tid + i T (E T = NC B) and the
// Nyquist value X_NC of row tid < B.
template <int NC, int E, int B, int LS, int T, class Store>
__device__ __forceinline__ void split_fwd_store(const float2* lds, const float2* tw, int tid,
                                                const Store& store) {
  auto val = [](float2 zk, float2 zc, float2 w) {
    const float2 ev = make_float2(0.5f * (zk.x + zc.x), 0.5f * (zk.y + zc.y));
    const float2 od = make_float2(0.5f * (zk.x - zc.x), 0.5f * (zk.y - zc.y));
    const float2 t = cmul(w, od);   // w^k (Z_k - conj Z_{NC-k}) / 2
    return make_float2(ev.x + t.y, ev.y - t.x);   // ev - i t
  };
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int e = tid + i * T;
    const int c = e / NC, k = e % NC;
    const float2 zk = lds[k * LS + c];
    const float2 zc = cconj(lds[(k == 0 ? 0 : NC - k) * LS + c]);
    store(c, k, val(zk, zc, tw[k]));
  }
  if (tid < B) {
    const float2 z0 = lds[tid];
    store(tid, NC, val(z0, cconj(z0), make_float2(-1.f, 0.f)));
  }
}

// Forward Z pass: real rows of n = 2 NC floats (pitch 2*pitch floats) -> half-complex rows
// of NC + 1 values (pitch `pitch`).  Twiddles tw[t] = exp(-2 pi i t / n).
template <int NC>
__global__ void __launch_bounds__(RowCfg<NC>::T)
k_fft_r2c_row(const float* __restrict__ in, float2* __restrict__ out, int64_t nrows, int /*n*/,
              int pitch, int64_t plane, const float2* __restrict__ tw_g) {
  constexpr int B = RowCfg<NC>::B, E = RowCfg<NC>::E, T = RowCfg<NC>::T, LS = RowCfg<NC>::LS;
  __shared__ float2 lds[NC * LS];
  __shared__ float2 tw[2 * NC];   // split twiddles, then the per-stage table (row_twiddles)
  const int tid = threadIdx.x;
  using O = Off<2 * NC>;
  constexpr int kN = 2 * NC;   // real row length
  // Persistent: the work-group takes row blocks blockIdx.x, + gridDim.x, ...; the rows of
  // the next block are loaded into registers while this block is transformed and stored
  // (in place, in may alias out: a block's rows are read and written only by its owner).
  const int64_t nblk = (nrows + B - 1) / B;
  float2 v[E];
  using RB = RowBlock<kN, B, O>;
  auto issue = [&](int64_t blk) {
    const RB rb(blk, nrows, pitch, plane);
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int e = tid + i * T;
      const int c = e / NC, m = e % NC;
      v[i] = make_float2(0.f, 0.f);
      if (rb.valid(c)) v[i] = reinterpret_cast<const float2*>(in + 2 * rb.off(c))[m];
    }
  };
  int64_t blk = blockIdx.x;
  if (blk < nblk) issue(blk);
  row_twiddles<NC>(tw, tw_g, tid, T);   // after the row loads issue
  for (; blk < nblk; blk += gridDim.x) {
    const RB rb(blk, nrows, pitch, plane);
    __syncthreads();   // twiddles staged; the previous block has left the tile
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int e = tid + i * T;
      lds[(e % NC) * LS + e / NC] = v[i];
    }
    if (blk + gridDim.x < nblk) issue(blk + gridDim.x);
    __syncthreads();
    lds_fft<NC, -1, E, B, LS, 0, RowPlan<NC>>(lds, tid, T, tw + NC);
    split_fwd_store<NC, E, B, LS, T>(lds, tw, tid, [&](int c, int k, float2 v) {
      if (rb.valid(c)) out[rb.off(c) + k] = v;
    });
  }
}

// Inverse Z pass: half-complex rows (NC + 1 values) -> real rows of n = 2 NC floats,
// unnormalised.  Z_k = (X_k + conj X_{NC-k}) + i w^{-k} (X_k - conj X_{NC-k}), w = e^{-2 pi i/n};
// the unnormalised NC-point inverse of Z is (x_{2m} + i x_{2m+1}) with x the unnormalised
// length-n inverse of X.
template <int NC>
__global__ void __launch_bounds__(RowCfg<NC>::T)
k_fft_c2r_row(const float2* __restrict__ in, float* __restrict__ out, int64_t nrows, int /*n*/,
              int pitch, int64_t plane, const float2* __restrict__ tw_g) {
  constexpr int B = RowCfg<NC>::B, E = RowCfg<NC>::E, T = RowCfg<NC>::T, LS = RowCfg<NC>::LS;
  __shared__ float2 lds[NC * LS];
  __shared__ float2 tw[2 * NC];   // split twiddles, then the per-stage table (row_twiddles)
  const int tid = threadIdx.x;
  using O = Off<2 * NC>;
  constexpr int kN = 2 * NC;   // real row length
  // Persistent: the work-group takes row blocks blockIdx.x, + gridDim.x, ...; the rows of
  // the next block are loaded into registers while this block is transformed and stored
  // (in place, in may alias out: a block's rows are read and written only by its owner).
  const int64_t nblk = (nrows + B - 1) / B;
  using RB = RowBlock<kN, B, O>;
  auto rows_at = [&](int64_t blk) {
    const RB rb(blk, nrows, pitch, plane);
    return [=](int c) -> const float2* { return rb.valid(c) ? in + rb.off(c) : nullptr; };
  };
  InvSplit<NC, E / 2> sp;   // all row loads are issued before any is used
  int64_t blk = blockIdx.x;
  if (blk < nblk) sp.load(tid, T, rows_at(blk));
  row_twiddles<NC>(tw, tw_g, tid, T);   // after the row loads issue
  for (; blk < nblk; blk += gridDim.x) {
    const RB rb(blk, nrows, pitch, plane);
    __syncthreads();   // twiddles staged; the previous block has left the tile
    sp.store(tid, T, tw, lds, LS);
    if (blk + gridDim.x < nblk) sp.load(tid, T, rows_at(blk + gridDim.x));
    __syncthreads();
    lds_fft<NC, +1, E, B, LS, 0, RowPlan<NC>>(lds, tid, T, tw + NC);
    for (int e = tid; e < NC * B; e += T) {
      const int c = e / NC, m = e % NC;
      if (rb.valid(c)) reinterpret_cast<float2*>(out + 2 * rb.off(c))[m] = lds[m * LS + c];
    }
  }
}

// Inverse Z pass of the three force components in one sweep, written as one interleaved
// (F_x, F_y, F_z) mesh (unpadded rows), so that the CIC gather reads 24 contiguous bytes
// per pair of cells instead of three separate meshes.  The work-group splits into three
// thread groups, one per component, each transforming the same B rows through its own
// LDS tile as in k_fft_c2r_row; the last stage writes the interleaved rows into LDS over
// the three tiles, and all threads copy them out -- one contiguous block -- with 16-byte
// stores.  Tiles as in RowCfg (1024-point rows one to a work-group: 41 KB of LDS, three
// work-groups per CU).
template <int NC>
struct Row3Cfg {
  static constexpr int E = kRowE<NC>;
  static constexpr int B = NC >= 1024 ? 1 : (RowCfg<NC>::B >= 2 ? RowCfg<NC>::B / 2 : 1);
  static constexpr bool kPersist = RowCfg<NC>::kPersist;
  static constexpr int TC = NC * B / E;   // threads per component
  static constexpr int T = 3 * TC;
  static constexpr int LS = B == 1 ? 1 : B + 1;
};

template <int NC>
__global__ void __launch_bounds__(Row3Cfg<NC>::T)
k_fft_c2r_row3(const float2* __restrict__ in0, const float2* __restrict__ in1,
               const float2* __restrict__ in2, float* __restrict__ out, int64_t nrows,
               int pitch, int64_t plane, const float2* __restrict__ tw_g) {
  constexpr int B = Row3Cfg<NC>::B, E = Row3Cfg<NC>::E, TC = Row3Cfg<NC>::TC;
  constexpr int T = Row3Cfg<NC>::T, LS = Row3Cfg<NC>::LS;
  using O = Off<2 * NC>;
  using O3 = typename std::conditional<(3ull * 8 * NC * NC * NC < (1ull << 32)), uint32_t,
                                       uint64_t>::type;
  constexpr int kN = 2 * NC;
  constexpr int kRowF = 3 * kN;   // floats per interleaved row (a multiple of 4)
  static_assert(kRowF % 4 == 0, "interleaved rows must hold whole float4s");
  __shared__ __align__(16) float2 lds[3][NC * LS];   // also read as float4 at the end
  __shared__ float2 tw[2 * NC];   // split twiddles, then the per-stage table (row_twiddles)
  const int tid = threadIdx.x;
  const int comp = tid / TC, lt = tid - comp * TC;
  const float2* in = comp == 0 ? in0 : (comp == 1 ? in1 : in2);
  float2* tile = lds[comp];
  // Persistent: the work-group takes row blocks blockIdx.x, + gridDim.x, ...; the rows of
  // the next block are loaded into registers while this block is transformed and stored.
  const int64_t nblk = (nrows + B - 1) / B;
  using RB = RowBlock<kN, B, O>;
  auto rows_at = [&](int64_t blk) {
    const RB rb(blk, nrows, pitch, plane);
    return [=](int c) -> const float2* { return rb.valid(c) ? in + rb.off(c) : nullptr; };
  };
  InvSplit<NC, E / 2> sp;   // each row value is read from HBM once
  int64_t blk = blockIdx.x;
  if (blk < nblk) sp.load(lt, TC, rows_at(blk));
  row_twiddles<NC>(tw, tw_g, tid, T);   // after the row loads issue
  // The last Stockham stage writes the B interleaved output rows straight into LDS, over
  // the three tiles (every group has read its tile by the stage's barrier): element m of
  // row c of component t holds cells (2m, 2m + 1), at floats 3 (2m) + t and 3 (2m + 1) + t
  // of the row.  The rows then leave as one contiguous block of 16-byte stores.
  float* ilv = reinterpret_cast<float*>(&lds[0][0]);
  static_assert(B * kRowF <= 3 * 2 * NC * LS, "interleaved rows must fit the three tiles");
  for (; blk < nblk; blk += gridDim.x) {
    const O r0 = (O)blk * B;
    __syncthreads();   // twiddles staged; the previous block's rows have left the tiles
    sp.store(lt, TC, tw, tile, LS);
    if (blk + gridDim.x < nblk) sp.load(lt, TC, rows_at(blk + gridDim.x));
    __syncthreads();
    {
      auto load = [&](int, int, int j, int c) -> float2 { return tile[j * LS + c]; };
      auto store = [&](int m, int c, float2 v) {
        float* rowp = ilv + c * kRowF + 6 * m + comp;
        rowp[0] = v.x;
        rowp[3] = v.y;
      };
      GStages<NC, +1, E, B, LS, 0, 0, 1, kFirstFromLds | kLastToLds, RowPlan<NC>>::run(tile, lt, TC, tw + NC, load, store);
    }
    __syncthreads();
    const O rows_here = (O)nrows - r0 < (O)B ? (O)nrows - r0 : (O)B;
    const int nq = (int)rows_here * (kRowF / 4);
    float4* dst = reinterpret_cast<float4*>(out + (O3)r0 * kRowF);
    const float4* src4 = reinterpret_cast<const float4*>(ilv);
    for (int q = tid; q < nq; q += T) dst[q] = src4[q];
  }
}

// Screening in one row pass (Sec. 6): inverse Z transform of the filtered field (the
// smoothed density contrast for nDGP, the Newtonian potential for f(R)), the real-space
// screening factor eps and the source S = delta eps, and the forward Z transform of S --
// the filtered field and S never reach HBM in real space.  S may also be written out in
// real space (s_out) for diagnostics.
// Screening row pass tiles.  The pass keeps the next rows, their densities and two
// transforms' operands in registers (about 150 per lane); with one row of 512 or 1024
// complex values per work-group (16-24 KB of LDS) enough work-groups share a CU to overlap
// loads with transforms: 32 % faster than four-row tiles at 1024 and 40 % faster than
// eight-row tiles at 512.  The pass is persistent at every size.
template <int NC>
struct ScreenCfg {
  static constexpr int E = RowCfg<NC>::E;
  static constexpr int B = NC >= 512 ? 1 : RowCfg<NC>::B;
  static constexpr bool kPersist = true;
  static constexpr int T = NC * B / E;
  static constexpr int LS = B == 1 ? 1 : B + 1;
};

// With 12 elements per thread (the radix-3 lengths and 12) the compiler takes about 280
// registers, one wave per SIMD; held to two waves it spills 30-90 bytes per lane and runs
// 20-25 % faster.
template <int NC, int MODEL>
__global__ void __launch_bounds__(ScreenCfg<NC>::T)
__attribute__((amdgpu_waves_per_eu(ScreenCfg<NC>::E == 12 ? 2 : 1)))
k_fft_screen_row(float2* __restrict__ data, const float* __restrict__ rho, float* __restrict__ s_out,
                 int64_t nrows, int /*n*/, int pitch, int64_t plane, const float2* __restrict__ tw_g,
                 ScreenArgs sa) {
  constexpr int B = ScreenCfg<NC>::B, E = ScreenCfg<NC>::E, T = ScreenCfg<NC>::T;
  constexpr int LS = ScreenCfg<NC>::LS;
  if (sa.steps) {
    const StepDev& sd = sa.steps[*sa.step_ctr];
    sa.thr = sd.thr;
    sa.vx = sd.vx;
    sa.vx0 = sd.vx0;
    sa.cn = sd.cn;
    sa.c5 = sd.c5;
  }
  const float thr = sa.thr, vx = sa.vx, vx0 = sa.vx0, cn = sa.cn, c5 = sa.c5;
  __shared__ float2 lds[NC * LS];
  __shared__ float2 tw[2 * NC];   // split twiddles, then the per-stage table (row_twiddles)
  const int tid = threadIdx.x;
  using O = Off<2 * NC>;
  constexpr int kN = 2 * NC;   // real row length
  // Thread (i, r) handles element m = j + r NC/RL of row c (b = tid + i T, c = b % B,
  // j = b / B): the output of operand r of its butterfly i in the last inverse stage of
  // radix RL.  Its density pair (x_2m, x_2m+1) is loaded with the row, so that the
  // latency hides behind the inverse transform.
  using RP = RowPlan<NC>;
  constexpr int RL = RP::rad[RP::nst - 1], NBL = E / RL;
  constexpr bool kHandOff = RL == RP::rad[0];
  // Persistent: the work-group takes row blocks blockIdx.x, + gridDim.x, ...; the field
  // and density rows of the next block are loaded into registers while this block is
  // transformed and stored.
  const int64_t nblk = (nrows + B - 1) / B;
  InvSplit<NC, E / 2> sp;
  float2 rv[NBL][RL], rn[NBL][RL];
  using RB = RowBlock<kN, B, O>;
  auto issue = [&](int64_t blk) {
    const RB rb(blk, nrows, pitch, plane);
    sp.load(tid, T, [=](int c) -> const float2* { return rb.valid(c) ? data + rb.off(c) : nullptr; });
#pragma unroll
    for (int i = 0; i < NBL; ++i) {
      const int b = tid + i * T, c = b % B, j = b / B;
      const float2* rr = reinterpret_cast<const float2*>(rho + 2 * rb.off(c));
#pragma unroll
      for (int q = 0; q < RL; ++q)
        rn[i][q] = rb.valid(c) ? rr[j + q * (NC / RL)] : make_float2(1.f, 1.f);
    }
  };
  int64_t blk = blockIdx.x;
  if (blk < nblk) issue(blk);
  row_twiddles<NC>(tw, tw_g, tid, T);   // after the row loads issue
  for (; blk < nblk; blk += gridDim.x) {
    const RB rb(blk, nrows, pitch, plane);
    __syncthreads();   // twiddles staged; the previous block has left the tile
    sp.store(tid, T, tw, lds, LS);
#pragma unroll
    for (int i = 0; i < NBL; ++i)
#pragma unroll
      for (int q = 0; q < RL; ++q) rv[i][q] = rn[i][q];
    if (blk + gridDim.x < nblk) issue(blk + gridDim.x);
    __syncthreads();
    // field value f at the pair -> S = (rho - 1) eps(f) (written to s_out) and the value
    // (rho - 1)(cn + c5 eps) that the forward transform takes
    auto source = [&](float2 f, float2 rho2, int m, int c) {
      float e0, e1;
      if (MODEL == COLA_FR_HS1) {
        const float a0 = fabsf(f.x), a1 = fabsf(f.y);
        e0 = a0 > thr ? thr * fast_rcp(a0) : 1.f;
        e1 = a1 > thr ? thr * fast_rcp(a1) : 1.f;
      } else {
        // x = vx max(-1, delta_R) + vx0: vx0 = 0 for the mean-overdensity reading, vx for
        // the total-density one (1 + x > 1/9 either way)
        const float x0 = fmaf(vx, fmaxf(-1.f, f.x), vx0), x1 = fmaf(vx, fmaxf(-1.f, f.y), vx0);
        e0 = 2.f * fast_rcp(1.f + fast_sqrt(1.f + x0));
        e1 = 2.f * fast_rcp(1.f + fast_sqrt(1.f + x1));
      }
      const float2 dl = make_float2(rho2.x - 1.f, rho2.y - 1.f);
      if (s_out && rb.valid(c))
        reinterpret_cast<float2*>(s_out + 2 * rb.off(c))[m] = make_float2(dl.x * e0, dl.y * e1);
      return make_float2(dl.x * (cn + c5 * e0), dl.y * (cn + c5 * e1));
    };
    if constexpr (kHandOff) {
      // the last inverse stage hands its outputs to the first forward stage in registers
      float2 tv[NBL][RL];
      {
        auto load = [&](int, int, int j, int c) -> float2 { return lds[j * LS + c]; };
        auto store = [&](int m, int c, float2 f, int i, int r) { tv[i][r] = source(f, rv[i][r], m, c); };
        GStages<NC, +1, E, B, LS, 0, 0, 1, kFirstFromLds | kStoreIR, RP>::run(lds, tid, T, tw + NC, load, store);
      }
      __syncthreads();   // every thread has read its last operands out of the tile
      {
        auto load = [&](int i, int r, int, int) -> float2 { return tv[i][r]; };
        auto store = [&](int j, int c, float2 v) { lds[j * LS + c] = v; };
        GStages<NC, -1, E, B, LS, 0, 0, 1, kLastToLds, RP>::run(lds, tid, T, tw + NC, load, store);
      }
    } else {
      lds_fft<NC, +1, E, B, LS, 0, RowPlan<NC>>(lds, tid, T, tw + NC);
#pragma unroll
      for (int i = 0; i < NBL; ++i) {
        const int b = tid + i * T, c = b % B, j = b / B;
#pragma unroll
        for (int r = 0; r < RL; ++r) {
          const int m = j + r * (NC / RL);
          lds[m * LS + c] = source(lds[m * LS + c], rv[i][r], m, c);
        }
      }
      __syncthreads();
      lds_fft<NC, -1, E, B, LS, 0, RowPlan<NC>>(lds, tid, T, tw + NC);
    }
    __syncthreads();
    split_fwd_store<NC, E, B, LS, T>(lds, tw, tid, [&](int c, int k, float2 v) {
      if (rb.valid(c)) data[rb.off(c) + k] = v;
    });
  }
}

// ------------------------------------------------------------------ dispatch
// Grid of a persistent kernel: as many work-groups as the device holds at once (by the
// kernel's occupancy), at most `blocks`.  Occupancy and CU count are looked up once per
// kernel and device.
static unsigned persistent_grid(const void* kernel, int threads, int64_t blocks) {
  static std::mutex mu;
  static std::map<std::pair<const void*, int>, int> cache;
  int dev = 0;
  COLA_HIP_CHECK(hipGetDevice(&dev));
  int resident;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find({kernel, dev});
    if (it == cache.end()) {
      int per_cu = 0, cus = 0;
      COLA_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0));
      COLA_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
      it = cache.emplace(std::make_pair(kernel, dev), std::max(1, per_cu) * std::max(1, cus)).first;
    }
    resident = it->second;
  }
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(blocks, resident));
}

bool fft_size_supported(int n) {
  switch (n) {
    case 8: case 12: case 16: case 24: case 32: case 48: case 64: case 96: case 128:
    case 192: case 256: case 384: case 512: case 768: case 1024: case 1536: case 2048:
      return true;
    default:
      return false;
  }
}

template <int N, int DIR, int KIND, int BB = ColCfg<N>::B>
static void col_pass(float2* data, int64_t elemStride, int64_t tiles, int64_t tilesPerBlock,
                     int64_t blockStride, const float2* tw, const KOp& op, hipStream_t s,
                     const char* name) {
  ProfScope ps(name, s);
  hipLaunchKernelGGL((k_fft_col<N, DIR, KIND, BB>), dim3((unsigned)tiles), dim3(N * BB / ColCfg<N>::E), 0, s,
                     data, elemStride, tilesPerBlock, blockStride, tiles, tw, op);
  COLA_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ Y-pass tile widths
// The Y passes (stride one row pitch) can run with 4, 8 or 16 columns per tile where the
// tile fits LDS and the work-group limit; every choice computes the same butterflies on
// each column, so results are bitwise independent of it.  The width per transform size
// and direction comes from a process-wide table: the LDS-limited default, or what
// fft_autotune measured fastest, or what the caller set.
template <int N, int B>
constexpr bool kTileOk = (N * B / ColCfg<N>::E) <= 1024 && (N * B / ColCfg<N>::E) % B == 0 &&
                         (size_t)N * B * 8 + (size_t)N * 8 <= 163840;

static constexpr int kSizes[] = {8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768,
                                 1024, 1536, 2048};
static int size_index(int n) {
  for (int i = 0; i < (int)(sizeof(kSizes) / sizeof(int)); ++i)
    if (kSizes[i] == n) return i;
  return -1;
}
static std::atomic<int> g_ytile[sizeof(kSizes) / sizeof(int)][2];   // 0 = default

template <int N>
static int y_tile(int dir) {
  const int i = size_index(N);
  const int t = g_ytile[i][dir > 0 ? 1 : 0].load(std::memory_order_relaxed);
  return t ? t : ColCfg<N>::B;
}

template <int N, int DIR, int B>
static void y_pass_b(float2* data, const FFTPlan& pl, const KOp& op, hipStream_t s, const char* name) {
  if constexpr (kTileOk<N, B>) {
    const int P = pl.pitch;
    col_pass<N, DIR, K_COPY, B>(data, P, (int64_t)pl.n * (P / B), P / B, pl.plane, pl.tw, op, s, name);
  } else {
    throw Error{COLA_E_ARG, "Y-pass tile width not valid for this size"};
  }
}

template <int N, int DIR>
static void y_pass(float2* data, const FFTPlan& pl, const KOp& op, hipStream_t s, const char* name) {
  switch (y_tile<N>(DIR)) {
    case 4: y_pass_b<N, DIR, 4>(data, pl, op, s, name); break;
    case 8: y_pass_b<N, DIR, 8>(data, pl, op, s, name); break;
    default: y_pass_b<N, DIR, 16>(data, pl, op, s, name); break;
  }
}

template <int N>
static bool tile_valid(int b) {
  return (b == 4 && kTileOk<N, 4>) || (b == 8 && kTileOk<N, 8>) || (b == 16 && kTileOk<N, 16>);
}

// fwd, inv: 4, 8 or 16 sets the width, 0 restores the default, -1 leaves it
template <int N>
static void set_tiles_impl(int fwd, int inv) {
  for (int w : {fwd, inv})
    if (w != -1 && w != 0 && !tile_valid<N>(w))
      throw Error{COLA_E_ARG, "tile width must be 4, 8 or 16 and fit this transform size"};
  const int i = size_index(N);
  if (fwd >= 0) g_ytile[i][0].store(fwd);
  if (inv >= 0) g_ytile[i][1].store(inv);
}

// Times every valid width of the forward and inverse Y passes of an N-point transform on
// `data` (a work field laid out by pl; its contents are overwritten) and keeps the fastest.
template <int N>
static void autotune_impl(const FFTPlan& pl, float2* data, hipStream_t s, int out[2]) {
  hipEvent_t e0, e1;
  COLA_HIP_CHECK(hipEventCreate(&e0));
  COLA_HIP_CHECK(hipEventCreate(&e1));
  KOp none;
  for (int d = 0; d < 2; ++d) {
    float best = 1e30f;
    int best_b = ColCfg<N>::B;
    for (int b : {4, 8, 16}) {
      if (!tile_valid<N>(b)) continue;
      auto run = [&] {
        if (d == 0) {
          if (b == 4) y_pass_b<N, -1, 4>(data, pl, none, s, "fft_y_tune");
          else if (b == 8) y_pass_b<N, -1, 8>(data, pl, none, s, "fft_y_tune");
          else y_pass_b<N, -1, 16>(data, pl, none, s, "fft_y_tune");
        } else {
          if (b == 4) y_pass_b<N, 1, 4>(data, pl, none, s, "fft_y_tune");
          else if (b == 8) y_pass_b<N, 1, 8>(data, pl, none, s, "fft_y_tune");
          else y_pass_b<N, 1, 16>(data, pl, none, s, "fft_y_tune");
        }
      };
      run();   // warm-up
      COLA_HIP_CHECK(hipEventRecord(e0, s));
      for (int r = 0; r < 3; ++r) run();
      COLA_HIP_CHECK(hipEventRecord(e1, s));
      COLA_HIP_CHECK(hipEventSynchronize(e1));
      float ms = 0.f;
      COLA_HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best) {
        best = ms;
        best_b = b;
      }
    }
    g_ytile[size_index(N)][d].store(best_b);
    out[d] = best_b;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

template <int N>
static void r2c_impl(const FFTPlan& pl, const float* in, float2* out, bool x_pass, hipStream_t s) {
  const int n = pl.n, P = pl.pitch;
  const int64_t rows = (int64_t)n * n;
  {
    ProfScope ps("fft_r2c_z", s);
    constexpr int B = RowCfg<N / 2>::B;
    const unsigned grid = RowCfg<N / 2>::kPersist
        ? persistent_grid(reinterpret_cast<const void*>(&k_fft_r2c_row<N / 2>), RowCfg<N / 2>::T,
                          (rows + B - 1) / B)
        : (unsigned)((rows + B - 1) / B);
    hipLaunchKernelGGL((k_fft_r2c_row<N / 2>), dim3(grid), dim3(RowCfg<N / 2>::T), 0, s, in, out,
                       rows, n, P, pl.plane, pl.tw);
    COLA_LAUNCH_CHECK();
  }
  KOp op;
  // Y pass: per x-plane, tiles of B z-columns, element stride = pitch
  y_pass<N, -1>(out, pl, op, s, "fft_y_fwd");
  // X pass: tiles of XCfg B (y, z) columns, element stride = plane
  constexpr int BX = XCfg<N>::B;
  if (x_pass)
    col_pass<N, -1, K_COPY, BX>(out, pl.plane, (int64_t)n * P / BX, (int64_t)n * P / BX, 0, pl.tw,
                                op, s, "fft_x_fwd");
}

template <int N>
static void c2r_impl(const FFTPlan& pl, int kind, const KOp& op_in, float2* data, float* out,
                     hipStream_t s) {
  const int n = pl.n, P = pl.pitch;
  const int64_t rows = (int64_t)n * n;
  KOp op = op_in;
  op.n = n;
  op.pitch = P;
  op.plane = pl.plane;
  constexpr int BX = XCfg<N>::B;
  const int64_t xtiles = (int64_t)n * P / BX;
  const int64_t ES = pl.plane;
  switch (kind) {
    case K_COPY: col_pass<N, 1, K_COPY, BX>(data, ES, xtiles, xtiles, 0, pl.tw, op, s, "fft_x_inv"); break;
    case K_FORCE: col_pass<N, 1, K_FORCE, BX>(data, ES, xtiles, xtiles, 0, pl.tw, op, s, "fft_x_inv_force"); break;
    case K_POT: col_pass<N, 1, K_POT, BX>(data, ES, xtiles, xtiles, 0, pl.tw, op, s, "fft_x_inv_pot"); break;
    case K_SMOOTH: col_pass<N, 1, K_SMOOTH, BX>(data, ES, xtiles, xtiles, 0, pl.tw, op, s, "fft_x_inv_smooth"); break;
    case K_LPT: col_pass<N, 1, K_LPT, BX>(data, ES, xtiles, xtiles, 0, pl.tw, op, s, "fft_x_inv_lpt"); break;
    case K_HESS: col_pass<N, 1, K_HESS, BX>(data, ES, xtiles, xtiles, 0, pl.tw, op, s, "fft_x_inv_hess"); break;
    case K_GRAD: col_pass<N, 1, K_GRAD, BX>(data, ES, xtiles, xtiles, 0, pl.tw, op, s, "fft_x_inv_grad"); break;
    default: throw Error{COLA_E_ARG, "unknown k-space operator"};
  }
  // the particle-grid transforms of the LPT terms are timed under names of their own
  const bool lpt = kind == K_LPT;
  KOp none;
  y_pass<N, 1>(data, pl, none, s, lpt ? "lpt_fft_y_inv" : "fft_y_inv");
  {
    ProfScope ps(lpt ? "lpt_fft_c2r_z" : "fft_c2r_z", s);
    constexpr int BR = RowCfg<N / 2>::B;
    const unsigned grid = RowCfg<N / 2>::kPersist
        ? persistent_grid(reinterpret_cast<const void*>(&k_fft_c2r_row<N / 2>), RowCfg<N / 2>::T,
                          (rows + BR - 1) / BR)
        : (unsigned)((rows + BR - 1) / BR);
    hipLaunchKernelGGL((k_fft_c2r_row<N / 2>), dim3(grid), dim3(RowCfg<N / 2>::T), 0, s, data, out,
                       rows, n, P, pl.plane, pl.tw);
    COLA_LAUNCH_CHECK();
  }
}

static void r2c_dispatch(const FFTPlan& pl, const float* in, float2* out, bool x_pass, hipStream_t s) {
  switch (pl.n) {
#define CASE(N_) case N_: r2c_impl<N_>(pl, in, out, x_pass, s); return;
    CASE(8) CASE(12) CASE(16) CASE(24) CASE(32) CASE(48) CASE(64) CASE(96) CASE(128)
    CASE(192) CASE(256) CASE(384) CASE(512) CASE(768) CASE(1024) CASE(1536) CASE(2048)
#undef CASE
    default: throw Error{COLA_E_UNSUPPORTED, "FFT size not supported"};
  }
}

void fft_r2c(const FFTPlan& pl, const float* in, float2* out, hipStream_t s) {
  r2c_dispatch(pl, in, out, true, s);
}

void fft_r2c_zy(const FFTPlan& pl, const float* in, float2* out, hipStream_t s) {
  r2c_dispatch(pl, in, out, false, s);
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

// Y and Z passes shared by the force and LPT transforms: work[0] holds G0 after its X
// pass (the x component), work[1] G; the inverse Y pass of G0, the two-component Y pass
// of G into work[1] (y) and work[2] (z), and one real Z pass of all three writing the
// interleaved rows out3[((x n + y) n + z) 3 + c].
template <int N>
static void grad3_tail(const FFTPlan& pl, const KOp& op, float2* const work[3], float* out3,
                       bool lpt, hipStream_t s) {
  const int n = pl.n, P = pl.pitch;
  const int64_t rows = (int64_t)n * n;
  constexpr int B = ColCfg<N>::B;
  KOp none;
  const int64_t ytiles = (int64_t)n * (P / B);
  y_pass<N, 1>(work[0], pl, none, s, lpt ? "lpt_fft_y_inv" : "fft_y_inv");
  {
    ProfScope ps(lpt ? "lpt_fft_y_inv_yz" : "fft_y_inv_yz", s);
    hipLaunchKernelGGL((k_fft_col_inv_yz<N>), dim3((unsigned)ytiles), dim3(FusedCfg<N, B>::T), 0, s,
                       work[1], work[1], work[2], (int64_t)P, (int64_t)(P / B), pl.plane, pl.tw, op);
    COLA_LAUNCH_CHECK();
  }
  {
    ProfScope ps(lpt ? "lpt_fft_c2r_z3" : "fft_c2r_z3", s);
    constexpr int BR = Row3Cfg<N / 2>::B;
    const int64_t nblk = (rows + BR - 1) / BR;
    const unsigned grid = Row3Cfg<N / 2>::kPersist
        ? persistent_grid(reinterpret_cast<const void*>(&k_fft_c2r_row3<N / 2>), Row3Cfg<N / 2>::T, nblk)
        : (unsigned)nblk;
    hipLaunchKernelGGL((k_fft_c2r_row3<N / 2>), dim3(grid), dim3(Row3Cfg<N / 2>::T), 0, s, work[0],
                       work[1], work[2], out3, rows, P, pl.plane, pl.tw);
    COLA_LAUNCH_CHECK();
  }
}

template <int N>
static void force3_impl(const FFTPlan& pl, const KOp& op_in, const float2* dk, const float2* src,
                        float2* const work[3], float* f3, hipStream_t s) {
  const int n = pl.n, P = pl.pitch;
  constexpr int B = ColCfg<N>::B;
  KOp op = op_in;
  op.n = n;
  op.pitch = P;
  op.plane = pl.plane;
  {
    const dim3 g((unsigned)((int64_t)n * P / B)), b(FusedCfg<N, B>::T);
    if (dk) {
      ProfScope ps("fft_x_fwd_force", s);
      hipLaunchKernelGGL((k_fft_col_fwd_force<N, true>), g, b, 0, s, dk, src, work[0], work[1],
                         pl.plane, pl.tw, op);
    } else {
      ProfScope ps("fft_x_fwd_force_1src", s);
      hipLaunchKernelGGL((k_fft_col_fwd_force<N, false>), g, b, 0, s, dk, src, work[0], work[1],
                         pl.plane, pl.tw, op);
    }
    COLA_LAUNCH_CHECK();
  }
  grad3_tail<N>(pl, op, work, f3, false, s);
}

template <int N>
static void lpt3_impl(const FFTPlan& pl, const KOp& op_in, const float2* phi1, const float2* phi2,
                      float2* const work[3], float* out3, hipStream_t s) {
  const int n = pl.n, P = pl.pitch;
  KOp op = op_in;
  op.n = n;
  op.pitch = P;
  op.plane = pl.plane;
  {
    ProfScope ps("lpt_fft_x_inv", s);
    constexpr int B = LptXCfg<N>::B;
    hipLaunchKernelGGL((k_fft_col_lpt<N>), dim3((unsigned)((int64_t)n * P / B)),
                       dim3(LptXCfg<N>::T), 0, s, phi1, phi2, work[0], work[1], pl.plane, pl.tw, op);
    COLA_LAUNCH_CHECK();
  }
  grad3_tail<N>(pl, op, work, out3, true, s);
}

template <int N>
static void screen_impl(const FFTPlan& pl, int kind, const KOp& op_in, float2* dk, float2* data,
                        const float* rho, float* s_out, int model, const ScreenArgs& sa,
                        hipStream_t s) {
  const int n = pl.n, P = pl.pitch;
  const int64_t rows = (int64_t)n * n;
  KOp op = op_in;
  op.n = n;
  op.pitch = P;
  op.plane = pl.plane;
  {
    const dim3 g((unsigned)((int64_t)n * P / OpCfg<N>::B)), b(OpCfg<N>::T);
    if (kind == K_POT) {
      ProfScope ps("fft_x_fwd_pot", s);
      hipLaunchKernelGGL((k_fft_col_fwd_op<N, K_POT, true>), g, b, 0, s, dk, data, pl.plane, pl.tw, op);
    } else {
      ProfScope ps("fft_x_fwd_smooth", s);
      hipLaunchKernelGGL((k_fft_col_fwd_op<N, K_SMOOTH, false>), g, b, 0, s, dk, data, pl.plane, pl.tw, op);
    }
    COLA_LAUNCH_CHECK();
  }
  KOp none;
  y_pass<N, 1>(data, pl, none, s, "fft_y_inv");
  {
    ProfScope ps("fft_z_screen", s);
    constexpr int BR = ScreenCfg<N / 2>::B;
    const int64_t nblk = (rows + BR - 1) / BR;
    const dim3 b(ScreenCfg<N / 2>::T);
    if (model == COLA_FR_HS1 || model == COLA_SYMMETRON || model == COLA_MBETA) {   // eps = min(1, thr/|Phi|)
      const dim3 g(ScreenCfg<N / 2>::kPersist
          ? persistent_grid(reinterpret_cast<const void*>(&k_fft_screen_row<N / 2, COLA_FR_HS1>),
                            ScreenCfg<N / 2>::T, nblk)
          : (unsigned)nblk);
      hipLaunchKernelGGL((k_fft_screen_row<N / 2, COLA_FR_HS1>), g, b, 0, s, data, rho, s_out, rows, n,
                         P, pl.plane, pl.tw, sa);
    } else {
      const dim3 g(ScreenCfg<N / 2>::kPersist
          ? persistent_grid(reinterpret_cast<const void*>(&k_fft_screen_row<N / 2, COLA_NDGP>),
                            ScreenCfg<N / 2>::T, nblk)
          : (unsigned)nblk);
      hipLaunchKernelGGL((k_fft_screen_row<N / 2, COLA_NDGP>), g, b, 0, s, data, rho, s_out, rows, n, P,
                         pl.plane, pl.tw, sa);
    }
    COLA_LAUNCH_CHECK();
  }
  y_pass<N, -1>(data, pl, none, s, "fft_y_fwd");
}

void fft_c2r_force3(const FFTPlan& pl, const KOp& op, const float2* dk, const float2* src,
                    float2* const work[3], float* f3, hipStream_t s) {
  switch (pl.n) {
#define CASE(N_) case N_: force3_impl<N_>(pl, op, dk, src, work, f3, s); return;
    CASE(8) CASE(12) CASE(16) CASE(24) CASE(32) CASE(48) CASE(64) CASE(96) CASE(128)
    CASE(192) CASE(256) CASE(384) CASE(512) CASE(768) CASE(1024) CASE(1536) CASE(2048)
#undef CASE
    default: throw Error{COLA_E_UNSUPPORTED, "FFT size not supported"};
  }
}

void fft_c2r_lpt3(const FFTPlan& pl, const KOp& op, const float2* phi1, const float2* phi2,
                  float2* const work[3], float* out3, hipStream_t s) {
  switch (pl.n) {
#define CASE(N_) case N_: lpt3_impl<N_>(pl, op, phi1, phi2, work, out3, s); return;
    CASE(8) CASE(12) CASE(16) CASE(24) CASE(32) CASE(48) CASE(64) CASE(96) CASE(128)
    CASE(192) CASE(256) CASE(384) CASE(512) CASE(768) CASE(1024) CASE(1536) CASE(2048)
#undef CASE
    default: throw Error{COLA_E_UNSUPPORTED, "FFT size not supported"};
  }
}

void fft_set_tiles(int n, int fwd, int inv) {
  switch (n) {
#define CASE(N_) case N_: set_tiles_impl<N_>(fwd, inv); return;
    CASE(8) CASE(12) CASE(16) CASE(24) CASE(32) CASE(48) CASE(64) CASE(96) CASE(128)
    CASE(192) CASE(256) CASE(384) CASE(512) CASE(768) CASE(1024) CASE(1536) CASE(2048)
#undef CASE
    default: throw Error{COLA_E_ARG, "transform size not supported"};
  }
}

void fft_get_tiles(int n, int out[2]) {
  switch (n) {
#define CASE(N_) case N_: out[0] = y_tile<N_>(-1); out[1] = y_tile<N_>(1); return;
    CASE(8) CASE(12) CASE(16) CASE(24) CASE(32) CASE(48) CASE(64) CASE(96) CASE(128)
    CASE(192) CASE(256) CASE(384) CASE(512) CASE(768) CASE(1024) CASE(1536) CASE(2048)
#undef CASE
    default: throw Error{COLA_E_ARG, "transform size not supported"};
  }
}

void fft_autotune(const FFTPlan& pl, float2* data, hipStream_t s, int out[2]) {
  switch (pl.n) {
#define CASE(N_) case N_: autotune_impl<N_>(pl, data, s, out); return;
    CASE(8) CASE(12) CASE(16) CASE(24) CASE(32) CASE(48) CASE(64) CASE(96) CASE(128)
    CASE(192) CASE(256) CASE(384) CASE(512) CASE(768) CASE(1024) CASE(1536) CASE(2048)
#undef CASE
    default: throw Error{COLA_E_UNSUPPORTED, "FFT size not supported"};
  }
}

void fft_screen(const FFTPlan& pl, int kind, const KOp& op, float2* dk, float2* data, const float* rho,
                float* s_out, int model, const ScreenArgs& sa, hipStream_t s) {
  switch (pl.n) {
#define CASE(N_) case N_: screen_impl<N_>(pl, kind, op, dk, data, rho, s_out, model, sa, s); return;
    CASE(8) CASE(12) CASE(16) CASE(24) CASE(32) CASE(48) CASE(64) CASE(96) CASE(128)
    CASE(192) CASE(256) CASE(384) CASE(512) CASE(768) CASE(1024) CASE(1536) CASE(2048)
#undef CASE
    default: throw Error{COLA_E_UNSUPPORTED, "FFT size not supported"};
  }
}

}  // namespace cola
