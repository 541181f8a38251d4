// Particle-mesh kernels: CIC deposit, real-space screening, CIC gather fused with the
// COLA kick and drift, stand-alone k-space operators, layout copies and P(k) binning.
//
// Particle p sits in row-major Lagrangian order, p = (ix*np + iy)*np + iz, at
// q = (ix*ratio + 1/2) cells per axis (ratio = nmesh/np, an integer), so its position in
// cells is s = ix*ratio + f with f = 1/2 + u/cell.  The integer and fractional parts are
// kept apart: the CIC offset d = f - floor(f) is exact in single precision, whatever the
// box size, and only u/cell carries rounding.

#include <algorithm>

#include "internal.h"
#include "kspace.h"

namespace cola {

// ------------------------------------------------------------------ helpers
struct CicCell {
  int64_t i0[3], i1[3];   // wrapped mesh coordinates of the two nodes per axis
  float w0[3], w1[3];     // their weights (1 - d, d)
};

__device__ __forceinline__ void cic_axis(int ixq, float u, int nm, int ratio, float inv_cell,
                                         int64_t& i0, int64_t& i1, float& w0, float& w1) {
  const float f = 0.5f + u * inv_cell;
  const float fl = floorf(f);
  const float d = f - fl;
  int i = ixq * ratio + (int)fl;
  i %= nm;
  if (i < 0) i += nm;
  i0 = i;
  i1 = (i + 1 == nm) ? 0 : i + 1;
  w0 = 1.f - d;
  w1 = d;
}

static bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
static int ilog2(int v) {
  int l = 0;
  while ((1 << (l + 1)) <= v) ++l;
  return l;
}

static unsigned grid_for(int64_t n, int block, int64_t cap = 1 << 20) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + block - 1) / block, cap));
}

// ------------------------------------------------------------------ fill
__global__ void k_fill(float* __restrict__ p, int64_t n, float v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

void launch_fill(float* p, size_t n, float v, hipStream_t s) {
  ProfScope ps("fill", s);
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n, 256)), dim3(256), 0, s, p, (int64_t)n, v);
  COLA_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ CIC deposit
// rho_j = sum_p m W(x_p - x_j), m = (nmesh/np)^3 so that rho averages to 1.
//
// Device-wide float atomics on a multi-GB mesh resolve beyond the per-XCD L2 caches and
// run far below HBM bandwidth, so the deposit is a counting sort instead:
//  1. count: every particle finds its home tile (the T^3-cell tile holding its lower CIC
//     corner i0) and its class c = bitmask of the axes on which i0 sits on the tile's
//     last layer (c != 0: some corners spill into the next tile).  Work-groups take
//     Lagrangian bricks of 4x8x8 particles, which land in few tiles; the lanes of a wave
//     that share a (tile, class) make one global add between them;
//  2. scan: exclusive prefix over tiles, then per-class cursors inside each tile;
//  3. scatter: the same bricks write CIC records into the tile/class segments;
//  4. deposit: one work-group per tile accumulates in LDS the corners that fall inside it
//     -- from every particle of its own tile and from the class-c particles of the seven
//     lower neighbour tiles T - delta with (c & delta) == delta -- and writes the tile
//     once with plain stores, so the mesh needs no zeroing pass.
constexpr int kBrickX = 4, kBrickY = 8, kBrickZ = 8;   // 256 particles per brick
constexpr int kBinBricks = 2;                           // bricks per binning work-group
constexpr int kScanBlock = 1024;                        // tiles per scan block
constexpr float kFix = 16777216.f;                      // 2^24: deposit fixed-point unit
// Threads per tile work-group: the LDS accumulator (32 KB for 16^3 cells) allows four
// work-groups per CU, and eight waves each keep more entry loads and LDS atomics in
// flight than four (sixteen measured slower).
constexpr int kDepositThreads = 512;

size_t bins_bytes(int64_t ntiles) {
  const int64_t nblk = (ntiles + kScanBlock - 1) / kScanBlock;
  return align_up((size_t)(17 * ntiles + 2 * nblk + 64) * sizeof(uint32_t));
}

struct BinGeo {
  int np, nm, ratio, nt1, tile;
  int lt;         // log2(tile); the tile side is always a power of two
  int lnp, lnm;   // log2(np), log2(nm) when both are powers of two (the P2 kernels)
  float inv_cell;
  int64_t N;
};

// Lower CIC corner (cell) and offset of one axis; the same arithmetic as cic_axis().
// P2: nm is a power of two, and the wrap is a mask (exact for negative cells too).
template <bool P2>
__device__ __forceinline__ int axis_cell(int ixq, float u, const BinGeo& g, float& d) {
  const float f = 0.5f + u * g.inv_cell;
  const float fl = floorf(f);
  d = f - fl;
  if (P2) return (ixq * g.ratio + (int)fl) & (g.nm - 1);
  int i = (ixq * g.ratio + (int)fl) % g.nm;
  return i < 0 ? i + g.nm : i;
}

template <bool P2>
__device__ __forceinline__ bool brick_particle(const BinGeo& g, int b, int& ix, int& iy, int& iz,
                                               int64_t& p) {
  const int nbz = (g.np + kBrickZ - 1) / kBrickZ, nby = (g.np + kBrickY - 1) / kBrickY;
  const int nbx = (g.np + kBrickX - 1) / kBrickX;
  if (b >= nbx * nby * nbz) return false;
  int bz, by, bx;
  if (P2 && g.np >= kBrickY) {   // np / 8 bricks per axis, a power of two
    const int l = g.lnp - 3;
    bz = b & ((1 << l) - 1);
    by = (b >> l) & ((1 << l) - 1);
    bx = b >> (2 * l);
  } else {
    bz = b % nbz;
    by = (b / nbz) % nby;
    bx = b / (nbz * nby);
  }
  const int t = threadIdx.x;
  ix = bx * kBrickX + (t >> 6);
  iy = by * kBrickY + ((t >> 3) & 7);
  iz = bz * kBrickZ + (t & 7);
  if (ix >= g.np || iy >= g.np || iz >= g.np) return false;
  p = ((int64_t)ix * g.np + iy) * g.np + iz;
  return true;
}

// CIC record of a particle (12 bytes): per axis, the lower corner's cell inside its home
// tile (bits 28-31) and the offset d in [0, 1) as a 28-bit fraction (bits 0-27).  The
// record is lossless: f = 1/2 + u/cell is an FP32 sum with 1/2, so f and d = f - floor(f)
// are multiples of 2^-25 (of 2^-23 once |f| >= 1), and d * 2^28 is an integer below 2^28
// whose conversion back to FP32 is exact.  Four bytes less per particle than a float4
// record, written by the scatter and read by the deposit.
struct CicRec {
  uint32_t x, y, z;
};
__device__ __forceinline__ uint32_t rec_axis(int local, float d) {
  return ((uint32_t)local << 28) | (uint32_t)(d * 268435456.f);
}
__device__ __forceinline__ float rec_d(uint32_t v) {
  return (float)(v & 0x0FFFFFFFu) * (1.f / 268435456.f);
}

// MODE 0: count into cnt[tile*8 + cls];  MODE 1: scatter the particle's CIC record
// (offsets and lower corner relative to its home tile) to entries[cur[tile*8 + cls]++].
// A work-group takes kBinBricks consecutive bricks and each thread one particle of each,
// with all displacement loads issued up front.  The lanes of a wave that share a
// (tile, class) key are served by one atomic that adds their number; in MODE 1 each lane
// takes the returned base plus its rank among them.  A wave holds an 8 x 8 patch of one
// lattice plane, so it meets only a few keys.
template <int MODE, bool P2>
__global__ void __launch_bounds__(256)
k_bin(const float* __restrict__ disp, BinGeo g, uint32_t* __restrict__ cnt,
      uint32_t* __restrict__ cur, CicRec* __restrict__ entries) {
  constexpr int S = kBinBricks;
  const int b0 = (int)xcd_block(blockIdx.x, gridDim.x) * S;
  bool valid[S];
  int64_t p[S];
  int ix[S], iy[S], iz[S];
  float ux[S], uy[S], uz[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    p[s] = 0;
    ix[s] = iy[s] = iz[s] = 0;
    valid[s] = brick_particle<P2>(g, b0 + s, ix[s], iy[s], iz[s], p[s]);
    ux[s] = uy[s] = uz[s] = 0.f;
    if (valid[s]) {
      ux[s] = disp[p[s]];
      uy[s] = disp[g.N + p[s]];
      uz[s] = disp[2 * g.N + p[s]];
    }
  }
  const int lane = (int)__lane_id();
  uint32_t gbase[S], myrank[S];
  int mygroup[S];
  CicRec rec[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    unsigned key = 0xffffffffu;
    rec[s] = CicRec{0u, 0u, 0u};
    if (valid[s]) {
      float dx, dy, dz;
      const int cx = axis_cell<P2>(ix[s], ux[s], g, dx);
      const int cy = axis_cell<P2>(iy[s], uy[s], g, dy);
      const int cz = axis_cell<P2>(iz[s], uz[s], g, dz);
      const int lt = g.lt, m = g.tile - 1;
      const int tile = ((cx >> lt) * g.nt1 + (cy >> lt)) * g.nt1 + (cz >> lt);
      const int cls = ((cx & m) == m ? 1 : 0) | ((cy & m) == m ? 2 : 0) | ((cz & m) == m ? 4 : 0);
      rec[s] = CicRec{rec_axis(cx & m, dx), rec_axis(cy & m, dy), rec_axis(cz & m, dz)};
      key = (unsigned)tile * 8u + (unsigned)cls;
    }
    // group the wave's lanes by key with ballots (no memory traffic); group i's key and
    // size land in lane i, which then makes the group's one atomic -- all groups' atomics
    // go out as a single wave instruction
    unsigned long long todo = __ballot(valid[s]);
    int it = 0;
    uint32_t gcnt = 0;
    unsigned gkey = 0;
    mygroup[s] = 0;
    myrank[s] = 0;
    while (todo) {   // wave-uniform: every lane runs the same iterations, at most 64
      const int leader = __ffsll((unsigned long long)todo) - 1;
      const unsigned lkey = __shfl(key, leader);
      const unsigned long long m = __ballot(key == lkey) & todo;
      if (lane == it) {
        gkey = lkey;
        gcnt = (uint32_t)__popcll(m);
      }
      if ((m >> lane) & 1ull) {
        mygroup[s] = it;
        myrank[s] = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
      }
      todo &= ~m;
      ++it;
    }
    gbase[s] = 0;
    if (lane < it) {
      if (MODE == 0)
        atomicAdd(&cnt[gkey], gcnt);
      else
        gbase[s] = atomicAdd(&cur[gkey], gcnt);
    }
  }
  if (MODE == 1) {
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const uint32_t base = __shfl(gbase[s], mygroup[s]);
      if (valid[s]) entries[base + myrank[s]] = rec[s];
    }
  }
}

// Tile totals -> per-block sums (block of kScanBlock tiles).
__global__ void __launch_bounds__(256)
k_scan_reduce(const uint32_t* __restrict__ cnt, uint32_t* __restrict__ bsum, int64_t ntiles) {
  __shared__ uint32_t red[256];
  const int64_t t0 = (int64_t)blockIdx.x * kScanBlock;
  uint32_t s = 0;
  for (int i = threadIdx.x; i < kScanBlock; i += 256) {
    const int64_t t = t0 + i;
    if (t < ntiles) {
      const uint4* c4 = reinterpret_cast<const uint4*>(cnt + t * 8);
      const uint4 a = c4[0], b = c4[1];
      s += a.x + a.y + a.z + a.w + b.x + b.y + b.z + b.w;
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = red[0];
}

// Exclusive scan of the block sums (one work-group; nblk <= 4096 for nmesh <= 2048).
__global__ void __launch_bounds__(1024) k_scan_top(uint32_t* __restrict__ bsum, int nblk) {
  __shared__ uint32_t part[1024];
  const int t = threadIdx.x;
  const int per = (nblk + 1023) / 1024;
  uint32_t s = 0;
  for (int i = 0; i < per; ++i) {
    const int j = t * per + i;
    if (j < nblk) s += bsum[j];
  }
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const uint32_t v = t >= off ? part[t - off] : 0u;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  uint32_t run = part[t] - s;
  for (int i = 0; i < per; ++i) {
    const int j = t * per + i;
    if (j < nblk) {
      const uint32_t v = bsum[j];
      bsum[j] = run;
      run += v;
    }
  }
}

// Per block: scan of tile totals + block offset -> start[tile]; per-class cursors.
__global__ void __launch_bounds__(kScanBlock)
k_scan_apply(const uint32_t* __restrict__ cnt, const uint32_t* __restrict__ boff,
             uint32_t* __restrict__ start, uint32_t* __restrict__ cur, int64_t ntiles) {
  __shared__ uint32_t part[kScanBlock];
  const int t = threadIdx.x;
  const int64_t tile = (int64_t)blockIdx.x * kScanBlock + t;
  uint32_t c[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (tile < ntiles) {
    const uint4* c4 = reinterpret_cast<const uint4*>(cnt + tile * 8);
    const uint4 a = c4[0], b = c4[1];
    c[0] = a.x; c[1] = a.y; c[2] = a.z; c[3] = a.w; c[4] = b.x; c[5] = b.y; c[6] = b.z; c[7] = b.w;
  }
  const uint32_t tot = c[0] + c[1] + c[2] + c[3] + c[4] + c[5] + c[6] + c[7];
  part[t] = tot;
  __syncthreads();
  for (int off = 1; off < kScanBlock; off <<= 1) {
    const uint32_t v = t >= off ? part[t - off] : 0u;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  if (tile < ntiles) {
    uint32_t run = boff[blockIdx.x] + part[t] - tot;
    start[tile] = run;
    uint32_t cc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      cc[k] = run;
      run += c[k];
    }
    uint4* o4 = reinterpret_cast<uint4*>(cur + tile * 8);
    o4[0] = make_uint4(cc[0], cc[1], cc[2], cc[3]);
    o4[1] = make_uint4(cc[4], cc[5], cc[6], cc[7]);
  }
}

// Fixed-point sum -> density: the two 32-bit halves combine exactly in double (sums stay
// below 2^53), so the one rounding to float gives the correctly rounded v * 2^-24, as a
// direct 64-bit integer conversion would, in a handful of instructions.
__device__ __forceinline__ float fix_to_float(unsigned long long v) {
  const double d = (double)(uint32_t)(v >> 32) * 4294967296.0 + (double)(uint32_t)v;
  return (float)(d * (1.0 / kFix));
}

template <int T>
__global__ void __launch_bounds__(kDepositThreads)
k_deposit_tiles(const CicRec* __restrict__ entries, const uint32_t* __restrict__ start,
                const uint32_t* __restrict__ cnt, BinGeo g, float* __restrict__ rho, int rpitch,
                int64_t rplane, float mass) {
  // 64-bit fixed-point accumulation in units of 2^-24: integer LDS atomics run several
  // times faster than float ones here, and integer sums do not depend on the order of
  // the particles, so the density mesh is bitwise reproducible.  A contribution is at
  // most the particle mass (nmesh/np)^3 <= 64 (< 2^32 units), and a cell overflows only
  // beyond ~10^12 in mean-density units.
  __shared__ unsigned long long acc[T * T * T];
  const int nt1 = g.nt1;
  const int tile = (int)xcd_block(blockIdx.x, gridDim.x);
  const int tx = tile / (nt1 * nt1), ty = (tile / nt1) % nt1, tz = tile % nt1;
  for (int i = threadIdx.x; i < T * T * T; i += blockDim.x) acc[i] = 0ull;
  // Flatten the (offset d, class c) segments that reach this tile into one list, so the
  // entries are read in a single strided sweep: the whole own tile (d = 0) and, from the
  // lower neighbour T - d, every class c with (c & d) == d (at most 1 + 19 segments).
  // Wave 0 builds it with one lane per (d, c): class offsets inside the source tile by an
  // 8-lane scan, list positions by ballot, list offsets by a wave scan.
  __shared__ uint32_t sb[20], so[21];
  __shared__ int sdd[20], nseg;
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x, d = lane >> 3, c = lane & 7;
    const int sx = (tx - (d & 1) + nt1) % nt1, sy = (ty - ((d >> 1) & 1) + nt1) % nt1,
              sz = (tz - ((d >> 2) & 1) + nt1) % nt1;
    const int64_t src = ((int64_t)sx * nt1 + sy) * nt1 + sz;
    const uint32_t nc = cnt[src * 8 + c], st0 = start[src];
    uint32_t incl = nc;   // inclusive scan over the 8 classes of the source tile
#pragma unroll
    for (int o = 1; o < 8; o <<= 1) {
      const uint32_t t = __shfl_up(incl, o, 8);
      if (c >= o) incl += t;
    }
    const uint32_t tot = __shfl(incl, 7, 8);
    const bool valid = d == 0 ? (c == 0 && tot > 0) : ((c & d) == d && nc > 0);
    const uint32_t n = d == 0 ? tot : nc;
    const unsigned long long vm = __ballot(valid);
    const int pos = __popcll(vm & ((1ull << lane) - 1ull));
    uint32_t x = valid ? n : 0u;   // inclusive scan of the segment lengths over the wave
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t t = __shfl_up(x, o, 64);
      if (lane >= o) x += t;
    }
    if (valid) {
      sb[pos] = d == 0 ? st0 : st0 + incl - nc;
      so[pos] = x - n;
      sdd[pos] = d;
    }
    if (lane == 63) {
      nseg = __popcll(vm);
      so[__popcll(vm)] = x;
    }
  }
  __syncthreads();
  const uint32_t total = so[nseg];
  int sg = 0;
  // batches of KB records per thread: all loads are issued before the LDS accumulation
  constexpr int KB = 4;
  for (uint32_t e0 = threadIdx.x; e0 < total; e0 += KB * blockDim.x) {
    CicRec r[KB];
    int dd[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const uint32_t e = e0 + k * blockDim.x;
      dd[k] = -1;
      r[k] = CicRec{0u, 0u, 0u};
      if (e < total) {
        while (so[sg + 1] <= e) ++sg;
        dd[k] = sdd[sg];
        r[k] = entries[sb[sg] + (e - so[sg])];
      }
    }
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const int d = dd[k];
      if (d < 0) continue;
      // the lower corner of a particle of tile T - d lies at (home-tile coordinate - T)
      // on every axis where d is set
      const int lx0 = (int)(r[k].x >> 28) - ((d & 1) ? T : 0);
      const int ly0 = (int)(r[k].y >> 28) - (((d >> 1) & 1) ? T : 0);
      const int lz0 = (int)(r[k].z >> 28) - (((d >> 2) & 1) ? T : 0);
      const float dx = rec_d(r[k].x), dy = rec_d(r[k].y), dz = rec_d(r[k].z);
      const float wx[2] = {1.f - dx, dx}, wy[2] = {1.f - dy, dy}, wz[2] = {1.f - dz, dz};
#pragma unroll
      for (int o = 0; o < 8; ++o) {
        const int lx = lx0 + (o & 1), ly = ly0 + ((o >> 1) & 1), lz = lz0 + ((o >> 2) & 1);
        if (lx >= 0 && lx < T && ly >= 0 && ly < T && lz >= 0 && lz < T)
          atomicAdd(&acc[(lx * T + ly) * T + lz],
                    (unsigned long long)__float2uint_rn(
                        mass * wx[o & 1] * wy[(o >> 1) & 1] * wz[(o >> 2) & 1] * kFix));
      }
    }
  }
  __syncthreads();
  // 16-byte stores: T, the row pitch and the plane stride are multiples of 4 floats
  const int ox = tx * T, oy = ty * T, oz = tz * T;
  for (int i4 = threadIdx.x; i4 < T * T * T / 4; i4 += blockDim.x) {
    const int i = 4 * i4;
    const int lx = i / (T * T), ly = (i / T) % T, lz = i % T;
    *reinterpret_cast<float4*>(rho + (int64_t)(ox + lx) * rplane + (int64_t)(oy + ly) * rpitch + oz + lz) =
        make_float4(fix_to_float(acc[i]), fix_to_float(acc[i + 1]), fix_to_float(acc[i + 2]),
                    fix_to_float(acc[i + 3]));
  }
}

void launch_deposit(const Layout& L, const float* disp, float* rho, void* bins, void* entries_raw,
                    hipStream_t s) {
  CicRec* entries = static_cast<CicRec*>(entries_raw);
  BinGeo g;
  g.np = L.np;
  g.nm = L.nm;
  g.ratio = L.nm / L.np;
  g.nt1 = L.nt1;
  g.tile = L.tile;
  g.inv_cell = L.inv_cell;
  g.N = L.N;
  g.lt = ilog2(L.tile);
  const bool p2 = is_pow2(L.np) && is_pow2(L.nm);
  g.lnp = p2 ? ilog2(L.np) : -1;
  g.lnm = p2 ? ilog2(L.nm) : -1;
  const int64_t nblk = (L.ntiles + kScanBlock - 1) / kScanBlock;
  uint32_t* cnt = static_cast<uint32_t*>(bins);
  uint32_t* cur = cnt + 8 * L.ntiles;
  uint32_t* start = cur + 8 * L.ntiles;
  uint32_t* bsum = start + L.ntiles;
  const int64_t nbricks = (int64_t)((L.np + kBrickX - 1) / kBrickX) *
                          ((L.np + kBrickY - 1) / kBrickY) * ((L.np + kBrickZ - 1) / kBrickZ);
  const unsigned bricks = (unsigned)((nbricks + kBinBricks - 1) / kBinBricks);
  {
    ProfScope ps("bin_count", s);
    hipLaunchKernelGGL(k_fill, dim3(grid_for(8 * L.ntiles, 256)), dim3(256), 0, s,
                       reinterpret_cast<float*>(cnt), 8 * L.ntiles, 0.f);
    if (p2)
      hipLaunchKernelGGL((k_bin<0, true>), dim3(bricks), dim3(256), 0, s, disp, g, cnt, cur, entries);
    else
      hipLaunchKernelGGL((k_bin<0, false>), dim3(bricks), dim3(256), 0, s, disp, g, cnt, cur, entries);
    COLA_LAUNCH_CHECK();
  }
  {
    ProfScope ps("bin_scan", s);
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nblk), dim3(256), 0, s, cnt, bsum, L.ntiles);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, bsum, (int)nblk);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nblk), dim3(kScanBlock), 0, s, cnt, bsum, start,
                       cur, L.ntiles);
    COLA_LAUNCH_CHECK();
  }
  {
    ProfScope ps("bin_scatter", s);
    if (p2)
      hipLaunchKernelGGL((k_bin<1, true>), dim3(bricks), dim3(256), 0, s, disp, g, cnt, cur, entries);
    else
      hipLaunchKernelGGL((k_bin<1, false>), dim3(bricks), dim3(256), 0, s, disp, g, cnt, cur, entries);
    COLA_LAUNCH_CHECK();
  }
  ProfScope ps("deposit", s);
  const float mass = (float)g.ratio * g.ratio * g.ratio;
  const dim3 grid((unsigned)L.ntiles), block(kDepositThreads);
  switch (L.tile) {
    case 16: hipLaunchKernelGGL(k_deposit_tiles<16>, grid, block, 0, s, entries, start, cnt, g, rho, 2 * L.pitch_m, 2 * L.plane_m, mass); break;
    case 8: hipLaunchKernelGGL(k_deposit_tiles<8>, grid, block, 0, s, entries, start, cnt, g, rho, 2 * L.pitch_m, 2 * L.plane_m, mass); break;
    default: hipLaunchKernelGGL(k_deposit_tiles<4>, grid, block, 0, s, entries, start, cnt, g, rho, 2 * L.pitch_m, 2 * L.plane_m, mass); break;
  }
  COLA_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ gather + kick + drift
struct GatherDev {
  const float* F3;   // interleaved force mesh, 3 floats per cell, unpadded rows
  float* disp; float* vel;
  const float* psi1; const float* psi2;
  const float* l3; const float* d3;   // interleaved L'' and Delta (MODE 1)
  const double* table; int64_t slice0, slice1;
  float dtk, dtd;
  float* force_out;
  const StepDev* steps; const int* step_ctr;
};

// F_p = sum_corners W F_j (same CIC weights as the deposit); then
// v += dtk (F_p - L''(q_p)), u += dtd v + Delta(q_p)   (kick-drift about the LPT path).
// MODE 0: scale-independent LPT (Psi1, Psi2 per particle, growth scalars from the table);
// MODE 1: scale-dependent LPT (L'' and Delta fields on the particle grid);
// MODE 2: force only (write F_p).
//
// Work order.  Each wave takes 64 consecutive particles of one Lagrangian z-line, so its
// particle loads and (early on) its mesh rows are contiguous.  When the lattice allows
// (np a multiple of 64 and of kGatherBrick), the waves of one XCD are further grouped into
// bricks of kGatherBrick x kGatherBrick z-lines of 64 particles, taken brick after brick:
// the particles an XCD has in flight then form a compact Lagrangian region rather than a
// sheet of one lattice plane, and late in the run, when the particles of a halo come from
// many lattice planes, their force cells are fetched once into that XCD's L2 and reused.
// Otherwise blocks take consecutive particles.
constexpr int kGatherBrick = 16;

template <int MODE>
__global__ void __launch_bounds__(256)
k_gather(GatherDev g, int64_t N, int np, int nm, int ratio, float inv_cell, int bricks) {
  if (MODE != 2 && g.steps) {
    const StepDev& sd = g.steps[*g.step_ctr];
    g.dtk = sd.dtk;
    g.dtd = sd.dtd;
    g.slice0 = sd.slice0;
    g.slice1 = sd.slice1;
  }
  const unsigned blk = xcd_block(blockIdx.x, gridDim.x);
  int64_t p;
  if (bricks) {
    constexpr int kBlocksPerBrick = kGatherBrick * kGatherBrick / 4;
    const int nbz = np / 64, nby = np / kGatherBrick;
    const int brick = (int)(blk / kBlocksPerBrick);
    const int line = (int)(blk % kBlocksPerBrick) * 4 + (int)(threadIdx.x >> 6);
    const int bz = brick % nbz, by = (brick / nbz) % nby, bx = brick / (nbz * nby);
    const int ix = bx * kGatherBrick + line / kGatherBrick, iy = by * kGatherBrick + line % kGatherBrick;
    p = ((int64_t)ix * np + iy) * np + bz * 64 + (threadIdx.x & 63);
  } else {
    p = blk * (int64_t)blockDim.x + threadIdx.x;
  }
  if (p >= N) return;
  // the particle's own values (velocity, LPT terms) do not depend on its cell: their
  // loads go out first, so that they are in flight while the force corners are fetched
  float uu[3], vv[3], l[3], d[3], s1[3], s2[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) uu[a] = g.disp[a * N + p];
  if (MODE != 2) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      vv[a] = g.vel[a * N + p];
      if (MODE == 0) {
        s1[a] = g.psi1[a * N + p];
        s2[a] = g.psi2[a * N + p];
      } else {
        l[a] = g.l3[3 * p + a];
        d[a] = g.d3[3 * p + a];
      }
    }
  }
  CicCell c;
  {
    const int ip = (int)p;
    const int ix = ip / (np * np), iy = (ip / np) % np, iz = ip % np;
    cic_axis(ix, uu[0], nm, ratio, inv_cell, c.i0[0], c.i1[0], c.w0[0], c.w1[0]);
    cic_axis(iy, uu[1], nm, ratio, inv_cell, c.i0[1], c.i1[1], c.w0[1], c.w1[1]);
    cic_axis(iz, uu[2], nm, ratio, inv_cell, c.i0[2], c.i1[2], c.w0[2], c.w1[2]);
  }
  float f0 = 0.f, f1 = 0.f, f2 = 0.f;
#pragma unroll
  for (int ox = 0; ox < 2; ++ox) {
    const int64_t x = ox ? c.i1[0] : c.i0[0];
    const float wx = ox ? c.w1[0] : c.w0[0];
#pragma unroll
    for (int oy = 0; oy < 2; ++oy) {
      const int64_t y = oy ? c.i1[1] : c.i0[1];
      const float wxy = wx * (oy ? c.w1[1] : c.w0[1]);
      const int64_t row = (x * nm + y) * nm;
      const float* a = g.F3 + 3 * (row + c.i0[2]);
      const float* b = g.F3 + 3 * (row + c.i1[2]);
      const float wa = wxy * c.w0[2], wb = wxy * c.w1[2];
      f0 += wa * a[0] + wb * b[0];
      f1 += wa * a[1] + wb * b[1];
      f2 += wa * a[2] + wb * b[2];
    }
  }
  if (MODE == 2) {
    g.force_out[p] = f0;
    g.force_out[N + p] = f1;
    g.force_out[2 * N + p] = f2;
    return;
  }
  if (MODE == 0) {
    const double* t0 = g.table + g.slice0;
    const double* t1 = g.table + g.slice1;
    const float c1 = (float)t0[2], c2 = (float)t0[5];
    const float e1 = (float)(t1[0] - t0[0]), e2 = (float)(t1[3] - t0[3]);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      l[a] = c1 * s1[a] + c2 * s2[a];
      d[a] = e1 * s1[a] + e2 * s2[a];
    }
  }
  const float fv[3] = {f0, f1, f2};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float v = vv[a] + g.dtk * (fv[a] - l[a]);
    g.vel[a * N + p] = v;
    g.disp[a * N + p] = uu[a] + (g.dtd * v + d[a]);
  }
}

void launch_gather(const Layout& L, const GatherArgs& a, hipStream_t s) {
  GatherDev g;
  g.F3 = a.F3;
  g.disp = a.disp; g.vel = a.vel;
  g.psi1 = a.psi1; g.psi2 = a.psi2;
  g.l3 = a.lpp3; g.d3 = a.dlt3;
  g.table = a.table; g.slice0 = a.slice0; g.slice1 = a.slice1;
  g.dtk = (float)a.dtk; g.dtd = (float)a.dtd;
  g.force_out = a.force_out;
  g.steps = a.steps;
  g.step_ctr = a.step_ctr;
  const int ratio = L.nm / L.np;
  const dim3 grid((unsigned)((L.N + 255) / 256)), block(256);
  const int bricks = (L.np % 64 == 0 && L.np % kGatherBrick == 0) ? 1 : 0;
  if (a.force_out) {
    ProfScope ps("gather_force", s);
    hipLaunchKernelGGL(k_gather<2>, grid, block, 0, s, g, L.N, L.np, L.nm, ratio, L.inv_cell,
                       bricks);
  } else if (a.psi1) {
    ProfScope ps("gather_kick_drift", s);
    hipLaunchKernelGGL(k_gather<0>, grid, block, 0, s, g, L.N, L.np, L.nm, ratio, L.inv_cell,
                       bricks);
  } else {
    ProfScope ps("gather_kick_drift", s);
    hipLaunchKernelGGL(k_gather<1>, grid, block, 0, s, g, L.N, L.np, L.nm, ratio, L.inv_cell,
                       bricks);
  }
  COLA_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ k-Mouflage source
// X* >= 0 with P_X(X*)^2 X* = R, P_X = 1 + m K0 X^(m-1): Newton on y = ln X of
// f(y) = y + 2 ln P_X(e^y) - ln R, which rises with slope between 1 and 2m - 1, from the
// smaller of the two asymptotic roots; returns P_X(X*)
__device__ __forceinline__ float km_px_at_root(float R, float k0, int m) {
  if (!(R > 0.f)) return 1.f;
  const float mk = (float)m * k0, lr = __logf(R);
  float y = fminf(lr, (lr - 2.f * __logf(mk)) / (float)(2 * m - 1));
  float px = 1.f;
  for (int it = 0; it < 24; ++it) {
    const float t = mk * __expf((float)(m - 1) * y);   // m K0 X^(m-1)
    px = 1.f + t;
    const float f = y + 2.f * __logf(px) - lr;
    const float fp = 1.f + 2.f * (float)(m - 1) * t / px;
    y -= f / fp;
  }
  return 1.f + mk * __expf((float)(m - 1) * y);
}

__global__ void k_kmouflage_source(const float* __restrict__ rho, const float* __restrict__ f3,
                                   float* __restrict__ out, float* __restrict__ s_out, int n,
                                   int rpitch, int64_t rplane, KmArgs k) {
  if (k.steps) {
    const StepDev& sd = k.steps[*k.step_ctr];
    k.km_r = sd.km_r;
    k.cn = sd.cn;
    k.c5 = sd.c5;
  }
  const int64_t total = (int64_t)n * n * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / n;
    const int64_t pe = (r / n) * rplane + (r % n) * rpitch + (e - r * n);
    const float fx = f3[3 * e], fy = f3[3 * e + 1], fz = f3[3 * e + 2];
    const float px = km_px_at_root(k.km_r * (fx * fx + fy * fy + fz * fz), k.k0, k.m);
    const float eps = fminf(1.f, 1.f / px);
    const float dl = rho[pe] - 1.f;
    out[pe] = dl * (k.cn + k.c5 * eps);
    if (s_out) s_out[pe] = dl * eps;
  }
}

void launch_kmouflage_source(const Layout& L, const float* rho, const float* f3, float* out,
                             float* s_out, const KmArgs& k, hipStream_t s) {
  ProfScope ps("kmouflage_source", s);
  hipLaunchKernelGGL(k_kmouflage_source, dim3(grid_for(L.M, 256)), dim3(256), 0, s, rho, f3, out,
                     s_out, L.nm, 2 * L.pitch_m, 2 * L.plane_m, k);
  COLA_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ step table and counter
__global__ void k_write_step(StepDev* steps, int i, StepDev v) { steps[i] = v; }
__global__ void k_set_counter(int* ctr, int v) { *ctr = v; }
__global__ void k_step_advance(int* ctr) { *ctr += 1; }

void launch_write_step(StepDev* steps, int i, const StepDev& v, hipStream_t s) {
  hipLaunchKernelGGL(k_write_step, dim3(1), dim3(1), 0, s, steps, i, v);
  COLA_LAUNCH_CHECK();
}
void launch_set_counter(int* ctr, int v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_counter, dim3(1), dim3(1), 0, s, ctr, v);
  COLA_LAUNCH_CHECK();
}
void launch_step_advance(int* ctr, hipStream_t s) {
  hipLaunchKernelGGL(k_step_advance, dim3(1), dim3(1), 0, s, ctr);
  COLA_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ force mesh read-out
__global__ void k_split3(const float* __restrict__ f3, float* __restrict__ flat, int64_t M) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < M;
       i += (int64_t)gridDim.x * blockDim.x) {
    flat[i] = f3[3 * i];
    flat[M + i] = f3[3 * i + 1];
    flat[2 * M + i] = f3[3 * i + 2];
  }
}

void launch_split3(const Layout& L, const float* f3, float* flat, hipStream_t s) {
  ProfScope ps("split3", s);
  hipLaunchKernelGGL(k_split3, dim3(grid_for(L.M, 256)), dim3(256), 0, s, f3, flat, L.M);
  COLA_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ stand-alone k-space op
template <int KIND>
__global__ void __launch_bounds__(256) k_kspace(KOp op, float2* __restrict__ out, int64_t total) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int iz = (int)(e % op.pitch);
    const int64_t r = e / op.pitch;
    const int iy = (int)(r % op.n);
    const int ix = (int)(r / op.n);
    const int64_t idx = ix * op.plane + (int64_t)iy * op.pitch + iz;
    out[idx] = kspace_eval<KIND>(op, ix, iy, iz, idx);
  }
}

void launch_kspace(int kind, const KOp& op, float2* out, hipStream_t s) {
  ProfScope ps("kspace", s);
  const int64_t total = (int64_t)op.n * op.n * op.pitch;
  const dim3 g(grid_for(total, 256)), b(256);
  switch (kind) {
    case K_COPY: hipLaunchKernelGGL(k_kspace<K_COPY>, g, b, 0, s, op, out, total); break;
    case K_POT: hipLaunchKernelGGL(k_kspace<K_POT>, g, b, 0, s, op, out, total); break;
    case K_SMOOTH: hipLaunchKernelGGL(k_kspace<K_SMOOTH>, g, b, 0, s, op, out, total); break;
    case K_FORCE: hipLaunchKernelGGL(k_kspace<K_FORCE>, g, b, 0, s, op, out, total); break;
    default: throw Error{COLA_E_ARG, "unsupported stand-alone k-space operator"};
  }
  COLA_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ 2LPT source pieces
// d0 <- d0 d1 + d0 d2 + d1 d2 ;  acc <- acc - d^2   (S = sum_{i<j} phi_ii phi_jj - phi_ij^2)
__global__ void k_2lpt_diag(float* __restrict__ d0, const float* __restrict__ d1,
                            const float* __restrict__ d2, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float a = d0[i], b = d1[i], c = d2[i];
    d0[i] = a * b + a * c + b * c;
  }
}
__global__ void k_2lpt_sub(float* __restrict__ acc, const float* __restrict__ d, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float x = d[i];
    acc[i] -= x * x;
  }
}
void launch_2lpt_diag(float* d0, const float* d1, const float* d2, size_t n, hipStream_t s) {
  ProfScope ps("2lpt_source", s);
  hipLaunchKernelGGL(k_2lpt_diag, dim3(grid_for(n, 256)), dim3(256), 0, s, d0, d1, d2, (int64_t)n);
  COLA_LAUNCH_CHECK();
}
void launch_2lpt_sub(float* acc, const float* d, size_t n, hipStream_t s) {
  ProfScope ps("2lpt_source", s);
  hipLaunchKernelGGL(k_2lpt_sub, dim3(grid_for(n, 256)), dim3(256), 0, s, acc, d, (int64_t)n);
  COLA_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ layout copies
__global__ void k_unpad3(const float* __restrict__ a0, const float* __restrict__ a1,
                         const float* __restrict__ a2, const float* __restrict__ b0,
                         const float* __restrict__ b1, const float* __restrict__ b2, float alpha,
                         float beta, float* __restrict__ out, int64_t N, int np, int ppitch,
                         int64_t pplane) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < N;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int ip = (int)p;
    const int64_t q = (int64_t)(ip / (np * np)) * pplane + (int64_t)((ip / np) % np) * ppitch + ip % np;
    float x = alpha * a0[q], y = alpha * a1[q], z = alpha * a2[q];
    if (b0) {
      x += beta * b0[q];
      y += beta * b1[q];
      z += beta * b2[q];
    }
    out[p] = x;
    out[N + p] = y;
    out[2 * N + p] = z;
  }
}

void launch_unpad3(const Layout& L, const float* const f0[3], const float* const f1[3], float alpha,
                   float beta, float* out, hipStream_t s) {
  ProfScope ps("unpad", s);
  hipLaunchKernelGGL(k_unpad3, dim3(grid_for(L.N, 256)), dim3(256), 0, s, f0[0], f0[1], f0[2],
                     f1 ? f1[0] : nullptr, f1 ? f1[1] : nullptr, f1 ? f1[2] : nullptr, alpha, beta,
                     out, L.N, L.np, 2 * L.pitch_p, 2 * L.plane_p);
  COLA_LAUNCH_CHECK();
}

// u = D1(a_0) Psi1 + D2(a_0) Psi2 with the growth factors read from table slice 0
__global__ void k_combine_u0(const float* __restrict__ psi1, const float* __restrict__ psi2,
                             const double* __restrict__ t0, float* __restrict__ disp, int64_t n3) {
  const float c1 = (float)t0[0], c2 = (float)t0[3];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n3;
       i += (int64_t)gridDim.x * blockDim.x)
    disp[i] = c1 * psi1[i] + c2 * psi2[i];
}

void launch_combine_u0(const Layout& L, const float* psi1, const float* psi2, const double* table,
                       float* disp, hipStream_t s) {
  ProfScope ps("combine_u0", s);
  hipLaunchKernelGGL(k_combine_u0, dim3(grid_for(3 * L.N, 256)), dim3(256), 0, s, psi1, psi2, table,
                     disp, 3 * L.N);
  COLA_LAUNCH_CHECK();
}

__global__ void k_unpad_mesh(const float* __restrict__ in, float* __restrict__ out, int n,
                             int rpitch, int64_t rplane, float sub) {
  const int64_t total = (int64_t)n * n * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / n;
    out[e] = in[(r / n) * rplane + (r % n) * rpitch + (e - r * n)] - sub;
  }
}

void launch_unpad_mesh(const Layout& L, const float* padded, float* flat, hipStream_t s, float sub) {
  ProfScope ps("unpad_mesh", s);
  hipLaunchKernelGGL(k_unpad_mesh, dim3(grid_for(L.M, 256)), dim3(256), 0, s, padded, flat, L.nm,
                     2 * L.pitch_m, 2 * L.plane_m, sub);
  COLA_LAUNCH_CHECK();
}

// x = (q + u) mod L
__global__ void k_positions(const float* __restrict__ disp, float* __restrict__ xyz, int64_t N,
                            int np, int nm, int ratio, float inv_cell, float cell) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < N;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int ip = (int)p;
    const int ix[3] = {ip / (np * np), (ip / np) % np, ip % np};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float f = 0.5f + disp[a * N + p] * inv_cell;
      const float fl = floorf(f);
      int i = (ix[a] * ratio + (int)fl) % nm;
      if (i < 0) i += nm;
      xyz[a * N + p] = ((float)i + (f - fl)) * cell;
    }
  }
}

void launch_positions(const cola_params& p, const Layout& L, const float* disp, float* xyz,
                      hipStream_t s) {
  ProfScope ps("positions", s);
  hipLaunchKernelGGL(k_positions, dim3(grid_for(L.N, 256)), dim3(256), 0, s, disp, xyz, L.N, L.np,
                     L.nm, L.nm / L.np, L.inv_cell, (float)(p.box / p.nmesh1d));
  COLA_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ power spectrum
// Bin b = floor(|nu| + 1/2) from the integer |nu|^2: b^2 - b < n2 <= b^2 + b.
__device__ __forceinline__ int shell_of(int n2) {
  int b = (int)floorf(sqrtf((float)n2) + 0.5f);
  if (b > 0 && b * b - b >= n2) --b;
  if (n2 > b * b + b) ++b;
  return b;
}

__device__ __forceinline__ float sincf_pi(float x) {   // sin(pi x)/(pi x)
  return x == 0.f ? 1.f : sinpif(x) / (3.14159265358979323846f * x);
}

constexpr int kPkBlocks = 1024;
constexpr int kPkMaxBins = 2048;

// Per block: LDS shell sums of w, w P and w |k| over a grid-stride share of the modes.
// Each mode's terms are formed in FP32 and summed in FP64 (LDS double atomics), so the
// order in which a block's threads add them changes only the last bits of a 53-bit sum.
__global__ void __launch_bounds__(256)
k_pk_partial(const float2* __restrict__ dk, int n, int pitch, int64_t plane, int nbins, float kf,
             float vol,
             double* __restrict__ part_p, double* __restrict__ part_k,
             unsigned* __restrict__ part_w) {
  __shared__ double sp[kPkMaxBins], sk[kPkMaxBins];
  __shared__ unsigned sw[kPkMaxBins];
  for (int b = threadIdx.x; b < nbins; b += blockDim.x) {
    sp[b] = 0.0;
    sk[b] = 0.0;
    sw[b] = 0u;
  }
  __syncthreads();
  const int h = n / 2;
  const int64_t total = (int64_t)n * n * (h + 1);
  const float invM = 1.f / ((float)n * (float)n * (float)n);
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int iz = (int)(e % (h + 1));
    const int64_t r = e / (h + 1);
    const int iy = (int)(r % n), ix = (int)(r / n);
    const int nx = ix < h ? ix : ix - n, ny = iy < h ? iy : iy - n;
    const int n2 = nx * nx + ny * ny + iz * iz;
    if (n2 == 0) continue;
    const int b = shell_of(n2);
    if (b >= nbins) continue;
    const float2 v = dk[ix * plane + (int64_t)iy * pitch + iz];
    const float wx = sincf_pi((float)nx / n), wy = sincf_pi((float)ny / n),
                wz = sincf_pi((float)iz / n);
    const float W = wx * wx * wy * wy * wz * wz;
    const float ar = v.x * invM / W, ai = v.y * invM / W;
    const unsigned w = (iz > 0 && iz < h) ? 2u : 1u;
    atomicAdd(&sp[b], (double)((float)w * vol * (ar * ar + ai * ai)));
    atomicAdd(&sk[b], (double)((float)w * kf * sqrtf((float)n2)));
    atomicAdd(&sw[b], w);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nbins; b += blockDim.x) {
    part_p[(int64_t)blockIdx.x * nbins + b] = sp[b];
    part_k[(int64_t)blockIdx.x * nbins + b] = sk[b];
    part_w[(int64_t)blockIdx.x * nbins + b] = sw[b];
  }
}

// Cross-block reduction per bin in FP64, block after block (a fixed order), with
// Neumaier compensation; each sum leaves as an FP32 pair hi + lo.
__global__ void k_pk_final(const double* __restrict__ part_p, const double* __restrict__ part_k,
                           const unsigned* __restrict__ part_w, int nblk, int nbins,
                           float4* __restrict__ out, unsigned long long* __restrict__ counts) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbins) return;
  double sp = 0.0, cp = 0.0, sk = 0.0, ck = 0.0;
  unsigned long long w = 0;
  for (int i = 0; i < nblk; ++i) {
    const double xp = part_p[(int64_t)i * nbins + b];
    double t = sp + xp;
    cp += (fabs(sp) >= fabs(xp)) ? (sp - t) + xp : (xp - t) + sp;
    sp = t;
    const double xk = part_k[(int64_t)i * nbins + b];
    t = sk + xk;
    ck += (fabs(sk) >= fabs(xk)) ? (sk - t) + xk : (xk - t) + sk;
    sk = t;
    w += part_w[(int64_t)i * nbins + b];
  }
  const double P = sp + cp, K = sk + ck;
  const float ph = (float)P, kh = (float)K;
  out[b] = make_float4(ph, (float)(P - (double)ph), kh, (float)(K - (double)kh));
  counts[b] = w;
}

size_t pk_scratch_bytes(const Layout&, int nbins) {
  return align_up((size_t)kPkBlocks * nbins * (2 * sizeof(double) + sizeof(unsigned)));
}

void launch_pk(const Layout& L, const float2* dk, int nbins, void* scratch, float4* out,
               unsigned long long* counts, hipStream_t s) {
  if (nbins > kPkMaxBins) throw Error{COLA_E_ARG, "nbins exceeds 2048"};
  double* part_p = static_cast<double*>(scratch);
  double* part_k = part_p + (size_t)kPkBlocks * nbins;
  unsigned* part_w = reinterpret_cast<unsigned*>(part_k + (size_t)kPkBlocks * nbins);
  const float kf = (float)(2.0 * M_PI / L.box);
  const float vol = (float)(L.box * L.box * L.box);
  {
    ProfScope ps("pk_bin", s);
    hipLaunchKernelGGL(k_pk_partial, dim3(kPkBlocks), dim3(256), 0, s, dk, L.nm, L.pitch_m, L.plane_m, nbins,
                       kf, vol, part_p, part_k, part_w);
    COLA_LAUNCH_CHECK();
  }
  ProfScope ps("pk_final", s);
  hipLaunchKernelGGL(k_pk_final, dim3((nbins + 63) / 64), dim3(64), 0, s, part_p, part_k, part_w,
                     kPkBlocks, nbins, out, counts);
  COLA_LAUNCH_CHECK();
}

}  // namespace cola
