// Internal declarations shared by the libcola translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <string>

#include "cola.h"

namespace cola {

// ------------------------------------------------------------------ errors
struct Error {
  cola_status code;
  std::string msg;
};
void set_error(const std::string& msg);
#define COLA_HIP_CHECK(expr)                                                        \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess)                                                           \
      throw ::cola::Error{COLA_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)}; \
  } while (0)
#define COLA_LAUNCH_CHECK() COLA_HIP_CHECK(hipGetLastError())

// ------------------------------------------------------------------ profiling
// Records a pair of events around launches that carry `name` when enabled.
struct ProfScope {
  ProfScope(const char* name, hipStream_t s);
  ~ProfScope();
  const char* name_;
  hipStream_t s_;
  hipEvent_t a_ = nullptr, b_ = nullptr;
};

// ------------------------------------------------------------------ XCD-aware block order
// Work-groups are dispatched round-robin over the 8 XCDs (each with its own L2), so
// block b runs on XCD b % 8.  xcd_block() renumbers blocks so that each XCD works on one
// contiguous range of logical blocks: neighbouring tiles or particle chunks, which share
// cache lines, then meet in the same L2.  It is a bijection on [0, nblocks).
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nblocks) {
  const unsigned q = nblocks >> 3, r = nblocks & 7, x = b & 7, l = b >> 3;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + l;
}

// ------------------------------------------------------------------ layout
constexpr size_t kAlign = 256;
inline size_t align_up(size_t x, size_t a = kAlign) { return (x + a - 1) / a * a; }

// Half-complex row pitch (complex elements): n/2 + 1 rounded up to 16, so every row of
// a padded real or half-complex mesh starts on a 128-byte boundary.
inline int half_pitch(int n) { return (n / 2 + 1 + 15) / 16 * 16; }
// x-plane stride (complex elements): n * pitch plus 16 elements (128 B).  Without the pad
// the stride of the X pass is 33 * 2^17 bytes at n = 1024, and all 1024 elements of a
// column sit at addresses congruent modulo 128 KB (same HBM channel); the odd multiple of
// 128 B spreads them over the channels.
inline int64_t plane_stride(int n) { return (int64_t)n * half_pitch(n) + 16; }

struct Layout {
  int np, nm;               // particle grid and mesh sizes (per dimension)
  double box;               // L, Mpc/h
  float inv_cell;           // nmesh / L
  int64_t N, M;             // particles, mesh cells
  int pitch_p, pitch_m;     // half-complex row pitches
  int64_t plane_p, plane_m; // half-complex x-plane strides
  size_t pgrid_elems;       // float2 elements of a particle-grid half-complex field
  size_t mesh_elems;        // float2 elements of a PM mesh half-complex field
  bool kdep;                // scale-dependent LPT (k-space store)
  int64_t n_k;              // entries per growth-table slice
  int n_steps;
  // offsets (bytes) inside `tables`
  size_t off_growth, off_ref, off_tw_m, off_tw_p, off_scratch, off_lpt_coef, off_steps,
      off_ctr, tables_bytes;
  size_t scratch_bytes;
  // offsets (bytes) inside `work`: six mesh slots (padded half-complex / real meshes);
  // the interleaved force mesh [nm][nm][nm][3] spans slots 3-5, and the sorted CIC
  // records of the deposit reuse slot 5 when they fit there.  Scale-dependent LPT: three
  // particle-grid half-complex work fields and the interleaved L'' and Delta arrays
  // (3 N floats each), over slots 0-2 when they fit there (they are written after the
  // force mesh and read with it by the gather), else in an area of their own.
  size_t off_mesh[6], off_lptw[3], off_lpp3, off_dlt3, work_bytes;
  // binned deposit: tile edge (cells), tiles per axis, tile count, and the offsets of
  // the per-tile counters and of the particle-index list sorted by home tile
  int tile, nt1;
  int64_t ntiles;
  size_t off_bins, off_entries;
  size_t lpt_bytes, disp_bytes;
};
Layout make_layout(const cola_params& p);
void validate(const cola_params& p);   // throws Error{COLA_E_ARG}

// ------------------------------------------------------------------ static scratch
// Size of the library's scratch array (the work area of cola_step_static) and the number
// of devices it keeps addresses for.
constexpr size_t kStaticWorkBytes = COLA_STATIC_WORK_BYTES;
constexpr int kMaxDevices = 64;
// Device address of this device's scratch array (looked up once per device); throws
// Error{COLA_E_SIZE} when `need` exceeds it.
void* static_work(size_t need);

// ------------------------------------------------------------------ general {m, beta} tables
// Natural cubic splines of beta and of ln(m^2/H0^2) over the knots x = ln a of a
// COLA_MBETA run: values and second derivatives at the knots (the second derivatives
// vanish at both ends).  Evaluated the same way on the host and in the growth kernels.
struct MBSpline {
  int n;
  double x[COLA_MBETA_MAX_KNOTS];
  double yb[COLA_MBETA_MAX_KNOTS], Mb[COLA_MBETA_MAX_KNOTS];
  double ym[COLA_MBETA_MAX_KNOTS], Mm[COLA_MBETA_MAX_KNOTS];
};
MBSpline mb_spline(const cola_params& p);   // zero n unless p.model == COLA_MBETA

// beta, m^2/H0^2 and d(m^2/H0^2)/da at scale factor a (the end cubics continue outside
// the knots)
__host__ __device__ inline void mb_eval(const MBSpline& s, double a, double& beta, double& m2,
                                        double& dm2_da) {
  const double x = log(a);
  int lo = 0, hi = s.n - 1;   // interval [x_lo, x_lo+1] holding x, clamped to the ends
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (x < s.x[mid])
      hi = mid;
    else
      lo = mid;
  }
  const double h = s.x[lo + 1] - s.x[lo], t = x - s.x[lo], u = s.x[lo + 1] - x;
  auto val = [&](const double* y, const double* M, double& d) {
    const double c0 = y[lo] / h - M[lo] * h / 6.0, c1 = y[lo + 1] / h - M[lo + 1] * h / 6.0;
    d = -M[lo] * u * u / (2.0 * h) + M[lo + 1] * t * t / (2.0 * h) - c0 + c1;
    return M[lo] * u * u * u / (6.0 * h) + M[lo + 1] * t * t * t / (6.0 * h) + c0 * u + c1 * t;
  };
  double db, dl;
  beta = val(s.yb, s.Mb, db);
  const double lm = val(s.ym, s.Mm, dl);
  m2 = exp(lm);
  dm2_da = m2 * dl / a;
}

// ------------------------------------------------------------------ host physics (FP64)
struct Cosmo {
  double om, ol;
  double E(double a) const;
};
double tau_between(const Cosmo& c, double a0, double a1);
double sigma8_norm(const cola_params& p);        // A with sigma8^2 = A * I
double eh_transfer(const cola_params& p, double k);
struct StepScalars {         // PM-force scalars at scale factor a
  double a;
  float kappa, a2m2, coupling;
  float cham_thr;   // potential screening threshold on |Phi_code|: Phi_crit(a) a^2/(H0/c)^2,
                    // Phi_crit = (3/2)|f_R(a)| for f(R), the App. C integral for the symmetron
  float vx_pref;    // nDGP: x = vx_pref max(-1, delta_R) + vx_off,
                    // vx_pref = 8 (rc H0)^2 Om / (9 beta^2 a^3) (a^3 -> 1 under READ_X_NO_A3)
  float vx_off;     // 0, or vx_pref under COLA_READ_X_TOTAL_DENSITY (x from 1 + delta_R)
  float beta;
  int fifth, screen;  // fifth force on, screening on
};
StepScalars step_scalars(const cola_params& p, double a);
double a_of_step(const cola_params& p, int i);

// The PM force's scalars at scale factor a in the form the kernels take them: the force
// pass's Green's-function coefficients g_n, g_5 and a^2 m^2, the potential-screening X
// pass's -kappa, and the screening row pass's threshold, Vainshtein prefactor and offset
// and source weights (cn + c5 eps).  For nDGP (massless fifth force, Sec. 5.2) the row
// pass folds both sources into (rho - 1)(cn + c5 eps) and the force pass takes that one
// field with g_n = 1.
struct PMScalars {
  float g_n, g_5, a2m2, sop_g_n;
  float thr, vx, vx0, cn, c5;
  float km_r;      // k-Mouflage: (lambda (H0/c)^2 / a^2)^2, turning |F_Newton|^2 into R
  int screen;      // screening on
  int potential;   // potential screening (f(R), symmetron, tabulated {m, beta})
  int gradient;    // gradient screening (k-Mouflage); neither: density screening (nDGP)
};
PMScalars pm_scalars(const cola_params& p, double a);

// Per-step scalars of cola_step i (a_i -> a_{i+1}), built once per run into the tables
// buffer; the step's kernels read entry [*step counter], so one captured step can be
// replayed for every step.  Values equal what the same step computes on the host.
struct StepDev {
  float g_n, g_5, a2m2, sop_g_n;   // PMScalars at a_i
  float thr, vx, vx0, cn, c5;
  float dtk, dtd;                  // kick tau(a_{i+1/2}) - tau(a_{i-1/2}), drift tau(a_{i+1}) - tau(a_i)
  float km_r;
  int64_t slice0, slice1;          // growth-table element offsets of slices i and i + 1
};
StepDev step_dev(const cola_params& p, const Layout& L, int i);
// a_i, a_{i+1} and the kick and drift intervals of step i in FP64 (what step_dev rounds)
void step_times(const cola_params& p, int i, double out[4]);

// ------------------------------------------------------------------ k-space operators
enum KKind : int {
  K_COPY = 0,      // out = scale * a
  K_FORCE = 1,     // out = -i k_c [g_n/k^2 a + g_5/(k^2+a2m2) b] * scale
  K_POT = 2,       // out = g_n/k^2 a * scale
  K_SMOOTH = 3,    // out = W(kR) a * scale (k = 0 -> 0)
  K_LPT = 4,       // out = i k_c (X1 a + X2 b) * scale, X from the growth table
  K_HESS = 5,      // out = -k_i k_j a * scale
  K_GRAD = 6,      // out = i k_c a * scale
  K_INVLAP = 7,    // out = g_n/k^2 a * scale (alias of K_POT with separate name)
};

struct KOp {
  const float2* a = nullptr;
  const float2* b = nullptr;
  const double* table = nullptr;   // growth table base (K_LPT)
  int64_t tab_slice0 = 0, tab_slice1 = 0;   // element offsets of two slices (K_LPT)
  int lpt_mode = 0;                // 0: X = D''(slice0); 1: X = D(slice1) - D(slice0); 2: X = D(slice0)
  const float2* coef = nullptr;    // K_LPT: the step's (X1, X2) per |nu|^2 in FP32, if built
  // when set, the step-dependent coefficients (g_n, g_5, a2m2) come from steps[*step_ctr];
  // with step_newton the force pass takes the Newtonian part alone (g_n = the step's cn)
  const StepDev* steps = nullptr;
  const int* step_ctr = nullptr;
  int step_newton = 0;
  int comp = 0, comp2 = 0;
  float scale = 1.f;
  float kf = 1.f;                  // 2 pi / L
  float g_n = 0.f, g_5 = 0.f, a2m2 = 0.f;
  float r_smooth = 0.f;
  int filter = 0;
  int n = 0, pitch = 0;
  int64_t plane = 0;
  int kdep = 0;                    // growth table indexed by |nu|^2 (else entry 0)
};

// ------------------------------------------------------------------ FFT
struct FFTPlan {
  int n = 0;            // transform size per dimension
  int pitch = 0;        // half-complex row pitch
  int64_t plane = 0;    // half-complex x-plane stride
  const float2* tw = nullptr;   // exp(-2 pi i t / n), t = 0..n-1 (device)
};
bool fft_size_supported(int n);
// forward real-to-complex 3D transform (unnormalised, e^{-ikx}); in may alias out
void fft_r2c(const FFTPlan& pl, const float* in, float2* out, hipStream_t s);
// its Z and Y passes only: the X pass is left to fft_screen / fft_c2r_force3
void fft_r2c_zy(const FFTPlan& pl, const float* in, float2* out, hipStream_t s);
// inverse complex-to-real 3D transform (unnormalised, e^{+ikx}).  The first pass reads
// through the k-space operator `op` (kind) and writes `data`; later passes are in place;
// the real result goes to `out` (may alias data).
void fft_c2r(const FFTPlan& pl, int kind, const KOp& op, float2* data, float* out,
             hipStream_t s);

// Forward X pass of `src` (Z and Y passes done) fused with the inverse force transforms:
// one X pass forms the Green's function g of delta_k and S_k (delta_k read from dk; S_k is
// the forward transform of src; S_k = delta_k when dk is null) and writes X^-1[-i k_x g]
// into work[0] and X^-1[g] into work[1] (both may alias dk and src); the inverse Y passes
// give the x component in work[0] and the y and z components in work[1] and work[2]; one
// real Z pass over all three writes the interleaved force mesh
// f3[((x nm + y) nm + z) 3 + c] (unpadded).
void fft_c2r_force3(const FFTPlan& pl, const KOp& op, const float2* dk, const float2* src,
                    float2* const work[3], float* f3, hipStream_t s);
// The three components of IDFT[i k (c1 phi1_k + c2 phi2_k)] / N on the particle grid (a
// scale-dependent LPT term, App. A), c1 and c2 read per mode from op.coef[|nu|^2]: one X
// pass forms the field from phi1 and phi2 and writes its two X transforms into work[0]
// and work[1] (none may alias phi1 or phi2), then the Y and Z passes of fft_c2r_force3
// write the interleaved rows out3[((x n + y) n + z) 3 + c].  op needs kf, scale and coef.
void fft_c2r_lpt3(const FFTPlan& pl, const KOp& op, const float2* phi1, const float2* phi2,
                  float2* const work[3], float* out3, hipStream_t s);
// Screened source in Fourier space.  dk holds the density contrast after the forward Z
// and Y passes: one X pass completes delta_k (written back in place for K_POT, where the
// force needs it; not kept for K_SMOOTH) and applies `kind` (K_POT: Newtonian potential
// for f(R) and the symmetron; K_SMOOTH: smoothed density for nDGP) on the way back into
// `data`; then the inverse Y pass, one row pass doing inverse Z -> eps -> forward Z of
// (rho - 1) (cn + c5 eps), and the forward Y pass: `data` ends holding that field after
// the forward Z and Y passes (its X pass is done by fft_c2r_force3).  cn = 0, c5 = 1
// give S = delta eps; for a massless fifth force (nDGP) cn = g_n and c5 = g_5 fold the
// Newtonian and fifth-force sources into one field with one Green's function 1/k^2.
// s_out (optional, padded real) receives S = delta eps.
struct ScreenArgs {
  float thr, vx, vx0, cn, c5;      // see PMScalars
  const StepDev* steps = nullptr;  // when set, the five come from steps[*step_ctr]
  const int* step_ctr = nullptr;
};
void fft_screen(const FFTPlan& pl, int kind, const KOp& op, float2* dk, float2* data,
                const float* rho, float* s_out, int model, const ScreenArgs& sa, hipStream_t s);

// Tile widths (columns per work-group) of the Y passes of n-point transforms, per
// direction: fwd / inv = 4, 8 or 16 sets one (COLA_E_ARG if it does not fit LDS or the
// work-group limit at n), 0 restores the default, -1 leaves it.  fft_get_tiles gives the
// widths in use.  fft_autotune times every valid width of both directions on `data` (a
// field of pl's layout; overwritten), keeps the fastest and returns them in out[2].
void fft_set_tiles(int n, int fwd, int inv);
void fft_get_tiles(int n, int out[2]);
void fft_autotune(const FFTPlan& pl, float2* data, hipStream_t s, int out[2]);

// ------------------------------------------------------------------ kernels (launchers)
void launch_fill(float* p, size_t n, float v, hipStream_t s);
void launch_growth_ode(const cola_params& p, const Layout& L, double* table, double* ref,
                       hipStream_t s);
// exact D2 of triangles tri[i] = (k, k1, k2) and D2_hat(k)(1 - cos^2 theta) at a into
// out[i] = (exact, approximation); NaN for sets that are no triangle
void launch_growth_triangles(const cola_params& p, int n, const double* tri, double a, double* out,
                             hipStream_t s);
void launch_noise(const cola_params& p, int n, int pitch, int64_t plane, float* dst_padded,
                  float* dst_flat, hipStream_t s);
void launch_ic_phi1(const cola_params& p, const Layout& L, const float2* wk, float2* phi1,
                    double A_norm, const double* ref, hipStream_t s);
void launch_kspace(int kind, const KOp& op, float2* out, hipStream_t s);
void launch_2lpt_diag(float* d0, const float* d1, const float* d2, size_t n, hipStream_t s);
void launch_2lpt_sub(float* acc, const float* d, size_t n, hipStream_t s);
// out[c][p] = alpha * f0[c](q_p) + beta * f1[c](q_p) from padded particle-grid fields
void launch_unpad3(const Layout& L, const float* const f0[3], const float* const f1[3],
                   float alpha, float beta, float* out, hipStream_t s);
void launch_combine_u0(const Layout& L, const float* psi1, const float* psi2,
                       const double* table, float* disp, hipStream_t s);
// The growth-table values the step's LPT transforms read, rounded once to FP32 per |nu|^2:
// coef[k] = (D1''(a_i), D2''(a_i)) and coef[n_k + k] = (D1(a_i+1) - D1(a_i), D2(a_i+1) -
// D2(a_i)) (differences taken in FP64), from table slices at element offsets slice0/slice1.
void launch_lpt_coef(const Layout& L, const double* table, int64_t slice0, int64_t slice1,
                     const StepDev* steps, const int* ctr, float2* coef, hipStream_t s);
// step table and counter: steps[i] = v; *ctr = v; *ctr += 1 (single-thread kernels)
void launch_write_step(StepDev* steps, int i, const StepDev& v, hipStream_t s);
void launch_set_counter(int* ctr, int v, hipStream_t s);
void launch_step_advance(int* ctr, hipStream_t s);
// k-Mouflage source (App. B): out = (rho - 1)(cn + c5 eps) in the padded real layout, with
// eps = min(1, 1/P_X(X*)), P_X(X*)^2 X* = km_r |F|^2 from the interleaved Newtonian force
// mesh f3; s_out (optional, padded real) gets S = (rho - 1) eps.  With steps set, km_r, cn
// and c5 come from steps[*step_ctr].
struct KmArgs {
  float km_r, k0, cn, c5;
  int m;
  const StepDev* steps = nullptr;
  const int* step_ctr = nullptr;
};
void launch_kmouflage_source(const Layout& L, const float* rho, const float* f3, float* out,
                             float* s_out, const KmArgs& k, hipStream_t s);
// CIC deposit into the padded real mesh.  `bins` is the work area at off_bins, `entries`
// the packed per-particle CIC records sorted by home tile (12 bytes each).
void launch_deposit(const Layout& L, const float* disp, float* rho_padded, void* bins,
                    void* entries, hipStream_t s);
size_t bins_bytes(int64_t ntiles);
struct GatherArgs {
  const float* F3;            // interleaved force mesh (F_x, F_y, F_z) per cell
  float* disp;
  float* vel;
  const float* psi1;          // scale-independent LPT (else null)
  const float* psi2;
  const float* lpp3;          // scale-dependent LPT: L''(q) and Delta(q) per particle,
  const float* dlt3;          // interleaved (3 floats per lattice site, lattice order)
  const double* table;        // growth table (scale-independent coefficients)
  int64_t slice0, slice1;     // element offsets of slices i and i+1
  double dtk, dtd;
  float* force_out;           // cola_pm_force: write F_p instead of updating
  const StepDev* steps;       // when set, dtk, dtd, slice0, slice1 come from steps[*step_ctr]
  const int* step_ctr;
};
void launch_gather(const Layout& L, const GatherArgs& g, hipStream_t s);
// the three components of the interleaved force mesh into flat [3][nm^3]
void launch_split3(const Layout& L, const float* f3, float* flat, hipStream_t s);
// flat = padded - sub over the n^3 valid cells
void launch_unpad_mesh(const Layout& L, const float* padded, float* flat, hipStream_t s,
                       float sub = 0.f);
void launch_positions(const cola_params& p, const Layout& L, const float* disp, float* xyz,
                      hipStream_t s);
// P(k) shell sums with per-block partials and a compensated cross-block reduction.
// Writes out[b] = (sum w P hi, lo, sum w |k| hi, lo) and counts[b] = sum w (device).
size_t pk_scratch_bytes(const Layout& L, int nbins);
void launch_pk(const Layout& L, const float2* dk, int nbins, void* scratch, float4* out,
               unsigned long long* counts, hipStream_t s);

}  // namespace cola
