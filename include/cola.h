/*
 * cola.h -- C ABI of libcola, an MI355X (gfx950) implementation of the particle-mesh
 * hot path of COLA with scale-dependent growth and approximate screening
 * (Winther, Koyama, Manera, Wright & Zhao, arXiv:1703.00879).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Units: lengths in Mpc/h, time in 1/H0, super-comoving time d tau = dt/a^2 (Sec. 2).
 * Particles: N = np1d^3, stored in row-major Lagrangian order p = (ix*np1d + iy)*np1d + iz,
 *   with Lagrangian position q = (L/np1d)*(ix,iy,iz) + cell/2 (cell = L/nmesh1d).
 *   The state holds FP32 structure-of-arrays displacements u = x - q (never wrapped)
 *   and FP32 residual velocities v = d(delta x)/d tau about the LPT path (Sec. 2).
 * Memory: the library allocates nothing.  Every buffer is caller-owned device memory
 *   whose size comes from cola_query_sizes(); the state struct is caller-owned host
 *   memory holding those device pointers and the step counter.
 * Streams: every call enqueues work on the caller's stream and returns without
 *   synchronising, except cola_power_spectrum (writes host arrays) and the
 *   profiling read-out.
 * Errors: every call returns a cola_status; on error nothing has been enqueued and
 *   outputs are untouched; cola_last_error() gives a message for the calling thread.
 * Concurrency: different states may be used from different streams at once; calls on
 *   one state must be serialised by the caller.
 */
#ifndef COLA_H
#define COLA_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t cola_status;
#define COLA_OK 0
#define COLA_E_ARG (-1)          /* invalid parameter or NULL pointer */
#define COLA_E_SIZE (-2)         /* buffer too small / size overflow */
#define COLA_E_STATE (-3)        /* call out of order (e.g. step before make_ic) */
#define COLA_E_HIP (-4)          /* a HIP runtime call failed */
#define COLA_E_UNSUPPORTED (-5)  /* valid request the library does not implement */

/* Gravity models (Sec. 5, App. C): LCDM, Hu-Sawicki f(R) with n = 1, normal-branch DGP,
 * the symmetron, and the general {m(a), beta(a)} model given by tables, both of the
 * latter with potential screening. */
#define COLA_LCDM 0
#define COLA_FR_HS1 1
#define COLA_NDGP 2
#define COLA_SYMMETRON 3
#define COLA_MBETA 4        /* general {m(a), beta(a)} model given as tables (App. C) */
#define COLA_KMOUFLAGE 5    /* k-Mouflage: gradient screening (App. B) */
#define COLA_MBETA_MAX_KNOTS 64

/* Fourier-space smoothing windows for density (Vainshtein) screening (App. B). */
#define COLA_SMOOTH_GAUSS 0
#define COLA_SMOOTH_TOPHAT 1
#define COLA_SMOOTH_SHARPK 2

/* Bit flags of cola_params.readings: alternative readings of passages the paper leaves
 * ambiguous.  With readings = 0 the library takes these readings:
 *  - Vainshtein x (Sec. 6.2) = 8 (r_c H0)^2 Omega_m delta_R / (9 beta^2 a^3), delta_R the
 *    smoothed density contrast clamped at -1: the spherical solution of the nDGP field
 *    equation (eq. ndgpfieldeq) makes x proportional to the mean overdensity inside the
 *    radius, and kappa over the a^4 of its nonlinear term leaves a^-3;
 *  - the second-order growth source uses D1(k, a)^2, as printed (Sec. 4.2, App. B). */
#define COLA_READ_X_TOTAL_DENSITY 1  /* x from rho/rho_bar = 1 + delta_R, as printed */
#define COLA_READ_X_NO_A3 2          /* x without the a^-3, as printed */
#define COLA_READ_D2_HALF_K 4        /* D2 source D1(k/sqrt2, a)^2: the k1 = k2 = k/sqrt2 of gamma_2 */
#define COLA_READ_ALL 7

/* Run parameters.  Background: flat LCDM (App. B).  Initial power: Eisenstein-Hu
 * no-wiggle shape normalised to sigma8 of linear LCDM at z = 0 and scaled back to
 * a_ini with the LCDM growth factor.  Model inputs per Sec. 5; screening per Sec. 6.
 * growth_mode 0 uses the model's own D1(k,a), D2(k,a) (Sec. 4); 1 uses the LCDM
 * growth factors with the modified force (Sec. 7.1).
 * Valid ranges (else COLA_E_ARG): 0 < omega_m <= 1, 0 <= omega_b < omega_m, h > 0,
 * sigma8 > 0, t_cmb > 0, np1d and nmesh1d of the form 2^a 3^b with b <= 1,
 * 8 <= np1d <= 1024, np1d <= nmesh1d <= min(2048, 4 np1d), nmesh1d a multiple of np1d,
 * box > 0, z_init > 0,
 * 1 <= n_steps <= 4096, fr0_abs > 0 for f(R), rc_h0 > 0 for nDGP, sym_beta >= 0,
 * sym_mass > 0 and 0 < sym_astar < 1 for the symmetron, r_smooth >= 0, filter in 0..2,
 * model in 0..5, growth_mode in 0..1, screening in 0..1, readings & ~COLA_READ_ALL = 0;
 * for COLA_KMOUFLAGE km_beta >= 0, km_k0 > 0, 2 <= km_m <= 8, km_lambda >= 0, km_x0 >= 0;
 * for COLA_MBETA 4 <= mb_n <= COLA_MBETA_MAX_KNOTS, mb_lna strictly ascending with
 * mb_lna[0] <= ln a_ini and mb_lna[mb_n - 1] >= 0, mb_beta >= 0, mb_m2 > 0, all finite. */
typedef struct cola_params {
  double omega_m, omega_b, h, n_s, sigma8, t_cmb;
  double fr0_abs;     /* |f_R0| of Hu-Sawicki f(R) (Sec. 5.1) */
  double rc_h0;       /* r_c H0 of nDGP (Sec. 5.2) */
  double r_smooth;    /* smoothing radius R for Vainshtein screening, Mpc/h (Sec. 6.2) */
  double box;         /* L, Mpc/h */
  double z_init;      /* initial redshift; a_ini = 1/(1 + z_init) */
  uint64_t seed;      /* seed of the counter-based white noise */
  int32_t model, screening, filter, growth_mode;
  int32_t np1d, nmesh1d, n_steps;
  int32_t readings;   /* COLA_READ_* bit flags; 0 = the readings stated above */
  /* symmetron (App. C): beta(a) = sym_beta sqrt(s), m^2(a) = (sym_mass H0)^2 s with
   * s = 1 - (sym_astar / a)^3 after a = sym_astar, beta = m = 0 before; the field equation
   * couples with C = 2 beta^2 and screens with eps = min(1, |Phi_crit/Phi_N|), Phi_crit the
   * App. C integral 3 Omega_m / (sym_astar^3 sym_mass^2) */
  double sym_beta;    /* beta_star */
  double sym_mass;    /* m_star / H0 (dimensionless; 2997.92458 is a 1 Mpc/h range) */
  double sym_astar;   /* a_star */
  /* general {m(a), beta(a)} model (App. C): beta(a) and m^2(a)/H0^2 at mb_n knots ln a;
   * interpolated by natural cubic splines of beta and of ln(m^2/H0^2) in ln a.  mu =
   * 1 + 2 beta^2 k^2/(k^2 + a^2 m^2), gamma_2^E from m^2, dm^2/da and beta (App. C), the
   * field equation couples with C = 2 beta^2 and screens with eps = min(1, |Phi_crit/Phi_N|),
   * Phi_crit(a) = (9 Omega_m / (2 beta(a))) int_{a_0}^{a} beta / ((m^2/H0^2) a'^4) da' from the
   * first knot a_0 (where Phi_crit = 0), by quadrature */
  int32_t mb_n, mb_reserved;
  double mb_lna[COLA_MBETA_MAX_KNOTS];
  double mb_beta[COLA_MBETA_MAX_KNOTS];
  double mb_m2[COLA_MBETA_MAX_KNOTS];
  /* k-Mouflage (App. B) with the kinetic function P(X) = -1 + X + km_k0 X^km_m: the fifth
   * force is massless with C = 2 km_beta^2 and screened by eps = min(1, 1/P_X(X*)), where
   * P_X(X*)^2 X* = (km_lambda |grad Phi_N|)^2, Phi_N the dimensionless Newtonian potential
   * and km_lambda in Mpc/h; linear growth mu = 1 + 2 km_beta^2 / P_X(X(a)) with the
   * cosmological X(a) = km_x0 a^km_xn, gamma_2 = 0 */
  double km_beta, km_k0, km_lambda, km_x0, km_xn;
  int32_t km_m, km_reserved;
} cola_params;

/* Byte sizes of the caller-owned device buffers of one state. */
typedef struct cola_sizes {
  size_t disp_bytes;    /* float [3][N] */
  size_t vel_bytes;     /* float [3][N] */
  size_t lpt_bytes;     /* LPT store.  k-independent growth: Psi1 float [3][N] at byte 0
                           and Psi2 float [3][N] at byte disp_bytes.  Scale-dependent
                           growth: phi1_k and phi2_k, padded half-complex fields on the
                           particle grid, the second at half of lpt_bytes */
  size_t tables_bytes;  /* FP64 growth tables, FFT twiddles, reduction scratch */
  size_t work_bytes;    /* PM meshes and particle-grid temporaries */
  size_t total_bytes;
} cola_sizes;

/* A run's device state (all pointers caller-owned device memory, 256-byte aligned). */
typedef struct cola_state {
  float* disp;          /* [3][N] u = x - q, Mpc/h */
  float* vel;           /* [3][N] residual velocity about the LPT path */
  void* lpt;
  void* tables;
  void* work;
  int32_t next_step;    /* index i of the next cola_step (a_i -> a_{i+1}); -1 = no IC */
  int32_t prepared;     /* set by cola_prepare / cola_make_ic */
} cola_state;

/* Sizes of every buffer a state with these parameters needs.  Pure host function:
 * no HIP call.  Returns COLA_E_ARG for invalid parameters. */
cola_status cola_query_sizes(const cola_params* p, cola_sizes* out);

/* Validate parameters only (pure host function). */
cola_status cola_validate(const cola_params* p);

/* Build the growth tables (Secs. 4.1-4.2 and App. B: D1'' = kappa mu D1 and the
 * approximate D2 equation with gamma_2 at k1 = k2 = k/sqrt(2), solved per integer
 * |nu|^2 of the particle grid in FP64 on the GPU) and the FFT twiddles.  Sets
 * st->prepared; leaves the particles untouched. */
cola_status cola_prepare(const cola_params* p, cola_state* st, hipStream_t stream);

/* 2LPT initial conditions (Secs. 3-4): seeded white noise -> delta_k with the initial
 * spectrum -> phi1_k = delta_k/k^2 -> the 2LPT source of eq. (lcdm2lpt) -> phi2_k
 * = -S_k/k^2; u = Psi_LPT(q, a_ini) = Psi1 - (3/7) Psi2, v = 0.  Stores the LPT fields
 * (per particle for k-independent growth, in Fourier space for scale-dependent
 * growth, App. A) and sets next_step = 0.  Calls cola_prepare if needed. */
cola_status cola_make_ic(const cola_params* p, cola_state* st, hipStream_t stream);

/* Particle-mesh force at scale factor a for the current displacements (Secs. 2, 6):
 * CIC density -> FFT -> Newtonian potential plus the screened linear fifth force
 * nabla^2 phi = a^2 m^2 phi + C kappa delta eps_screen, eps evaluated in real space
 * -> F = -grad(Phi_N + phi) by three inverse FFTs -> CIC interpolation.
 * force_out: device float [3][N] or NULL.  mesh_out: device float [5][nmesh^3] or NULL,
 * unpadded row-major meshes (rho = 1 + delta, screened source S = delta eps,
 * F_x, F_y, F_z).  Requires a prepared state; does not change it. */
cola_status cola_pm_force(const cola_params* p, cola_state* st, double a,
                          float* force_out, float* mesh_out, hipStream_t stream);

/* One COLA step a_i -> a_{i+1} (Sec. 2; leapfrog with merged kicks, a_i uniform in a):
 * PM force at x(a_i); v += dtau_kick (F - d^2 Psi_LPT/dtau^2 (q, a_i));
 * u += dtau_drift v + Psi_LPT(q, a_{i+1}) - Psi_LPT(q, a_i).  For scale-dependent
 * growth the LPT terms are rebuilt every step by inverse FFTs of the stored k-space
 * fields times D(k,a) (App. A).  i must equal st->next_step (else COLA_E_STATE);
 * increments it. */
cola_status cola_step(const cola_params* p, cola_state* st, int32_t i, hipStream_t stream);

/* Size of the library's own scratch array: the largest work area cola_step_static runs
 * (cola_sizes.work_bytes; e.g. 64^3 particles on a 128^3 mesh). */
#define COLA_STATIC_WORK_BYTES ((size_t)128 << 20)

/* cola_step without a work buffer, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same step, same kernels and the same results as cola_step; st->work is ignored and may
 * be NULL: the meshes and bins live in a scratch array of COLA_STATIC_WORK_BYTES that the
 * library holds on every device it runs on until the process ends.  The call allocates
 * nothing.  A run whose work_bytes exceed COLA_STATIC_WORK_BYTES gets COLA_E_SIZE before
 * any launch.  All calls on one device share its array, so calls that overlap on one
 * device (different streams, or host threads) race: serialise them.  The initial
 * conditions still need cola_make_ic with a work buffer, which may be shared by runs. */
cola_status cola_step_static(const cola_params* p, cola_state* st, int32_t i, hipStream_t stream);

/* Ensembles (the mock catalogues the method is for, Sec. 1): runs stepped together.
 * One step of every member with steps left is captured as one HIP graph, each member a
 * branch on one of n_streams capture streams (default priority), and the graph is
 * replayed while the same members have steps left; then a graph of the remaining members
 * is captured, until every member reaches z = 0.  Every step is the same kernels with the
 * same per-step values as cola_step (taken from the state's step table at the state's
 * device step counter), so each member's result is bitwise that of stepping it alone.
 * cola_ensemble_create: n >= 1 runs, params[j] and states[j] (host arrays; the states
 *   are caller-owned and must outlive the ensemble, each with its own buffers).  The
 *   handle holds host-side objects only (streams and events are made by the first run).
 * cola_ensemble_run: every member needs its initial conditions (cola_make_ic) and may
 *   start at any next_step; 1 <= n_streams <= 64; kernel profiling must be off.  Each
 *   member's next_step ends at n_steps.  Enqueues on `stream` and returns.
 * cola_ensemble_destroy: waits for the ensemble's work, then releases the handle and
 *   the graphs it made (NULL is accepted). */
typedef struct cola_ensemble cola_ensemble;
cola_status cola_ensemble_create(int32_t n, const cola_params* params, cola_state* const* states,
                                 cola_ensemble** out);
cola_status cola_ensemble_run(cola_ensemble* e, int32_t n_streams, hipStream_t stream);
cola_status cola_ensemble_destroy(cola_ensemble* e);

/* Shell-averaged power spectrum of the current particles (the P(k) output of Sec. 8):
 * CIC on the PM mesh, FFT, P_b = < L^3 |delta_k|^2 / (M^2 W_CIC^2) > over shells
 * b = floor(|nu| + 1/2), modes weighted 2 for 0 < nu_z < n/2.  Host outputs k_out,
 * p_out (double [nbins]) and nmodes_out (int64 [nbins], may be NULL); bin 0 (k = 0)
 * is reported as zero power.  Synchronises the stream. */
cola_status cola_power_spectrum(const cola_params* p, cola_state* st, int32_t nbins,
                                double* k_out, double* p_out, int64_t* nmodes_out,
                                hipStream_t stream);

/* Time step i (0 <= i < n_steps) of the leapfrog (Sec. 2), on the host in FP64, no HIP
 * call: out[0] = a_i, out[1] = a_{i+1} (uniform in a from a_ini to 1), out[2] = the kick
 * interval tau(a_{i+1/2}) - tau(a_{i-1/2}) (a_{-1/2} = a_0), out[3] = the drift interval
 * tau(a_{i+1}) - tau(a_i), with d tau = da / (a^3 H/H0) by Gauss-Legendre quadrature.
 * cola_step uses these, rounded to FP32.  COLA_E_ARG for invalid p or i. */
cola_status cola_step_times(const cola_params* p, int32_t i, double* out);

/* Wrapped comoving positions x = (q + u) mod L into device float [3][N]. */
cola_status cola_positions(const cola_params* p, const cola_state* st, float* xyz_out,
                           hipStream_t stream);

/* Copy the FP64 growth table slice of step i (0..n_steps) to host memory:
 * out[k*6 + c] = (D1, D1', D1'', D2, D2', D2'')[c] at a_i for integer |nu|^2 = k,
 * k = 0 .. n_k-1 (n_k = 1 for k-independent growth).  Synchronises.  *n_k_out gets n_k. */
cola_status cola_growth_table(const cola_params* p, const cola_state* st, int32_t i,
                              double* out, int64_t out_len, int64_t* n_k_out,
                              hipStream_t stream);

/* Fill dst (device float, nmesh^3 or np^3 unpadded row-major as chosen by `grid`:
 * 0 = particle grid) with the seeded unit Gaussian white noise the initial
 * conditions use (SplitMix64, Box-Muller).  For checking the generator. */
cola_status cola_white_noise(const cola_params* p, int32_t grid, float* dst,
                             hipStream_t stream);

/* Second-order growth of Fourier triangles k = k1 + k2 at scale factor a, exact and as
 * the path approximates it, for checking the approximation (Sec. 4.2, Fig. 1).  The
 * exact D2(k, k1, k2, a) solves the triangle's own second-order equation with
 * D1(k1) D1(k2), the cos^2 theta term and gamma_2 of the model (Sec. 4); the
 * approximation is D2_hat(k, a)(1 - cos^2 theta), D2_hat being what the growth tables
 * hold.  Cosmology and model come from p; growth_mode 1 gives LCDM growth.
 * tri: device double [n][3] = (|k|, |k1|, |k2|) in h/Mpc.  out: device double [n][2] =
 * (exact, approximation).  A set that is not a triangle (k1, k2 > 0 and
 * |k1 - k2| <= k <= k1 + k2, to 1e-12 relative) gets NaN in both outputs.
 * a_ini <= a <= 10.  Needs no state; n = 0 does nothing. */
cola_status cola_growth_triangles(const cola_params* p, int32_t n, const double* tri, double a,
                                  double* out, hipStream_t stream);

/* FFT tuning.  The Y passes of the 3D transforms (element stride one row pitch) run in
 * tiles of 4, 8 or 16 columns per work-group; each column gets the same butterflies in the
 * same order whatever the width, so every result is bitwise independent of it, and only
 * the speed changes.  The widths are process-wide, per transform size and direction; the
 * default is the widest tile whose 8-byte elements fit 128 KB of LDS.  A graph captured
 * (cola_ensemble_run) keeps the widths in use when it was captured.
 * cola_fft_tiles: n = a supported transform size (8 ... 2048, 2^a 3^b as the mesh);
 *   fwd / inv = 4, 8 or 16 sets the width of the forward / inverse pass, 0 restores the
 *   default, -1 leaves it; COLA_E_ARG if a width does not fit n (more than 1024 threads,
 *   n * width over the plan's elements per thread, or more than 160 KB of LDS), or if n
 *   is not supported.  cur_out (host int32 [2], may be NULL)
 *   receives the widths now in use (forward, inverse).
 * cola_autotune: times every valid width of both directions for the PM mesh and the
 *   particle grid of p on the state's work buffer (its contents are overwritten; the
 *   state must be prepared, and no step of it may be in flight), keeps the fastest and
 *   writes them to out (host int32 [4]: mesh forward, mesh inverse, particle-grid forward,
 *   particle-grid inverse; 0 where the grid was not tuned).  Synchronises the stream. */
cola_status cola_fft_tiles(int32_t n, int32_t fwd, int32_t inv, int32_t* cur_out);
cola_status cola_autotune(const cola_params* p, cola_state* st, int32_t* out, hipStream_t stream);

/* Kernel timing by HIP events on the launch stream: enable (1) / disable (0)
 * recording; read accumulated milliseconds and launch counts per kernel name
 * (synchronises the last recorded stream).  names/ms/counts are host arrays of
 * length cap; returns the number of kernels in *n_out. */
cola_status cola_profile_enable(int32_t on);
cola_status cola_profile_read(char (*names)[48], double* ms, int64_t* counts,
                              int32_t cap, int32_t* n_out);
cola_status cola_profile_reset(void);

const char* cola_status_string(cola_status s);
const char* cola_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* COLA_H */
