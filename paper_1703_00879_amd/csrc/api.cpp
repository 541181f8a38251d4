// C ABI of libcola: argument checks, buffer carving, and the order of kernel launches
// for the initial conditions, the PM force, the COLA step and the power spectrum.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace cola {

// ------------------------------------------------------------------ errors
static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

template <class F>
static cola_status guarded(F&& f) {
  try {
    f();
    return COLA_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::exception& e) {
    set_error(e.what());
    return COLA_E_HIP;
  }
}

// ------------------------------------------------------------------ profiling
namespace {
struct Pending {
  const char* name;
  hipEvent_t a, b;
};
struct ProfState {
  std::mutex mu;
  bool on = false;
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  std::map<std::string, std::pair<double, int64_t>> acc;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    COLA_HIP_CHECK(hipEventCreate(&e));
    return e;
  }
  void drain() {   // caller holds mu
    for (auto& p : pending) {
      COLA_HIP_CHECK(hipEventSynchronize(p.b));
      float ms = 0.f;
      COLA_HIP_CHECK(hipEventElapsedTime(&ms, p.a, p.b));
      auto& slot = acc[p.name];
      slot.first += ms;
      slot.second += 1;
      pool.push_back(p.a);
      pool.push_back(p.b);
    }
    pending.clear();
  }
};
ProfState& prof() {
  static ProfState s;
  return s;
}
}  // namespace

ProfScope::ProfScope(const char* name, hipStream_t s) : name_(name), s_(s) {
  ProfState& P = prof();
  if (!P.on) return;
  std::lock_guard<std::mutex> lk(P.mu);
  a_ = P.get();
  b_ = P.get();
  COLA_HIP_CHECK(hipEventRecord(a_, s_));
}

ProfScope::~ProfScope() {
  if (!a_) return;
  ProfState& P = prof();
  std::lock_guard<std::mutex> lk(P.mu);
  if (hipEventRecord(b_, s_) == hipSuccess) P.pending.push_back({name_, a_, b_});
  if (P.pending.size() > 4096) {
    try {
      P.drain();
    } catch (...) {
    }
  }
}

// ------------------------------------------------------------------ buffers of a state
struct Bufs {
  Layout L;
  double* growth;
  double* ref;
  float2* tw_m;
  float2* tw_p;
  void* pk_scratch;
  float4* pk_out;
  unsigned long long* pk_cnt;
  float2* mesh[6];
  float* force;       // interleaved force mesh over slots 3-5
  float2* lptw[3];    // scale-dependent LPT: particle-grid work fields
  float* lpp3;        // and the interleaved L'' and Delta arrays
  float* dlt3;
  float2* phi1;
  float2* phi2;
  float* psi1;
  float* psi2;
  void* bins;
  void* entries;     // the deposit's 12-byte CIC records
  StepDev* steps;     // per-step scalars of every step
  int* ctr;           // device step counter: the step the step kernels read
};

template <class T>
static T* at(void* base, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

static void check_ptr(const void* p, const char* what) {
  if (!p) throw Error{COLA_E_ARG, std::string(what) + " is NULL"};
  if (reinterpret_cast<uintptr_t>(p) % kAlign)
    throw Error{COLA_E_ARG, std::string(what) + " must be 256-byte aligned"};
}

// Device pointers of every buffer of a state.  `work` replaces st->work when given (the
// allocation-free step runs on the library's own scratch array).
static Bufs carve(const cola_params& p, const cola_state* st, void* work = nullptr) {
  if (!st) throw Error{COLA_E_ARG, "state is NULL"};
  Bufs b;
  b.L = make_layout(p);
  const Layout& L = b.L;
  check_ptr(st->disp, "state.disp");
  check_ptr(st->vel, "state.vel");
  check_ptr(st->lpt, "state.lpt");
  check_ptr(st->tables, "state.tables");
  if (!work) {
    check_ptr(st->work, "state.work");
    work = st->work;
  }
  b.growth = at<double>(st->tables, L.off_growth);
  b.ref = at<double>(st->tables, L.off_ref);
  b.tw_m = at<float2>(st->tables, L.off_tw_m);
  b.tw_p = at<float2>(st->tables, L.off_tw_p);
  b.pk_scratch = at<void>(st->tables, L.off_scratch);
  b.pk_out = at<float4>(st->tables, L.off_scratch + pk_scratch_bytes(L, 2048));
  b.pk_cnt = reinterpret_cast<unsigned long long*>(b.pk_out + 2048);
  b.steps = at<StepDev>(st->tables, L.off_steps);
  b.ctr = at<int>(st->tables, L.off_ctr);
  for (int i = 0; i < 6; ++i) b.mesh[i] = at<float2>(work, L.off_mesh[i]);
  b.force = at<float>(work, L.off_mesh[3]);
  for (int i = 0; i < 3; ++i) b.lptw[i] = L.kdep ? at<float2>(work, L.off_lptw[i]) : nullptr;
  b.lpp3 = L.kdep ? at<float>(work, L.off_lpp3) : nullptr;
  b.dlt3 = L.kdep ? at<float>(work, L.off_dlt3) : nullptr;
  b.bins = at<void>(work, L.off_bins);
  b.entries = at<void>(work, L.off_entries);
  if (L.kdep) {
    b.phi1 = at<float2>(st->lpt, 0);
    b.phi2 = at<float2>(st->lpt, align_up(L.pgrid_elems * sizeof(float2)));
    b.psi1 = b.psi2 = nullptr;
  } else {
    b.phi1 = b.phi2 = nullptr;
    b.psi1 = at<float>(st->lpt, 0);
    b.psi2 = at<float>(st->lpt, L.disp_bytes);
  }
  return b;
}

static FFTPlan plan_mesh(const Bufs& b) { return FFTPlan{b.L.nm, b.L.pitch_m, b.L.plane_m, b.tw_m}; }
static FFTPlan plan_part(const Bufs& b) { return FFTPlan{b.L.np, b.L.pitch_p, b.L.plane_p, b.tw_p}; }

static inline float* R(float2* p) { return reinterpret_cast<float*>(p); }

// Twiddle tables exp(-2 pi i t / n) in double precision, rounded once; kept for the life
// of the process so the asynchronous upload never reads freed host memory.
static const std::vector<float2>& twiddles(int n) {
  static std::mutex mu;
  static std::map<int, std::vector<float2>> cache;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(n);
  if (it != cache.end()) return it->second;
  std::vector<float2> t(n);
  for (int i = 0; i < n; ++i) {
    const double ang = -2.0 * M_PI * i / n;
    t[i] = make_float2((float)std::cos(ang), (float)std::sin(ang));
  }
  return cache.emplace(n, std::move(t)).first->second;
}

static void do_prepare(const cola_params& p, cola_state* st, const Bufs& b, hipStream_t s) {
  const auto& tm = twiddles(b.L.nm);
  const auto& tp = twiddles(b.L.np);
  COLA_HIP_CHECK(hipMemcpyAsync(b.tw_m, tm.data(), tm.size() * sizeof(float2), hipMemcpyHostToDevice, s));
  COLA_HIP_CHECK(hipMemcpyAsync(b.tw_p, tp.data(), tp.size() * sizeof(float2), hipMemcpyHostToDevice, s));
  launch_growth_ode(p, b.L, b.growth, b.ref, s);
  for (int i = 0; i < p.n_steps; ++i) launch_write_step(b.steps, i, step_dev(p, b.L, i), s);
  st->prepared = 1;
}

// ------------------------------------------------------------------ PM force core
// Writes the interleaved force mesh (b.force, over slots 3-5).
// mesh[0] holds rho after the deposit; mesh[1] delta after the forward Z and Y passes,
// then delta_k; mesh[2] the screening field and then S after the forward Z and Y passes;
// the three complex force components then take slots 0-2.  If flat_out is given, rho and
// S are copied there before being overwritten.
static void pm_core(const cola_params& p, const Bufs& b, const float* disp, double a,
                    float* flat_out, hipStream_t s, bool from_table = false) {
  const Layout& L = b.L;
  const FFTPlan pl = plan_mesh(b);
  const PMScalars sc = pm_scalars(p, a);
  const StepDev* steps = from_table ? b.steps : nullptr;
  const int* ctr = from_table ? b.ctr : nullptr;
  float2* const* M = b.mesh;
  const float invM = (float)(1.0 / (double)L.M);
  launch_deposit(L, disp, R(M[0]), b.bins, b.entries, s);
  if (flat_out) launch_unpad_mesh(L, R(M[0]), flat_out, s);
  fft_r2c_zy(pl, R(M[0]), M[1], s);   // the X pass is fused into what follows
  const float2* dk = nullptr;
  float2* src = M[1];
  KOp base;
  base.kf = (float)(2.0 * M_PI / p.box);
  base.steps = steps;
  base.step_ctr = ctr;
  KOp op = base;
  op.g_n = sc.g_n;
  op.g_5 = sc.g_5;
  op.a2m2 = sc.a2m2;
  op.scale = invM;
  if (sc.screen && sc.gradient) {
    // gradient screening (k-Mouflage, App. B): the Newtonian force mesh gives
    // |grad Phi_N|; the density is deposited again (bitwise the same) and the row kernel
    // forms (rho - 1)(cn + c5 eps); the massless fifth force then shares 1/k^2
    KOp nop = base;
    nop.g_n = sc.cn;
    nop.scale = invM;
    nop.step_newton = 1;
    float2* const w0[3] = {M[0], M[1], M[2]};
    fft_c2r_force3(pl, nop, nullptr, M[1], w0, b.force, s);
    launch_deposit(L, disp, R(M[0]), b.bins, b.entries, s);
    KmArgs ka;
    ka.km_r = sc.km_r;
    ka.k0 = (float)p.km_k0;
    ka.m = p.km_m;
    ka.cn = sc.cn;
    ka.c5 = sc.c5;
    ka.steps = steps;
    ka.step_ctr = ctr;
    launch_kmouflage_source(L, R(M[0]), b.force, R(M[1]), flat_out ? R(M[2]) : nullptr, ka, s);
    if (flat_out) launch_unpad_mesh(L, R(M[2]), flat_out + L.M, s);
    fft_r2c_zy(pl, R(M[1]), M[1], s);
    src = M[1];
  } else if (sc.screen) {
    KOp sop = base;
    sop.scale = invM;
    int kind = K_SMOOTH;
    if (sc.potential) {   // potential screening (f(R), symmetron): delta_k is kept
      sop.g_n = sc.sop_g_n;
      kind = K_POT;
      dk = M[1];
    } else {
      // nDGP: the fifth force is massless (Sec. 5.2), so g_n delta_k / k^2 + g_5 S_k / k^2
      // is the transform of g_n delta + g_5 delta eps over k^2: the row pass builds that
      // one field and delta_k need not be kept
      sop.r_smooth = (float)p.r_smooth;
      sop.filter = p.filter;
    }
    ScreenArgs sa;
    sa.thr = sc.thr;
    sa.vx = sc.vx;
    sa.vx0 = sc.vx0;
    sa.cn = sc.cn;
    sa.c5 = sc.c5;
    sa.steps = steps;
    sa.step_ctr = ctr;
    fft_screen(pl, kind, sop, M[1], M[2], R(M[0]), flat_out ? R(M[3]) : nullptr, p.model, sa, s);
    if (flat_out) launch_unpad_mesh(L, R(M[3]), flat_out + L.M, s);
    src = M[2];
  } else if (flat_out) {
    launch_unpad_mesh(L, R(M[0]), flat_out + L.M, s, 1.f);   // S = delta = rho - 1
  }
  // the X pass writes its two transforms over its own inputs where it can (delta_k in M[1]
  // and S in M[2]): a 2048-point X column visits one page per x-plane of every field it
  // touches, and two fields instead of three keep more of those translations cached
  float2* const work[3] = {M[1], M[2], M[0]};
  fft_c2r_force3(pl, op, dk, src, work, b.force, s);
}

// One COLA step on the given work area (st->work when null, else the library's scratch).
// Its step-dependent scalars come from the state's step table at the device step counter,
// which the step sets to i first (unless `replay`: a captured step that relies on the
// counter the previous step advanced) and advances at the end.
static void step_impl(const cola_params* p, cola_state* st, int32_t i, void* work, hipStream_t s,
                      bool replay = false) {
  if (!p) throw Error{COLA_E_ARG, "params is NULL"};
  const Bufs b = carve(*p, st, work);
  const Layout& L = b.L;
  if (!st->prepared || st->next_step < 0) throw Error{COLA_E_STATE, "no initial conditions"};
  if (i != st->next_step) throw Error{COLA_E_STATE, "step index out of order"};
  if (i < 0 || i >= p->n_steps) throw Error{COLA_E_STATE, "step index beyond n_steps"};
  if (!replay) launch_set_counter(b.ctr, i, s);
  GatherArgs g{};
  g.table = b.growth;
  g.steps = b.steps;
  g.step_ctr = b.ctr;
  pm_core(*p, b, st->disp, a_of_step(*p, i), nullptr, s, true);
  if (L.kdep) {
    // L''(q, a_i) and Psi_LPT(a_{i+1}) - Psi_LPT(a_i) from the stored k-space fields,
    // after the force (their work fields and outputs may lie over mesh slots 0-2)
    const FFTPlan pp = plan_part(b);
    float2* coef = at<float2>(st->tables, L.off_lpt_coef);
    launch_lpt_coef(L, b.growth, 0, 0, b.steps, b.ctr, coef, s);
    for (int t = 0; t < 2; ++t) {
      KOp op;
      op.kf = (float)(2.0 * M_PI / p->box);
      op.coef = coef + (t == 0 ? 0 : L.n_k);
      op.scale = (float)(1.0 / (double)L.N);
      fft_c2r_lpt3(pp, op, b.phi1, b.phi2, b.lptw, t == 0 ? b.lpp3 : b.dlt3, s);
    }
    g.lpp3 = b.lpp3;
    g.dlt3 = b.dlt3;
  } else {
    g.psi1 = b.psi1;
    g.psi2 = b.psi2;
  }
  g.F3 = b.force;
  g.disp = st->disp;
  g.vel = st->vel;
  launch_gather(L, g, s);
  launch_step_advance(b.ctr, s);
  st->next_step = i + 1;
}

// ------------------------------------------------------------------ ensembles
// Runs stepped together: one step of every member with steps left is captured as one HIP
// graph, one stream branch per member (members spread over the capture streams), and the
// graph is replayed while the set of members with steps left stays the same.
struct Ensemble {
  std::vector<cola_params> p;
  std::vector<cola_state*> st;
  std::vector<hipStream_t> streams;   // capture branches 1.. (branch 0 is the caller's stream)
  std::vector<hipEvent_t> events;     // fork event, one join event per branch, hand-over
  // graphs launched and not known to be finished: kept until the ensemble is destroyed
  std::vector<std::pair<hipGraph_t, hipGraphExec_t>> graphs;
  ~Ensemble() {
    if (!streams.empty()) (void)hipStreamSynchronize(streams[0]);
    for (auto& g : graphs) {
      (void)hipGraphExecDestroy(g.second);
      (void)hipGraphDestroy(g.first);
    }
    for (auto e : events) (void)hipEventDestroy(e);
    for (auto x : streams) (void)hipStreamDestroy(x);
  }
};

static void ensemble_run(Ensemble& E, int n_streams, hipStream_t s) {
  if (prof().on) throw Error{COLA_E_STATE, "kernel profiling must be off while a graph is captured"};
  const int nb = std::max(1, std::min<int>(n_streams, (int)E.st.size()));
  // streams[0] captures and replays (the caller's stream may be the null stream, which
  // cannot be captured); streams[1 ..] are the other branches
  while ((int)E.streams.size() < nb) {
    hipStream_t x;
    COLA_HIP_CHECK(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
    E.streams.push_back(x);
  }
  while ((int)E.events.size() < nb + 1) {
    hipEvent_t e;
    COLA_HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    E.events.push_back(e);
  }
  hipStream_t c0 = E.streams[0];
  for (;;) {
    std::vector<int> act;
    int reps = 1 << 30;
    for (int j = 0; j < (int)E.st.size(); ++j) {
      const int left = E.p[j].n_steps - E.st[j]->next_step;
      if (left > 0) {
        act.push_back(j);
        reps = std::min(reps, left);
      }
    }
    if (act.empty()) break;
    std::vector<int32_t> first(act.size());
    for (size_t m = 0; m < act.size(); ++m) {   // the counters the captured steps start from
      cola_state* st = E.st[act[m]];
      first[m] = st->next_step;
      const Bufs b = carve(E.p[act[m]], st);
      launch_set_counter(b.ctr, st->next_step, s);
    }
    COLA_HIP_CHECK(hipEventRecord(E.events[nb], s));   // c0 starts after the caller's work
    COLA_HIP_CHECK(hipStreamWaitEvent(c0, E.events[nb], 0));
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    COLA_HIP_CHECK(hipStreamBeginCapture(c0, hipStreamCaptureModeThreadLocal));
    try {
      COLA_HIP_CHECK(hipEventRecord(E.events[0], c0));
      for (int k = 1; k < nb; ++k) COLA_HIP_CHECK(hipStreamWaitEvent(E.streams[k], E.events[0], 0));
      for (size_t m = 0; m < act.size(); ++m)
        step_impl(&E.p[act[m]], E.st[act[m]], first[m], nullptr, E.streams[m % nb], true);
      for (int k = 1; k < nb; ++k) {
        COLA_HIP_CHECK(hipEventRecord(E.events[k], E.streams[k]));
        COLA_HIP_CHECK(hipStreamWaitEvent(c0, E.events[k], 0));
      }
    } catch (...) {
      (void)hipStreamEndCapture(c0, &graph);
      if (graph) (void)hipGraphDestroy(graph);
      for (size_t m = 0; m < act.size(); ++m) E.st[act[m]]->next_step = first[m];
      throw;
    }
    COLA_HIP_CHECK(hipStreamEndCapture(c0, &graph));
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
      (void)hipGraphDestroy(graph);
      for (size_t m = 0; m < act.size(); ++m) E.st[act[m]]->next_step = first[m];
      throw Error{COLA_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie)};
    }
    E.graphs.emplace_back(graph, exec);
    hipError_t le = hipSuccess;
    for (int r = 0; r < reps && le == hipSuccess; ++r) le = hipGraphLaunch(exec, c0);
    if (le != hipSuccess) throw Error{COLA_E_HIP, std::string("hipGraphLaunch: ") + hipGetErrorString(le)};
    for (size_t m = 0; m < act.size(); ++m) E.st[act[m]]->next_step = first[m] + reps;
    COLA_HIP_CHECK(hipEventRecord(E.events[nb], c0));   // the caller's stream waits for the steps
    COLA_HIP_CHECK(hipStreamWaitEvent(s, E.events[nb], 0));
  }
}

}  // namespace cola

using namespace cola;

// ------------------------------------------------------------------ C ABI
extern "C" {

const char* cola_status_string(cola_status s) {
  switch (s) {
    case COLA_OK: return "ok";
    case COLA_E_ARG: return "invalid argument";
    case COLA_E_SIZE: return "size error";
    case COLA_E_STATE: return "call out of order";
    case COLA_E_HIP: return "HIP runtime error";
    case COLA_E_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

const char* cola_last_error(void) { return g_last_error.c_str(); }

cola_status cola_validate(const cola_params* p) {
  return guarded([&] {
    if (!p) throw Error{COLA_E_ARG, "params is NULL"};
    validate(*p);
  });
}

cola_status cola_query_sizes(const cola_params* p, cola_sizes* out) {
  return guarded([&] {
    if (!p || !out) throw Error{COLA_E_ARG, "NULL argument"};
    const Layout L = make_layout(*p);
    out->disp_bytes = L.disp_bytes;
    out->vel_bytes = L.disp_bytes;
    out->lpt_bytes = L.lpt_bytes;
    out->tables_bytes = L.tables_bytes;
    out->work_bytes = L.work_bytes;
    out->total_bytes = 2 * L.disp_bytes + L.lpt_bytes + L.tables_bytes + L.work_bytes;
  });
}

cola_status cola_prepare(const cola_params* p, cola_state* st, hipStream_t s) {
  return guarded([&] {
    if (!p) throw Error{COLA_E_ARG, "params is NULL"};
    const Bufs b = carve(*p, st);
    do_prepare(*p, st, b, s);
  });
}

cola_status cola_make_ic(const cola_params* p, cola_state* st, hipStream_t s) {
  return guarded([&] {
    if (!p) throw Error{COLA_E_ARG, "params is NULL"};
    const Bufs b = carve(*p, st);
    const Layout& L = b.L;
    do_prepare(*p, st, b, s);
    const FFTPlan pp = plan_part(b);
    float2* const* M = b.mesh;
    const float invN = (float)(1.0 / (double)L.N);
    KOp base;
    base.kf = (float)(2.0 * M_PI / p->box);
    // white noise -> W_k -> phi1_k = delta_k / k^2
    launch_noise(*p, L.np, L.pitch_p, L.plane_p, R(M[0]), nullptr, s);
    fft_r2c(pp, R(M[0]), M[0], s);
    float2* phi1 = L.kdep ? b.phi1 : M[1];
    launch_ic_phi1(*p, L, M[0], phi1, sigma8_norm(*p), b.ref, s);
    // 2LPT source S = sum_{i<j} phi_ii phi_jj - phi_ij^2 (eq. lcdm2lpt)
    for (int c = 0; c < 3; ++c) {
      KOp op = base;
      op.a = phi1;
      op.comp = op.comp2 = c;
      op.scale = invN;
      fft_c2r(pp, K_HESS, op, M[2 + c], R(M[2 + c]), s);
    }
    const size_t nreal = 2 * L.pgrid_elems;
    launch_2lpt_diag(R(M[2]), R(M[3]), R(M[4]), nreal, s);
    const int mix[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    for (auto& ij : mix) {
      KOp op = base;
      op.a = phi1;
      op.comp = ij[0];
      op.comp2 = ij[1];
      op.scale = invN;
      fft_c2r(pp, K_HESS, op, M[0], R(M[0]), s);
      launch_2lpt_sub(R(M[2]), R(M[0]), nreal, s);
    }
    fft_r2c(pp, R(M[2]), M[2], s);
    float2* phi2 = L.kdep ? b.phi2 : M[3];
    {
      KOp op = base;
      op.a = M[2];
      op.g_n = -1.f;
      op.scale = 1.f;
      op.n = L.np;
      op.pitch = L.pitch_p;
      op.plane = L.plane_p;
      launch_kspace(K_POT, op, phi2, s);   // phi2_k = -S_k / k^2
    }
    float2* outs[3] = {M[0], M[2], M[4]};
    const float* f3[3] = {R(M[0]), R(M[2]), R(M[4])};
    if (L.kdep) {
      // u(a_ini) = IDFT[i k (D1(k, a_0) phi1_k + D2(k, a_0) phi2_k)]
      for (int c = 0; c < 3; ++c) {
        KOp op = base;
        op.a = phi1;
        op.b = phi2;
        op.table = b.growth;
        op.tab_slice0 = 0;
        op.lpt_mode = 2;
        op.kdep = 1;
        op.comp = c;
        op.scale = invN;
        fft_c2r(pp, K_LPT, op, outs[c], R(outs[c]), s);
      }
      launch_unpad3(L, f3, nullptr, 1.f, 0.f, st->disp, s);
    } else {
      float* dst[2] = {b.psi1, b.psi2};
      float2* src[2] = {phi1, phi2};
      for (int o = 0; o < 2; ++o) {
        for (int c = 0; c < 3; ++c) {
          KOp op = base;
          op.a = src[o];
          op.comp = c;
          op.scale = invN;
          fft_c2r(pp, K_GRAD, op, outs[c], R(outs[c]), s);
        }
        launch_unpad3(L, f3, nullptr, 1.f, 0.f, dst[o], s);
      }
      launch_combine_u0(L, b.psi1, b.psi2, b.growth, st->disp, s);
    }
    launch_fill(st->vel, 3 * (size_t)L.N, 0.f, s);
    st->next_step = 0;
  });
}

cola_status cola_pm_force(const cola_params* p, cola_state* st, double a, float* force_out,
                          float* mesh_out, hipStream_t s) {
  return guarded([&] {
    if (!p) throw Error{COLA_E_ARG, "params is NULL"};
    const Bufs b = carve(*p, st);
    if (!st->prepared) throw Error{COLA_E_STATE, "state not prepared"};
    if (!(a > 0.0 && a <= 10.0)) throw Error{COLA_E_ARG, "a must be in (0, 10]"};
    pm_core(*p, b, st->disp, a, mesh_out, s);
    if (mesh_out) launch_split3(b.L, b.force, mesh_out + 2 * b.L.M, s);
    if (force_out) {
      GatherArgs g{};
      g.F3 = b.force;
      g.disp = st->disp;
      g.vel = st->vel;
      g.force_out = force_out;
      launch_gather(b.L, g, s);
    }
  });
}

cola_status cola_step(const cola_params* p, cola_state* st, int32_t i, hipStream_t s) {
  return guarded([&] { step_impl(p, st, i, nullptr, s); });
}

cola_status cola_step_static(const cola_params* p, cola_state* st, int32_t i, hipStream_t s) {
  return guarded([&] {
    if (!p) throw Error{COLA_E_ARG, "params is NULL"};
    const Layout L = make_layout(*p);
    step_impl(p, st, i, static_work(L.work_bytes), s);
  });
}

cola_status cola_ensemble_create(int32_t n, const cola_params* params, cola_state* const* states,
                                 cola_ensemble** out) {
  return guarded([&] {
    if (!out) throw Error{COLA_E_ARG, "out is NULL"};
    *out = nullptr;
    if (n < 1 || !params || !states) throw Error{COLA_E_ARG, "need n >= 1 runs"};
    auto E = std::make_unique<Ensemble>();
    for (int j = 0; j < n; ++j) {
      const Bufs b = carve(params[j], states[j]);   // validates the run and its buffers
      (void)b;
      for (int i = 0; i < j; ++i)
        if (states[i] == states[j]) throw Error{COLA_E_ARG, "a state appears twice"};
      E->p.push_back(params[j]);
      E->st.push_back(states[j]);
    }
    *out = reinterpret_cast<cola_ensemble*>(E.release());
  });
}

cola_status cola_ensemble_run(cola_ensemble* e, int32_t n_streams, hipStream_t s) {
  return guarded([&] {
    if (!e) throw Error{COLA_E_ARG, "ensemble is NULL"};
    if (n_streams < 1 || n_streams > 64) throw Error{COLA_E_ARG, "n_streams must be in [1, 64]"};
    Ensemble& E = *reinterpret_cast<Ensemble*>(e);
    for (size_t j = 0; j < E.st.size(); ++j)
      if (!E.st[j]->prepared || E.st[j]->next_step < 0)
        throw Error{COLA_E_STATE, "every member needs its initial conditions"};
    ensemble_run(E, n_streams, s);
  });
}

cola_status cola_ensemble_destroy(cola_ensemble* e) {
  return guarded([&] { delete reinterpret_cast<Ensemble*>(e); });
}

cola_status cola_power_spectrum(const cola_params* p, cola_state* st, int32_t nbins, double* k_out,
                                double* p_out, int64_t* nmodes_out, hipStream_t s) {
  return guarded([&] {
    if (!p || !k_out || !p_out) throw Error{COLA_E_ARG, "NULL argument"};
    const Bufs b = carve(*p, st);
    if (!st->prepared) throw Error{COLA_E_STATE, "state not prepared"};
    if (nbins < 1 || nbins > 2048) throw Error{COLA_E_ARG, "nbins must be in [1, 2048]"};
    launch_deposit(b.L, st->disp, R(b.mesh[0]), b.bins, b.entries, s);
    fft_r2c(plan_mesh(b), R(b.mesh[0]), b.mesh[1], s);
    launch_pk(b.L, b.mesh[1], nbins, b.pk_scratch, b.pk_out, b.pk_cnt, s);
    std::vector<float4> o(nbins);
    std::vector<unsigned long long> c(nbins);
    COLA_HIP_CHECK(hipMemcpyAsync(o.data(), b.pk_out, nbins * sizeof(float4), hipMemcpyDeviceToHost, s));
    COLA_HIP_CHECK(hipMemcpyAsync(c.data(), b.pk_cnt, nbins * sizeof(unsigned long long),
                                  hipMemcpyDeviceToHost, s));
    COLA_HIP_CHECK(hipStreamSynchronize(s));
    for (int i = 0; i < nbins; ++i) {
      const double w = (double)c[i];
      const double sp = (double)o[i].x + (double)o[i].y;
      const double sk = (double)o[i].z + (double)o[i].w;
      k_out[i] = w > 0 ? sk / w : 0.0;
      p_out[i] = w > 0 ? sp / w : 0.0;
      if (nmodes_out) nmodes_out[i] = (int64_t)c[i];
    }
  });
}

cola_status cola_step_times(const cola_params* p, int32_t i, double* out) {
  return guarded([&] {
    if (!p || !out) throw Error{COLA_E_ARG, "NULL argument"};
    validate(*p);
    if (i < 0 || i >= p->n_steps) throw Error{COLA_E_ARG, "step index out of range"};
    step_times(*p, i, out);
  });
}

cola_status cola_fft_tiles(int32_t n, int32_t fwd, int32_t inv, int32_t* cur_out) {
  return guarded([&] {
    if (!fft_size_supported(n)) throw Error{COLA_E_ARG, "transform size not supported"};
    fft_set_tiles(n, fwd, inv);
    if (cur_out) {
      int t[2];
      fft_get_tiles(n, t);
      cur_out[0] = t[0];
      cur_out[1] = t[1];
    }
  });
}

cola_status cola_autotune(const cola_params* p, cola_state* st, int32_t* out, hipStream_t s) {
  return guarded([&] {
    if (!p || !out) throw Error{COLA_E_ARG, "NULL argument"};
    const Bufs b = carve(*p, st);
    if (!st->prepared) throw Error{COLA_E_STATE, "state not prepared"};
    int t[2];
    fft_autotune(plan_mesh(b), b.mesh[0], s, t);
    out[0] = t[0];
    out[1] = t[1];
    out[2] = out[3] = 0;
    // the particle-grid transforms run only when their field fits the work area
    if (b.L.pgrid_elems * sizeof(float2) <= b.L.work_bytes) {
      fft_autotune(plan_part(b), b.mesh[0], s, t);
      out[2] = t[0];
      out[3] = t[1];
    }
  });
}

cola_status cola_positions(const cola_params* p, const cola_state* st, float* xyz, hipStream_t s) {
  return guarded([&] {
    if (!p || !xyz) throw Error{COLA_E_ARG, "NULL argument"};
    const Bufs b = carve(*p, st);
    launch_positions(*p, b.L, st->disp, xyz, s);
  });
}

cola_status cola_growth_table(const cola_params* p, const cola_state* st, int32_t i, double* out,
                              int64_t out_len, int64_t* n_k_out, hipStream_t s) {
  return guarded([&] {
    if (!p || !out) throw Error{COLA_E_ARG, "NULL argument"};
    const Bufs b = carve(*p, st);
    if (!st->prepared) throw Error{COLA_E_STATE, "state not prepared"};
    if (i < 0 || i > p->n_steps) throw Error{COLA_E_ARG, "slice index out of range"};
    const int64_t n = b.L.n_k * 6;
    if (out_len < n) throw Error{COLA_E_SIZE, "output buffer too small"};
    COLA_HIP_CHECK(hipMemcpyAsync(out, b.growth + (int64_t)i * n, n * sizeof(double),
                                  hipMemcpyDeviceToHost, s));
    COLA_HIP_CHECK(hipStreamSynchronize(s));
    if (n_k_out) *n_k_out = b.L.n_k;
  });
}

cola_status cola_white_noise(const cola_params* p, int32_t grid, float* dst, hipStream_t s) {
  return guarded([&] {
    if (!p || !dst) throw Error{COLA_E_ARG, "NULL argument"};
    validate(*p);
    if (grid != 0) throw Error{COLA_E_UNSUPPORTED, "only the particle grid is supported"};
    launch_noise(*p, p->np1d, half_pitch(p->np1d), plane_stride(p->np1d), nullptr, dst, s);
  });
}

cola_status cola_growth_triangles(const cola_params* p, int32_t n, const double* tri, double a,
                                  double* out, hipStream_t s) {
  return guarded([&] {
    if (!p) throw Error{COLA_E_ARG, "params is NULL"};
    validate(*p);
    if (n < 0) throw Error{COLA_E_ARG, "n must be >= 0"};
    const double a_ini = 1.0 / (1.0 + p->z_init);
    if (!(a >= a_ini && a <= 10.0)) throw Error{COLA_E_ARG, "a must be in [a_ini, 10]"};
    if (n == 0) return;
    if (!tri || !out) throw Error{COLA_E_ARG, "NULL argument"};
    launch_growth_triangles(*p, n, tri, a, out, s);
  });
}

cola_status cola_profile_enable(int32_t on) {
  return guarded([&] {
    ProfState& P = prof();
    std::lock_guard<std::mutex> lk(P.mu);
    P.on = on != 0;
  });
}

cola_status cola_profile_reset(void) {
  return guarded([&] {
    ProfState& P = prof();
    std::lock_guard<std::mutex> lk(P.mu);
    P.drain();
    P.acc.clear();
  });
}

cola_status cola_profile_read(char (*names)[48], double* ms, int64_t* counts, int32_t cap,
                              int32_t* n_out) {
  return guarded([&] {
    ProfState& P = prof();
    std::lock_guard<std::mutex> lk(P.mu);
    P.drain();
    int32_t n = 0;
    for (auto& kv : P.acc) {
      if (n < cap && names && ms && counts) {
        std::strncpy(names[n], kv.first.c_str(), 47);
        names[n][47] = 0;
        ms[n] = kv.second.first;
        counts[n] = kv.second.second;
      }
      ++n;
    }
    if (n_out) *n_out = n;
  });
}

}  // extern "C"
