"""Benchmark of the COLA particle-mesh step on one MI355X.

Workload (the headline): Hu-Sawicki f(R), n = 1, |f_R0| = 1e-5, chameleon screening, with
its own scale-dependent growth factors D1(k,a), D2(k,a) (the LPT terms are rebuilt every
step by inverse FFTs on the particle grid, App. A); Np = 1024^3 particles stored as FP32
Lagrangian displacements, Nmesh = 2048^3 FP32 mesh, L = 2048 Mpc/h; seeded Gaussian
initial conditions (Eisenstein-Hu no-wiggle spectrum, Om = 0.3, h = 0.7, ns = 0.96,
sigma8 = 0.8), 2LPT at z = 19, 20 COLA steps to z = 0.  FP64 only in the growth tables and
the step coefficients.

A step is one cola_step: CIC deposit, forward FFT, potential screening (inverse FFT of
the Newtonian potential, the real-space factor, forward FFT of S), the fused
Green's-function / fifth-force / gradient inverse FFTs, the per-step LPT synthesis (two
fused particle-grid inverse FFTs, each giving the three components of L'' or Delta), and
the CIC gather fused with the kick and drift.  Warm-up steps run from
their own initial conditions; the K timed steps start from new ones, so the default
K = 20 times one whole run to z = 0 (initial conditions, made before each run, are never
inside a timed interval).

Prints one JSON line.  `value` is particle-steps per second over exactly K timed steps
(bracketed by device synchronisation); `roofline` reports the kernel with the largest
share of the step against the MI355X HBM peak, timed with HIP events on its launch
stream; `cpu_baseline` times the FP64 oracle on host cores on a bounded sample of the
same workload.  A secondary block repeats the measurement for nDGP (r_c H0 = 1,
Vainshtein screening) with 512^3 particles on a 1024^3 mesh in L = 1024 Mpc/h, 30 steps.
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "PM particle-steps/s + % HBM peak; mock runs/hour and p99 time-to-z=0"


WORKLOAD = ("f(R) Hu-Sawicki n=1 |fR0|=1e-5 chameleon-screened, scale-dependent D1(k,a), "
            "D2(k,a) (LPT terms rebuilt by particle-grid FFTs every step), Np=1024^3 FP32 "
            "Lagrangian displacements, Nmesh=2048^3 FP32, L=2048 Mpc/h, 2LPT at z=19, 20 COLA steps")
SECONDARY = ("nDGP rcH0=1 Vainshtein-screened (Gaussian R=1 Mpc/h), Np=512^3, Nmesh=1024^3, "
             "L=1024 Mpc/h, 2LPT at z=19, 30 COLA steps")


def workload_params(C):
    return C.Params(model=C.FR_HS1, fr0_abs=1e-5, screening=1, growth_mode=0,
                    np1d=1024, nmesh1d=2048, box=2048.0, z_init=19.0, n_steps=20, seed=1)


def secondary_params(C):
    return C.Params(model=C.NDGP, rc_h0=1.0, screening=1, filter=0, r_smooth=1.0,
                    np1d=512, nmesh1d=1024, box=1024.0, z_init=19.0, n_steps=30, seed=1)


def algorithmic_bytes(name, p):
    """Bytes a kernel must move per launch (single-precision fields, unpadded):
    mesh M = n^3 real cells, half-complex H = n^2 (n/2 + 1) complex values, N particles,
    and on the particle grid (the LPT transforms) Hp = np^2 (np/2 + 1)."""
    n = p.nmesh1d
    M = n ** 3
    H = n * n * (n // 2 + 1)
    N = p.np1d ** 3
    Hp = p.np1d ** 2 * (p.np1d // 2 + 1)
    table = {
        "bin_count": 12 * N,                         # read u; tile counts are negligible
        "bin_scan": 0,
        "bin_scatter": 12 * N + 12 * N,              # read u, write one 12-byte record each
        "deposit": 12 * N + 4 * M,                   # read records, write the density once
        "fft_r2c_z": 4 * M + 8 * H,                  # read real mesh, write half-complex
        "fft_c2r_z": 8 * H + 4 * M,
        "fft_y_fwd": 16 * H, "fft_x_fwd": 16 * H, "fft_y_inv": 16 * H,
        "fft_x_fwd_smooth": 8 * H + 8 * H,           # read delta; write X^-1[W delta_k]
        "fft_x_fwd_pot": 8 * H + 16 * H,             # read delta; write delta_k and X^-1[Phi_k]
        "fft_z_screen": 8 * H + 4 * M + 8 * H,       # read the filtered field and rho, write S
        "fft_x_fwd_force": 16 * H + 16 * H,          # read S and delta_k; write G0 and G
        "fft_x_fwd_force_1src": 8 * H + 16 * H,      # read one combined source; write G0 and G
        "fft_y_inv_yz": 8 * H + 16 * H,              # read G; write the y and z components
        "fft_c2r_z3": 24 * H + 12 * M,               # read 3 force passes, write (Fx, Fy, Fz)
        "gather_kick_drift": 12 * M + 72 * N,        # force mesh; u, v and the LPT terms in; u, v out
        "lpt_fft_x_inv": 16 * Hp + 16 * Hp,          # read phi1_k, phi2_k; write G0 and G
        "lpt_fft_y_inv": 16 * Hp,
        "lpt_fft_y_inv_yz": 8 * Hp + 16 * Hp,
        "lpt_fft_c2r_z3": 24 * Hp + 12 * N,          # write (x, y, z) of L'' or Delta
        "fft_x_inv_lpt": 16 * Hp + 8 * Hp,           # initial conditions: one component
        "lpt_fft_c2r_z": 8 * Hp + 4 * N,
        "fill": 0,
    }
    return table.get(name)


def yardstick_bytes_for(p, C):
    """Algorithmic bytes of one step, counting each 3D FFT as one read and one write of a
    real-sized mesh per pair of passes.  Deposit 12N + 4M, forward R2C 16M, screening
    (C2R of the filtered field, the real-space factor, R2C of S) 52M, the Green's function
    16M (LCDM) or 20M, three force C2Rs 48M, gather with kick and drift 12M + 72N, and for
    scale-dependent growth the LPT synthesis 128N (read phi1_k, phi2_k; six particle-grid
    C2Rs; the six fields read by the gather).  LCDM 96M + 84N; screened modified gravity
    with scale-independent LPT (nDGP, f(R) with LCDM growth) 152M + 84N; with
    scale-dependent growth (f(R), symmetron) 152M + 212N."""
    M, N = p.nmesh1d ** 3, p.np1d ** 3
    if p.model == C.LCDM:
        return 96 * M + 84 * N
    if p.model in (C.FR_HS1, C.SYMMETRON) and p.growth_mode == 0:
        return 152 * M + 212 * N
    return 152 * M + 84 * N


def _mock_params(C, rng, j, sizes, seed0, n_steps):
    """One mock of the ensemble and serving mixes: n_p drawn from `sizes`, n_mesh = 2 n_p,
    L = 2 n_p Mpc/h, z_ini = 19, model uniform over LCDM, f(R) |f_R0| = 1e-6, 1e-5, 1e-4
    and nDGP r_c H0 = 0.5, 1, all screened; seed = seed0 + j."""
    n = int(rng.choice(sizes))
    m = int(rng.integers(6))
    kw = dict(np1d=n, nmesh1d=2 * n, box=2.0 * n, z_init=19.0, n_steps=int(n_steps),
              seed=seed0 + j, screening=1)
    if m == 0:
        kw.update(model=C.LCDM)
    elif m <= 3:
        kw.update(model=C.FR_HS1, fr0_abs=(1e-6, 1e-5, 1e-4)[m - 1])
    else:
        kw.update(model=C.NDGP, rc_h0=(0.5, 1.0)[m - 4])
    return C.Params(**kw)


def bench_ensemble(C, torch, boxes=64, budget=160 << 30):
    """A mixed ensemble of small boxes (seeded draw, seed 4: n_p in {64, 96, 128, 192,
    256}, 10 steps) run one at a time on one stream, then all resident at once and
    interleaved on eight streams, then all resident and stepped as captured HIP graphs
    (cola_ensemble_run: one step of every box per graph, a branch per box over eight
    capture streams, replayed for the ten steps); aggregate particle-steps/s and
    yardstick HBM fraction.  Every leg's time runs from the first allocation to the end
    of the last step, initial conditions included; the graph leg also reports its steps
    alone."""
    import numpy as np
    from paper_1703_00879_amd.serve import GpuEngine, Request, Server, summarize
    rng = np.random.default_rng(4)
    ps = [_mock_params(C, rng, j, (64, 96, 128, 192, 256), 1000, 10) for j in range(boxes)]
    yard = sum(yardstick_bytes_for(p, C) * p.n_steps for p in ps)
    out = {"boxes": boxes, "n_steps": 10, "particle_steps": sum(p.np1d ** 3 * p.n_steps for p in ps)}
    for name, streams, active in (("one_at_a_time", 1, 1), ("interleaved_8_streams", 8, boxes)):
        res = Server(GpuEngine(n_streams=streams), budget, max_active=active).run(
            [Request(p, 0.0, j) for j, p in enumerate(ps)])
        sm = summarize(res)
        out[name] = {"seconds": sm["span_s"], "particle_steps_per_s": sm["particle_steps_per_s"],
                     "hbm_frac_yardstick": yard / sm["span_s"] / 1e9 / HBM_PEAK_GBS}
        torch.cuda.empty_cache()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    states = [C.State(p, device="cuda:0") for p in ps]
    ic_streams = [torch.cuda.Stream() for _ in range(8)]
    for j, (p, st) in enumerate(zip(ps, states)):   # initial conditions overlap on 8 streams
        C.cola_make_ic(p, st, stream=ic_streams[j % 8].cuda_stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ens = C.Ensemble(ps, states)
    ens.run(n_streams=8)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ens.close()
    ps_total = out["particle_steps"]
    out["graph_8_streams"] = {"seconds": t2 - t0, "particle_steps_per_s": ps_total / (t2 - t0),
                              "hbm_frac_yardstick": yard / (t2 - t0) / 1e9 / HBM_PEAK_GBS,
                              "steps_seconds": t2 - t1,
                              "steps_particle_steps_per_s": ps_total / (t2 - t1),
                              "steps_hbm_frac_yardstick": yard / (t2 - t1) / 1e9 / HBM_PEAK_GBS}
    del states, ens
    torch.cuda.empty_cache()
    return out


def bench_serving(C, torch, requests=96, budget=96 << 30, rates=(0.5, 0.8, 1.0)):
    """A Poisson stream of mock requests (n_p in {128, 256, 384}, 10-30 steps, models and
    parameters as the ensemble, seed = 100000 + j) through the serving loop: first all at
    once to measure the saturation rate, then arriving at 0.5, 0.8 and 1.0 of it (arrival
    RNG seed 5).  Reports runs/hour and p50 / p99 time to z = 0 at each rate."""
    import numpy as np
    from paper_1703_00879_amd.serve import GpuEngine, Request, Server, summarize
    rng = np.random.default_rng(5)
    ps = [_mock_params(C, rng, j, (128, 256, 384), 100000, rng.integers(10, 31))
          for j in range(requests)]
    srv = Server(GpuEngine(n_streams=4), budget, max_active=16)

    def progress(done, total):
        if done % 50 == 0 or done == total:
            print(f"[bench] serving: {done}/{total} runs done", file=sys.stderr, flush=True)

    sat = summarize(srv.run([Request(p, 0.0, j) for j, p in enumerate(ps)], on_result=progress))
    torch.cuda.empty_cache()
    gaps = rng.exponential(1.0, size=requests)   # unit-rate Poisson gaps, scaled per rate
    out = {"requests": requests, "saturation_runs_per_hour": sat["runs_per_hour"],
           "saturation_p50_time_to_z0_s": sat["p50_s"], "saturation_p99_time_to_z0_s": sat["p99_s"],
           "rates": {}}
    for f in rates:
        lam = f * sat["runs"] / sat["span_s"]
        t = np.cumsum(gaps / lam)
        t -= t[0]
        st = summarize(srv.run([Request(p, float(a), j) for j, (p, a) in enumerate(zip(ps, t))],
                               on_result=progress))
        torch.cuda.empty_cache()
        out["rates"][f"{f:g}"] = {"arrival_rate_per_s": lam, "runs_per_hour": st["runs_per_hour"],
                                  "p50_time_to_z0_s": st["p50_s"], "p99_time_to_z0_s": st["p99_s"],
                                  "particle_steps_per_s": st["particle_steps_per_s"]}
    # the headline serving figures: 0.8 of saturation
    r8 = out["rates"].get("0.8")
    if r8:
        out.update(runs_per_hour=r8["runs_per_hour"], p50_time_to_z0_s=r8["p50_time_to_z0_s"],
                   p99_time_to_z0_s=r8["p99_time_to_z0_s"])
    return out


def source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1703_00879_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


TRAFFIC_FILE = "traffic_fr5_1024_2048.json"
PROFILE_FILE = "pm_step_fr5_1024_2048.md"


def traffic_for(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, or None if
    the summary is missing or was taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", TRAFFIC_FILE)
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    if d.get("source_hash") != source_hash():
        return None
    k = d.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def counted_bytes_per_step():
    """HBM bytes of one step counted by rocprofv3 (FETCH_SIZE and WRITE_SIZE, copy-calibrated,
    summed over the step's kernels) from the committed summary, or None if it is missing
    or was taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", TRAFFIC_FILE)
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    if d.get("source_hash") != source_hash():
        return None
    return sum(k["bytes_per_launch"] * k["launches_per_step"] for k in d.get("kernels", {}).values()
               if k.get("bytes_per_launch") is not None)


# rocprofv3 kernel symbols of one step -> the names the library's HIP-event profiler uses
# ({n}: mesh size; {np}: particle-grid size; {nph} = np/2, the complex row length of the
# particle grid's real transforms); the first pattern that matches wins
_SYMBOLS = [("k_fft_col_fwd_force<{n}, true>", "fft_x_fwd_force"),
            ("k_fft_col_fwd_force<{n}, false>", "fft_x_fwd_force_1src"),
            ("k_fft_col_lpt<{np}>", "lpt_fft_x_inv"), ("k_fft_col_inv_yz<{np}>", "lpt_fft_y_inv_yz"),
            ("k_fft_c2r_row3<{nph}>", "lpt_fft_c2r_z3"),
            ("k_fft_col_inv_yz", "fft_y_inv_yz"), ("k_fft_col_fwd_op<{n}, 3,", "fft_x_fwd_smooth"),
            ("k_fft_col_fwd_op<{n}, 2,", "fft_x_fwd_pot"), ("k_fft_col<{n}, -1, 0,", "fft_y_fwd"),
            ("k_fft_col<{n}, 1, 0,", "fft_y_inv"), ("k_fft_col<{np}, 1, 4,", "fft_x_inv_lpt"),
            ("k_fft_col<{np}, 1, 0,", "lpt_fft_y_inv"), ("k_fft_c2r_row3", "fft_c2r_z3"),
            ("k_fft_c2r_row<{nph}>", "lpt_fft_c2r_z"),
            ("k_fft_screen_row", "fft_z_screen"), ("k_fft_r2c_row", "fft_r2c_z"),
            ("k_gather", "gather_kick_drift"), ("k_deposit_tiles", "deposit"), ("k_bin<0,", "bin_count"),
            ("k_bin<1,", "bin_scatter"), ("k_scan_", "bin_scan"), ("k_fill", "fill")]


def _profile_name(symbol, n, np_=None):
    np_ = np_ or n // 2
    for pat, name in _SYMBOLS:
        if pat.format(n=n, np=np_, nph=np_ // 2) in symbol:
            return name
    return symbol.split("(")[0].replace("void ", "")


def profile_command(steps, warmup):
    """The rocprofv3 runs whose summary summarize_rocprof condenses (D = output directory,
    REPO = repository root): a kernel trace and the FETCH_SIZE and WRITE_SIZE counters of
    the bench's own timed steps, and the same counters for a plain 1 GiB device copy."""
    b = (f"python3 $REPO/bench.py --steps {steps} --warmup {warmup} --headline-only "
         "--no-profile")
    c = "python3 $REPO/bench.py --calibrate-copy"
    return "; ".join([
        "cd /tmp && export TMPDIR=/tmp",
        f"rocprofv3 --kernel-trace --stats --output-format csv -d $D/trace -o trace -- {b}",
        f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d $D/fetch -o fetch -- {b}",
        f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d $D/write -o write -- {b}",
        f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d $D/cfetch -o cfetch -- {c}",
        f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d $D/cwrite -o cwrite -- {c}",
        f"python3 $REPO/bench.py --summarize-rocprof $D --steps {steps} --warmup {warmup}"])


def summarize_rocprof(d, out_dir, steps, warmup=0):
    """Condense the rocprofv3 runs of profile_command(steps, warmup) under directory d
    (trace/, fetch/, write/: kernel trace and FETCH_SIZE / WRITE_SIZE counters of the
    headline run; cfetch/, cwrite/: the same counters for `bench.py --calibrate-copy`) into
    per-kernel figures, written to out_dir as a markdown table and the traffic file bench.py
    reads.  The gather ends every step, so the timed steps are the last `steps` gathers of
    the trace; the summary covers the dispatches after the first of them up to the last,
    i.e. timed steps 2..K (timed step 1 follows the initial conditions of its run)."""
    import csv
    from collections import defaultdict
    from paper_1703_00879_amd import cola as C
    p = workload_params(C)
    n, np_ = p.nmesh1d, p.np1d

    def rows(path):
        with open(path) as f:
            return list(csv.DictReader(f))

    def step_window(recs, key):
        ids = sorted({int(r["Dispatch_Id"]) for r in recs if "k_gather" in r[key]})
        ids = ids[-steps:]
        return ids[0], ids[-1], len(ids) - 1

    tr = rows(os.path.join(d, "trace", "trace_kernel_trace.csv"))
    lo, hi, nsteps = step_window(tr, "Kernel_Name")
    dur = defaultdict(list)
    for r in tr:
        i = int(r["Dispatch_Id"])
        if lo < i <= hi:
            dur[_profile_name(r["Kernel_Name"], n, np_)].append(
                (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6)

    def counter(sub, name):
        recs = rows(os.path.join(d, sub, f"{sub}_counter_collection.csv"))
        a, b, _ = step_window(recs, "Kernel_Name")
        acc = defaultdict(list)
        for r in recs:
            if a < int(r["Dispatch_Id"]) <= b and r["Counter_Name"] == name:
                acc[_profile_name(r["Kernel_Name"], n, np_)].append(float(r["Counter_Value"]))
        return acc

    def copy_factor(sub, name):
        recs = rows(os.path.join(d, sub, f"{sub}_counter_collection.csv"))
        v = [float(r["Counter_Value"]) for r in recs
             if "copyBuffer" in r["Kernel_Name"] and r["Counter_Name"] == name]
        v = [x for x in v if x > 1e5]   # the 1 GiB copies, not small staging copies
        return (4 * (1 << 28) / 1024) / (sum(v) / len(v))

    fetch, write = counter("fetch", "FETCH_SIZE"), counter("write", "WRITE_SIZE")
    kf, kw = copy_factor("cfetch", "FETCH_SIZE"), copy_factor("cwrite", "WRITE_SIZE")
    kern = {}
    for name, ds in dur.items():
        fb = 1024 * kf * sum(fetch[name]) / len(fetch[name]) if fetch.get(name) else None
        wb = 1024 * kw * sum(write[name]) / len(write[name]) if write.get(name) else None
        kern[name] = {"launches_per_step": len(ds) / nsteps, "avg_ms": sum(ds) / len(ds),
                      "ms_per_step": sum(ds) / nsteps,
                      "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
                      "bytes_per_launch": (fb + wb) if fb is not None and wb is not None else None,
                      "algorithmic_bytes_per_launch": algorithmic_bytes(name, p)}
    cmd = profile_command(steps, warmup)
    traffic = {"source_hash": source_hash(), "workload": WORKLOAD, "steps_covered": nsteps,
               "fetch_scale": kf, "write_scale": kw, "command": cmd, "kernels": kern}
    os.makedirs(out_dir, exist_ok=True)
    with open(os.path.join(out_dir, TRAFFIC_FILE), "w") as f:
        json.dump(traffic, f, indent=1)
    tot = sum(k["ms_per_step"] for k in kern.values())
    yard = yardstick_bytes_for(p, C)
    counted = sum(k["bytes_per_launch"] * k["launches_per_step"] for k in kern.values()
                  if k["bytes_per_launch"] is not None)
    lines = [f"# PM step kernels: {WORKLOAD} (rocprofv3)", "",
             f"Source hash {traffic['source_hash']}; timed steps 2..{steps} of the bench's "
             f"{steps}-step timed run ({nsteps} steps, after {warmup} warm-up steps on a run of "
             "their own).", "",
             "Command (from the repository root on the GPU host, D = output directory, "
             "REPO = repository root):", "",
             "```", cmd.replace("; ", "\n"), "```", "",
             f"HBM bytes = FETCH_SIZE x {kf:.3f} + WRITE_SIZE x {kw:.3f} (KiB per dispatch), the "
             "factors that make the counters of a plain 1 GiB device copy read 1 GiB each.", "",
             "| kernel | launches/step | avg ms | ms/step | % | HBM GB/launch | algorithmic GB/launch "
             "| HBM GB/s | algorithmic GB/s |", "|---|---|---|---|---|---|---|---|---|"]
    for name, k in sorted(kern.items(), key=lambda kv: -kv[1]["ms_per_step"]):
        hb, ab = k["bytes_per_launch"], k["algorithmic_bytes_per_launch"]
        g = lambda x: "-" if x is None else f"{x / 1e9:.2f}"  # noqa: E731
        r = lambda x: "-" if x is None else f"{x / 1e9 / (k['avg_ms'] / 1e3):.0f}"  # noqa: E731
        lines.append(f"| {name} | {k['launches_per_step']:g} | {k['avg_ms']:.3f} | "
                     f"{k['ms_per_step']:.2f} | {100 * k['ms_per_step'] / tot:.1f} | {g(hb)} | {g(ab)} "
                     f"| {r(hb)} | {r(ab)} |")
    lines += ["", f"Sum of kernel time per step: {tot:.2f} ms.",
              f"Counted HBM bytes per step: {counted / 1e9:.1f} GB "
              f"({counted / 1e9 / (tot / 1e3) / HBM_PEAK_GBS:.3f} of the 8 TB/s peak over the summed "
              f"kernel time); yardstick {yard / 1e9:.1f} GB "
              f"({yard / 1e9 / (tot / 1e3) / HBM_PEAK_GBS:.3f})."]
    with open(os.path.join(out_dir, PROFILE_FILE), "w") as f:
        f.write("\n".join(lines) + "\n")
    return traffic


def host_cpu_model():
    """Host CPU as /proc/cpuinfo names it (model name, family, model, stepping) and the
    logical CPUs the process may use / the host has."""
    info = {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                k, _, v = line.partition(":")
                k = k.strip()
                if k in ("model name", "cpu family", "model", "stepping") and k not in info:
                    info[k] = v.strip()
    except OSError:
        pass
    name = info.get("model name", "unknown host CPU")
    return (f"{name} (family {info.get('cpu family', '?')}, model {info.get('model', '?')}, "
            f"stepping {info.get('stepping', '?')}); {len(os.sched_getaffinity(0))} of "
            f"{os.cpu_count()} logical CPUs available")


def cpu_baseline(steps=6):
    """The FP64 oracle on the host, on a bounded sample of the headline workload: F5 with
    scale-dependent growth, screened, on a 128^3-particle / 256^3-mesh / 256 Mpc/h sub-box
    (the workload's 2 Mpc/h particle spacing and 1 Mpc/h cells, its 20-step time grid and
    seed), timing `steps` COLA steps after the 2LPT initial conditions: once with serial
    transforms and once with the transforms on every host core.  The deposit and gather
    (numpy bincount / fancy indexing) run on one thread either way."""
    import oracle
    from oracle import fftlib
    from oracle.cola import Run
    p = oracle.Params(model=oracle.MODEL_FR, fr0_abs=1e-5, screening=1, growth_mode=0,
                      np1d=128, nmesh1d=256, box=256.0, z_init=19.0, n_steps=20, seed=1)
    host = host_cpu_model()
    cores = len(os.sched_getaffinity(0))
    res = {}
    for w in (1, cores):
        fftlib.set_workers(w)
        r = Run(p)
        t = time.perf_counter()
        for _ in range(steps):
            r.step()
        res[w] = time.perf_counter() - t
    fftlib.set_workers(1)
    return {"value": p.n_part * steps / res[cores], "unit": "particle-steps/s", "cores": cores,
            "kind": "oracle", "host_cpu": host,
            "value_one_core": p.n_part * steps / res[1],
            "sample": f"F5 scale-dependent, screened, 128^3 particles / 256^3 mesh / L=256 Mpc/h "
                      f"(the workload's spacing and cell), {steps} COLA steps of the 20-step grid "
                      f"after 2LPT ICs: {res[cores]:.1f} s with scipy FFTs on {cores} threads, "
                      f"{res[1]:.1f} s on one (CIC deposit and gather single-threaded numpy)"}


# FP64 operations of one classical Runge-Kutta step of the triangle system: four
# right-hand sides (three mu, gamma_2^E at the triangle and at k/sqrt2, exp, ~10 state
# terms: ~210 each) plus the update (10 x 8)
TRIANGLE_FLOP_PER_STEP = 4 * 210 + 80
FP64_VECTOR_PEAK_TFLOPS = 78.6


def bench_triangles(C, torch, n=1 << 16):
    """Exact second-order growth of n random triangles (F5, a = 1): the Fig. 1 check of
    the approximate D2, timed with HIP events on the launch stream."""
    import math
    import numpy as np
    p = C.Params(model=C.FR_HS1, fr0_abs=1e-5, z_init=19.0)
    rng = np.random.default_rng(7)
    k1, k2 = rng.uniform(0.005, 5.0, n), rng.uniform(0.005, 5.0, n)
    c = rng.uniform(-1.0, 1.0, n)
    k = np.sqrt(k1 * k1 + k2 * k2 + 2 * k1 * k2 * c)
    tri = torch.from_numpy(np.stack([k, k1, k2], axis=1)).cuda()
    out = torch.empty(n, 2, dtype=torch.float64, device="cuda")
    C.cola_growth_triangles(p, tri, 1.0, out)      # warm-up
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    C.cola_growth_triangles(p, tri, 1.0, out)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1)
    steps = math.ceil(math.log(1.0 / (1.0 / (1.0 + p.z_init))) / 1e-3)
    tflops = n * steps * TRIANGLE_FLOP_PER_STEP / (ms / 1e3) / 1e12
    return {"triangles": n, "ms": ms, "triangles_per_s": n / (ms / 1e3),
            "roofline": {"bound": "alu", "achieved": tflops, "peak": FP64_VECTOR_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": tflops / FP64_VECTOR_PEAK_TFLOPS}}


def bench_models(C, torch, steps=3):
    """ms per step of the other gravity models at the same 512^3 / 1024^3 size, from a
    mid-run step: LCDM, f(R) F5 with LCDM growth factors (no per-step LPT transforms),
    f(R) F5 with its own scale-dependent growth (six particle-grid inverse FFTs per step
    rebuild the LPT terms, App. A), and the symmetron of App. C (beta_* = 1, m_*/H0 = 2998,
    a_* = 0.5) timed after a_*, where its fifth force is on."""
    base = dict(np1d=512, nmesh1d=1024, box=1024.0, z_init=19.0, n_steps=30, seed=1)
    cases = {"lcdm": (dict(model=C.LCDM), 1),
             "fr5_lcdm_growth": (dict(model=C.FR_HS1, fr0_abs=1e-5, growth_mode=1), 1),
             "fr5_scale_dependent": (dict(model=C.FR_HS1, fr0_abs=1e-5, growth_mode=0), 1),
             "symmetron_scale_dependent": (dict(model=C.SYMMETRON, sym_beta=1.0,
                                                sym_mass=2997.92458, sym_astar=0.5), 16)}
    out = {}
    for name, (kw, first) in cases.items():
        p = C.Params(**base, **kw)
        st = C.State(p, device="cuda:0")
        C.cola_make_ic(p, st)
        for i in range(first):
            C.cola_step(p, st, i)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(first, first + steps):
            C.cola_step(p, st, i)
        torch.cuda.synchronize()
        out[name] = (time.perf_counter() - t0) * 1e3 / steps
        del st
        torch.cuda.empty_cache()
    return out


def run_timed(C, torch, p, st, warmup, steps, profile, log):
    """`warmup` untimed steps from initial conditions of their own, then exactly `steps`
    timed cola_step calls starting from new initial conditions.  A run has p.n_steps
    steps; when the timed steps go beyond one run they continue on further runs, each from
    new initial conditions made outside the timed intervals.  Every timed interval is
    bracketed by device synchronisation.  Returns (seconds, kernel profile, IC ms)."""
    ic_ms = []

    def new_run():
        torch.cuda.synchronize()
        t = time.perf_counter()
        C.cola_make_ic(p, st)
        torch.cuda.synchronize()
        ic_ms.append((time.perf_counter() - t) * 1e3)

    done = 0
    while done < warmup:
        new_run()
        k = min(p.n_steps, warmup - done)
        for i in range(k):
            C.cola_step(p, st, i)
        done += k
    torch.cuda.synchronize()
    log(f"{warmup} warm-up steps done; initial conditions {ic_ms[-1] if ic_ms else 0:.0f} ms")
    if profile:
        C.cola_profile_reset()
    elapsed, i = 0.0, p.n_steps
    left = steps
    while left:
        if i == p.n_steps:
            new_run()
            i = 0
        k = min(left, p.n_steps - i)
        if profile:
            C.cola_profile_enable(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for j in range(i, i + k):
            C.cola_step(p, st, j)
        torch.cuda.synchronize()
        elapsed += time.perf_counter() - t0
        C.cola_profile_enable(False)
        i += k
        left -= k
    prof = C.cola_profile_read() if profile else {}
    return elapsed, prof, ic_ms


def roofline_of(p, prof, traffic=None):
    """The kernel with the largest share of the timed steps: its algorithmic bytes per
    launch over its average launch time (HIP events on its launch stream)."""
    if not prof:
        return None
    dom, (dom_ms, dom_cnt) = max(prof.items(), key=lambda kv: kv[1][0])
    by = algorithmic_bytes(dom, p)
    avg_s = dom_ms / dom_cnt / 1e3
    ach = by / avg_s / 1e9 if by else None
    return {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS if ach else None,
            "traffic": traffic(dom) if traffic else None, "avg_launch_ms": avg_s * 1e3,
            "algorithmic_bytes_per_launch": by}


# Hardware-counter passes of counters_command (each within one pass's counter limits).
COUNTER_PASSES = [
    "SQ_WAVES SQ_INSTS_VALU SQ_INSTS_LDS SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR SQ_WAIT_INST_LDS "
    "SQ_LDS_BANK_CONFLICT SQ_BUSY_CYCLES",
    "TCP_UTCL1_TRANSLATION_MISS_sum TCP_UTCL1_TRANSLATION_HIT_sum TCP_UTCL1_REQUEST_sum "
    "TCP_UTCL1_STALL_MULTI_MISS_sum",
    "SQ_WAVE_CYCLES SQ_ACTIVE_INST_VALU SQ_ACTIVE_INST_LDS SQ_INST_LEVEL_VMEM SQ_ACTIVE_INST_ANY "
    "SQ_WAIT_ANY SQ_INSTS_SALU SQ_ACTIVE_INST_VMEM",
    "TCC_HIT_sum TCC_MISS_sum TCC_EA0_RDREQ_sum TCC_EA0_WRREQ_sum",
]
COUNTERS_FILE = "counters_fr5_1024_2048.md"


def counters_command(steps):
    """The rocprofv3 counter passes whose per-kernel ratios summarize_counters writes (D =
    output directory, REPO = repository root), one run of the headline workload each."""
    b = f"python3 $REPO/bench.py --steps {steps} --warmup 0 --headline-only --no-profile"
    cmds = ["cd /tmp && export TMPDIR=/tmp"]
    for i, c in enumerate(COUNTER_PASSES, 1):
        cmds.append(f"rocprofv3 --pmc {c} --output-format csv -d $D/p{i} -o p{i} -- {b}")
    cmds.append(f"python3 $REPO/bench.py --summarize-counters $D --steps {steps}")
    return "; ".join(cmds)


def summarize_counters(d, out_dir, steps):
    """Per-kernel ratios of the counter passes of counters_command(steps) under directory d,
    over the dispatches of timed steps 2..K (as in summarize_rocprof), written to out_dir
    as a markdown table: what the kernels spend their wave-cycles on, the LDS bank
    conflicts per LDS instruction, the address-translation (UTCL1) miss rate and the L2 hit
    rate."""
    import csv
    from collections import defaultdict
    from paper_1703_00879_amd import cola as C
    p = workload_params(C)
    n, np_ = p.nmesh1d, p.np1d
    acc = defaultdict(lambda: defaultdict(float))
    launches = defaultdict(set)
    nsteps = None
    for i in range(1, len(COUNTER_PASSES) + 1):
        with open(os.path.join(d, f"p{i}", f"p{i}_counter_collection.csv")) as fh:
            recs = list(csv.DictReader(fh))
        ids = sorted({int(r["Dispatch_Id"]) for r in recs if "k_gather" in r["Kernel_Name"]})[-steps:]
        lo, hi, nsteps = ids[0], ids[-1], len(ids) - 1
        for r in recs:
            if lo < int(r["Dispatch_Id"]) <= hi:
                name = _profile_name(r["Kernel_Name"], n, np_)
                acc[name][r["Counter_Name"]] += float(r["Counter_Value"])
                if i == 1:
                    launches[name].add(int(r["Dispatch_Id"]))

    def ratio(a, x, y, scale=1.0):
        return f"{scale * a[x] / a[y]:.2f}" if a.get(y) else "-"

    lines = [f"# Hardware counters of the PM step kernels: {WORKLOAD} (rocprofv3)", "",
             f"Source hash {source_hash()}; timed steps 2..{steps} of a {steps}-step run "
             f"({nsteps} steps), summed over each kernel's dispatches.", "",
             "Command (from the repository root on the GPU host, D = output directory, "
             "REPO = repository root):", "",
             "```", counters_command(steps).replace("; ", "\n"), "```", "",
             "Columns: wave instructions (VALU, LDS, and VMEM reads + writes: SQ_INSTS_VALU, "
             "SQ_INSTS_LDS, SQ_INSTS_VMEM_RD + _WR) per KiB of the kernel's algorithmic bytes; "
             "% of wave-cycles with a VALU or LDS instruction in flight and waiting on anything "
             "(SQ_ACTIVE_INST_VALU, SQ_ACTIVE_INST_LDS, SQ_WAIT_ANY over SQ_WAVE_CYCLES); LDS "
             "bank-conflict cycles per LDS instruction; UTCL1 address-translation misses per "
             "translation (MISS / (MISS + HIT)); L2 hits per L2 request (TCC_HIT / (TCC_HIT + "
             "TCC_MISS)).", "",
             "| kernel | launches/step | VALU/KiB | LDS/KiB | VMEM/KiB | VALU % | LDS % | wait % "
             "| bank conflicts/LDS | UTCL1 miss % | L2 hit % |",
             "|---|---|---|---|---|---|---|---|---|---|---|"]
    for name, a in sorted(acc.items(), key=lambda kv: -kv[1].get("SQ_WAVE_CYCLES", 0)):
        if not a.get("SQ_WAVES"):
            continue
        a = dict(a)
        nl = len(launches[name])
        ab = algorithmic_bytes(name, p)
        a["KiB"] = ab * nl / 1024 if ab else 0
        a["VMEM"] = a.get("SQ_INSTS_VMEM_RD", 0) + a.get("SQ_INSTS_VMEM_WR", 0)
        a["UTCL1"] = a.get("TCP_UTCL1_TRANSLATION_MISS_sum", 0) + a.get("TCP_UTCL1_TRANSLATION_HIT_sum", 0)
        a["TCC"] = a.get("TCC_HIT_sum", 0) + a.get("TCC_MISS_sum", 0)
        lines.append(
            f"| {name} | {nl / nsteps:g} | {ratio(a, 'SQ_INSTS_VALU', 'KiB')} "
            f"| {ratio(a, 'SQ_INSTS_LDS', 'KiB')} | {ratio(a, 'VMEM', 'KiB')} "
            f"| {ratio(a, 'SQ_ACTIVE_INST_VALU', 'SQ_WAVE_CYCLES', 100)} "
            f"| {ratio(a, 'SQ_ACTIVE_INST_LDS', 'SQ_WAVE_CYCLES', 100)} "
            f"| {ratio(a, 'SQ_WAIT_ANY', 'SQ_WAVE_CYCLES', 100)} "
            f"| {ratio(a, 'SQ_LDS_BANK_CONFLICT', 'SQ_INSTS_LDS')} "
            f"| {ratio(a, 'TCP_UTCL1_TRANSLATION_MISS_sum', 'UTCL1', 100)} "
            f"| {ratio(a, 'TCC_HIT_sum', 'TCC', 100)} |")
    os.makedirs(out_dir, exist_ok=True)
    with open(os.path.join(out_dir, COUNTERS_FILE), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return lines


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-models", action="store_true",
                    help="skip the per-step times of the other gravity models")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the ensemble and serving legs")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the headline run (what the rocprofv3 summary profiles)")
    ap.add_argument("--serve-requests", type=int, default=96,
                    help="requests in the serving stream (500 for the full stream)")
    ap.add_argument("--serving-only", action="store_true",
                    help="only the serving sweep (with --serve-requests), printed as JSON")
    ap.add_argument("--no-profile", action="store_true",
                    help="do not record per-kernel HIP events in the timed region")
    ap.add_argument("--summarize-rocprof", metavar="DIR",
                    help="condense rocprofv3 output under DIR into profiles/ and exit")
    ap.add_argument("--summarize-counters", metavar="DIR",
                    help="condense the hardware-counter passes under DIR into profiles/ and exit")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (three times), the "
                         "reference for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE readings")
    args = ap.parse_args()
    if args.summarize_rocprof:
        t = summarize_rocprof(args.summarize_rocprof, os.path.join(ROOT, "profiles"), args.steps,
                              args.warmup)
        print(json.dumps({k: v["bytes_per_launch"] for k, v in t["kernels"].items()}))
        return
    if args.summarize_counters:
        print("\n".join(summarize_counters(args.summarize_counters, os.path.join(ROOT, "profiles"),
                                           args.steps)))
        return
    if args.calibrate_copy:
        import torch
        n = 1 << 28
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "repeats": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the library runs each state on one GPU; a multi-GPU decomposition is not "
              "implemented)", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0:
        print("--steps must be >= 1 and --warmup >= 0", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1703_00879_amd import cola as C

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    if args.serving_only:
        torch.cuda.set_device(0)
        print(json.dumps({"serving": bench_serving(C, torch, requests=args.serve_requests)}))
        return

    torch.cuda.set_device(0)
    p = workload_params(C)
    st = C.State(p, device="cuda:0")
    log(f"state {C.cola_query_sizes(p)['total_bytes'] / 2 ** 30:.1f} GiB allocated")
    elapsed, prof, ic_ms = run_timed(C, torch, p, st, args.warmup, args.steps,
                                     not args.no_profile, log)
    log(f"{args.steps} timed steps: {elapsed:.3f} s")
    t0 = time.perf_counter()
    C.cola_power_spectrum(p, st)
    pk_ms = (time.perf_counter() - t0) * 1e3
    ok = bool(torch.isfinite(st.disp_f).all().item())
    del st
    torch.cuda.empty_cache()

    N = p.np1d ** 3
    ms_step = elapsed * 1e3 / args.steps
    yard = yardstick_bytes_for(p, C)
    kernels = {name: {"ms_per_step": ms / args.steps, "launches_per_step": cnt / args.steps}
               for name, (ms, cnt) in sorted(prof.items(), key=lambda kv: -kv[1][0])}
    out = {
        "metric": METRIC, "value": N * args.steps / elapsed, "unit": "particle-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "gravity": "f(R) Hu-Sawicki n=1", "fr0_abs": 1e-5,
                   "growth": "scale-dependent", "np1d": p.np1d, "nmesh1d": p.nmesh1d,
                   "box_mpc_h": p.box, "n_steps": p.n_steps, "seed": p.seed,
                   "parallelism": "single GPU"},
        "roofline": roofline_of(p, prof, traffic_for),
        # HBM fraction of the whole step: rocprofv3-counted bytes of a step (committed
        # profile of these kernel sources) over the measured step time; the modelled
        # yardstick figure beside it
        "hbm_frac_counted": (None if counted_bytes_per_step() is None else
                             counted_bytes_per_step() / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS),
        "counted_bytes_per_step": counted_bytes_per_step(),
        "hbm_frac_yardstick": yard / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS,
        "yardstick_bytes_per_step": yard,
        "ic_ms": ic_ms[-1], "pk_ms": pk_ms, "finite": ok,
        "kernels": kernels,
    }
    if not args.headline_only:
        q = secondary_params(C)
        st = C.State(q, device="cuda:0")
        e2, prof2, _ = run_timed(C, torch, q, st, 2, 10, not args.no_profile, log)
        del st
        torch.cuda.empty_cache()
        ms2 = e2 * 1e3 / 10
        out["secondary"] = {
            "workload": SECONDARY, "steps": 10, "warmup": 2, "ms_per_step": ms2,
            "particle_steps_per_s": q.np1d ** 3 * 10 / e2,
            "hbm_frac_yardstick": yardstick_bytes_for(q, C) / (ms2 / 1e3) / 1e9 / HBM_PEAK_GBS,
            "roofline": roofline_of(q, prof2),
            "kernels": {name: {"ms_per_step": ms / 10, "launches_per_step": cnt / 10}
                        for name, (ms, cnt) in sorted(prof2.items(), key=lambda kv: -kv[1][0])}}
        log(f"secondary: {ms2:.2f} ms/step")
        out["growth_triangles"] = bench_triangles(C, torch)
        if not args.no_models:
            out["other_models_ms_per_step"] = bench_models(C, torch)
        if not args.no_serving:
            log("ensemble and serving")
            out["ensemble"] = bench_ensemble(C, torch)
            out["serving"] = bench_serving(C, torch, requests=args.serve_requests)
    if not args.no_cpu_baseline and not args.headline_only:
        log("timing the FP64 oracle on the host")
        out["cpu_baseline"] = cpu_baseline()
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out))


if __name__ == "__main__":
    main()
