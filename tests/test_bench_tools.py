"""Host-side pieces of bench.py: the algorithmic byte counts, the yardstick, the mapping of
kernel symbols to step names, and the rocprofv3 summary built from synthetic CSV files."""

import csv
import importlib.util
import json
import os

import pytest

from paper_1703_00879_amd import cola as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_yardstick_per_particle_step(bench):
    # 1300 B per screened scale-independent particle-step at M = 8N; LCDM 852 B; with the
    # per-step LPT synthesis of scale-dependent growth 1428 B (the headline workload)
    p = bench.workload_params(C)
    N = p.np1d ** 3
    assert p.nmesh1d ** 3 == 8 * N
    assert bench.yardstick_bytes_for(p, C) == 1428 * N
    assert bench.yardstick_bytes_for(p.with_(model=C.LCDM), C) == 852 * N
    assert bench.yardstick_bytes_for(p.with_(model=C.NDGP), C) == 1300 * N
    assert bench.yardstick_bytes_for(p.with_(model=C.FR_HS1, growth_mode=1), C) == 1300 * N
    q = bench.secondary_params(C)
    assert bench.yardstick_bytes_for(q, C) == 1300 * q.np1d ** 3


def test_algorithmic_bytes(bench):
    p = bench.workload_params(C)
    n, N = p.nmesh1d, p.np1d ** 3
    M, H = n ** 3, n * n * (n // 2 + 1)
    ab = lambda k: bench.algorithmic_bytes(k, p)  # noqa: E731
    assert ab("gather_kick_drift") == 12 * M + 72 * N
    assert ab("fft_c2r_z3") == 24 * H + 12 * M
    assert ab("fft_x_fwd_smooth") == 16 * H and ab("fft_x_fwd_pot") == 24 * H
    assert ab("fft_x_fwd_force_1src") == 24 * H and ab("fft_x_fwd_force") == 32 * H
    assert ab("deposit") == 12 * N + 4 * M and ab("bin_scatter") == 24 * N
    Hp = p.np1d ** 2 * (p.np1d // 2 + 1)
    assert ab("lpt_fft_x_inv") == 32 * Hp and ab("lpt_fft_y_inv") == 16 * Hp
    assert ab("lpt_fft_y_inv_yz") == 24 * Hp and ab("lpt_fft_c2r_z3") == 24 * Hp + 12 * N
    assert ab("no_such_kernel") is None


@pytest.mark.parametrize("symbol,name", [
    ("void cola::k_fft_col<1024, -1, 0, 16>(HIP_vector_type<float, 2u>*, long)", "fft_y_fwd"),
    ("void cola::k_fft_col<1024, 1, 0, 16>(HIP_vector_type<float, 2u>*, long)", "fft_y_inv"),
    ("void cola::k_fft_col_fwd_force<1024, false>(float2 const*)", "fft_x_fwd_force_1src"),
    ("void cola::k_fft_col_fwd_force<1024, true>(float2 const*)", "fft_x_fwd_force"),
    ("void cola::k_fft_col_fwd_op<1024, 3, false>(float2*)", "fft_x_fwd_smooth"),
    ("void cola::k_fft_col_fwd_op<1024, 2, true>(float2*)", "fft_x_fwd_pot"),
    ("void cola::k_fft_screen_row<512, 2>(float2*)", "fft_z_screen"),
    ("void cola::k_fft_c2r_row3<512>(float2 const*)", "fft_c2r_z3"),
    ("void cola::k_gather<0>(cola::GatherDev, long)", "gather_kick_drift"),
    ("void cola::k_bin<0, true>(float const*)", "bin_count"),
    ("void cola::k_bin<1, true>(float const*)", "bin_scatter"),
    ("void cola::k_deposit_tiles<16>(float4 const*)", "deposit"),
    ("void cola::k_fft_col<512, 1, 4, 8>(HIP_vector_type<float, 2u>*, long)", "fft_x_inv_lpt"),
    ("void cola::k_fft_col<512, 1, 0, 16>(HIP_vector_type<float, 2u>*, long)", "lpt_fft_y_inv"),
    ("void cola::k_fft_c2r_row<256>(float2 const*)", "lpt_fft_c2r_z"),
    ("void cola::k_fft_col_lpt<512>(float2 const*)", "lpt_fft_x_inv"),
    ("void cola::k_fft_col_inv_yz<512>(float2 const*)", "lpt_fft_y_inv_yz"),
    ("void cola::k_fft_c2r_row3<256>(float2 const*)", "lpt_fft_c2r_z3"),
])
def test_profile_names(bench, symbol, name):
    assert bench._profile_name(symbol, 1024, 512) == name


def _write(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_summarize_rocprof_on_synthetic_runs(bench, tmp_path):
    """Three timed steps: the gather ends each step; the summary covers the two steps
    after the first gather, scales FETCH_SIZE and WRITE_SIZE by the factors that make a
    1 GiB copy read 1 GiB, and writes both profile files."""
    d = tmp_path / "prof"
    gather = "void cola::k_gather<0>(cola::GatherDev, long)"
    c2r3 = "void cola::k_fft_c2r_row3<1024>(float2 const*)"
    trace, fetch, write = [], [], []
    did = 0
    for step in range(3):
        for name, ms, kib_r, kib_w in ((c2r3, 5.0, 1000.0, 3000.0), (gather, 4.0, 2000.0, 500.0)):
            did += 1
            t0 = 1_000_000_000 * did
            trace.append([did, name, t0, t0 + int(ms * 1e6)])
            fetch.append([did, name, "FETCH_SIZE", kib_r])
            write.append([did, name, "WRITE_SIZE", kib_w])
    _write(str(d / "trace" / "trace_kernel_trace.csv"),
           ["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"], trace)
    _write(str(d / "fetch" / "fetch_counter_collection.csv"),
           ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"], fetch)
    _write(str(d / "write" / "write_counter_collection.csv"),
           ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"], write)
    gib_kib = (1 << 30) / 1024
    copy = "__amd_rocclr_copyBuffer"
    _write(str(d / "cfetch" / "cfetch_counter_collection.csv"),
           ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"],
           [[1, copy, "FETCH_SIZE", gib_kib / 2], [2, copy, "FETCH_SIZE", gib_kib / 2]])
    _write(str(d / "cwrite" / "cwrite_counter_collection.csv"),
           ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"],
           [[1, copy, "WRITE_SIZE", gib_kib]])
    out = tmp_path / "profiles"
    t = bench.summarize_rocprof(str(d), str(out), steps=3)
    assert t["fetch_scale"] == pytest.approx(2.0) and t["write_scale"] == pytest.approx(1.0)
    g, c = t["kernels"]["gather_kick_drift"], t["kernels"]["fft_c2r_z3"]
    assert g["launches_per_step"] == 1 and c["launches_per_step"] == 1
    assert g["avg_ms"] == pytest.approx(4.0) and c["ms_per_step"] == pytest.approx(5.0)
    assert g["bytes_per_launch"] == pytest.approx(1024 * (2 * 2000.0 + 500.0))
    assert c["bytes_per_launch"] == pytest.approx(1024 * (2 * 1000.0 + 3000.0))
    saved = json.load(open(out / bench.TRAFFIC_FILE))
    assert saved["source_hash"] == bench.source_hash()
    md = open(out / bench.PROFILE_FILE).read()
    assert "| fft_c2r_z3 | 1 | 5.000 |" in md and "rocprofv3 --kernel-trace" in md


def test_summarize_counters_on_synthetic_runs(bench, tmp_path):
    """Three timed steps of the counter passes: the summary covers the two steps after the
    first gather and gives per-kernel ratios of the summed counters."""
    d = tmp_path / "cnt"
    gather = "void cola::k_gather<0>(cola::GatherDev, long)"
    values = {"SQ_WAVES": 10.0, "SQ_INSTS_VALU": 300.0, "SQ_INSTS_LDS": 0.0,
              "SQ_INSTS_VMEM_RD": 20.0, "SQ_INSTS_VMEM_WR": 2.0, "SQ_WAIT_INST_LDS": 0.0,
              "SQ_LDS_BANK_CONFLICT": 0.0, "SQ_BUSY_CYCLES": 100.0,
              "TCP_UTCL1_TRANSLATION_MISS_sum": 1.0, "TCP_UTCL1_TRANSLATION_HIT_sum": 3.0,
              "TCP_UTCL1_REQUEST_sum": 4.0, "TCP_UTCL1_STALL_MULTI_MISS_sum": 0.0,
              "SQ_WAVE_CYCLES": 1000.0, "SQ_ACTIVE_INST_VALU": 50.0, "SQ_ACTIVE_INST_LDS": 0.0,
              "SQ_INST_LEVEL_VMEM": 0.0, "SQ_ACTIVE_INST_ANY": 60.0, "SQ_WAIT_ANY": 250.0,
              "SQ_INSTS_SALU": 5.0, "SQ_ACTIVE_INST_VMEM": 0.0,
              "TCC_HIT_sum": 9.0, "TCC_MISS_sum": 1.0, "TCC_EA0_RDREQ_sum": 1.0,
              "TCC_EA0_WRREQ_sum": 1.0}
    for i, names in enumerate(bench.COUNTER_PASSES, 1):
        rows = [[step + 1, gather, c, values[c]] for step in range(3) for c in names.split()]
        _write(str(d / f"p{i}" / f"p{i}_counter_collection.csv"),
               ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"], rows)
    out = tmp_path / "profiles"
    lines = bench.summarize_counters(str(d), str(out), steps=3)
    row = [ln for ln in lines if ln.startswith("| gather_kick_drift |")]
    assert len(row) == 1
    cells = [c.strip() for c in row[0].strip("|").split("|")]
    # launches/step, then VALU % 5, LDS % 0, wait % 25, UTCL1 miss 25 %, L2 hit 90 %
    assert cells[1] == "1"
    assert cells[5:8] == ["5.00", "0.00", "25.00"]
    assert cells[9:11] == ["25.00", "90.00"]
    md = open(out / bench.COUNTERS_FILE).read()
    assert bench.source_hash() in md and "rocprofv3 --pmc" in md
