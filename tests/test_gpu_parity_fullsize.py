"""Full-size GPU checks at the benchmark workload and at the largest supported mesh.

The benchmark workload runs in the same launch configuration bench.py times: nDGP with
r_c H0 = 1 and Vainshtein screening (Gaussian smoothing, R = 1 Mpc/h), 512^3 particles,
a 1024^3 mesh, L = 1024 Mpc/h and 30 steps.

The FP64 oracle cannot run a 1024^3 mesh, so two checks use planar configurations. There
the oracle's 1D reduction (oracle.planar, pinned against the 3D oracle) gives every cell
and every particle exactly.
- PM force: every cell of the density, screened-source and three force meshes and every
  particle force is compared, for displacements along each of the three axes.
- One COLA step: every particle's displacement and velocity is compared.

The same planar check runs on radix-3 meshes of 192^3, 384^3 and 768^3 cells (the sizes
of the serving mix) and of 1536^3 cells (the largest radix-3 plan).  The white noise and the scale-dependent growth table are checked on
samples the oracle computes one by one.

Tolerances are those of test_gpu_parity:
- meshes and forces: 1e-5 relative rms (screened source 1e-4);
- positions: 1e-3 cells rms;
- growth tables: 1e-10.
"""

import gc
import math

import numpy as np
import pytest

from oracle.growth import solve_growth
from oracle.models import Model
from oracle.planar import planar_pm, planar_step
from oracle.rng import splitmix64, to_unit
from paper_1703_00879_amd import cola as C
from tests.test_gpu_parity import record, to_oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

WORKLOAD = C.Params(model=C.NDGP, rc_h0=1.0, screening=1, filter=C.SMOOTH_GAUSS, r_smooth=1.0,
                    np1d=512, nmesh1d=1024, box=1024.0, z_init=19.0, n_steps=30, seed=1)


@pytest.fixture(autouse=True)
def _release_memory():
    yield
    gc.collect()
    torch.cuda.empty_cache()


def profile(n_p, box, seed, amp=1.0):
    """Per-plane displacement profile (Mpc/h): three sine modes plus seeded jitter."""
    q = np.arange(n_p) * box / n_p
    rng = np.random.default_rng(seed)
    return amp * (5.0 * np.sin(2 * np.pi * 3 * q / box) + 1.5 * np.cos(2 * np.pi * 17 * q / box + 0.4)
                  + 0.3 * np.sin(2 * np.pi * 150 * q / box) + 0.5 * rng.standard_normal(n_p))


def planar_view(x, ax, n):
    """(n, n, n) view of a flat n^3 tensor and the broadcast shape of a profile along ax."""
    shape = [1, 1, 1]
    shape[ax] = n
    return x.view(n, n, n), shape


def fill_planar(dst_flat, prof, ax, n):
    """dst (n^3 flat) <- prof broadcast along axis ax."""
    v, shape = planar_view(dst_flat, ax, n)
    v.copy_(torch.from_numpy(prof.astype(np.float32)).to(v.device).view(shape).expand(n, n, n))


def relrms_planar(flat, prof, ax, n, chunk=64):
    """||flat - broadcast(prof)|| / ||broadcast(prof)|| over the n^3 values, in FP64."""
    v, shape = planar_view(flat, ax, n)
    e = torch.from_numpy(np.asarray(prof, dtype=np.float64)).to(flat.device).view(shape)
    num = den = 0.0
    for x0 in range(0, n, chunk):
        blk = v[x0:x0 + chunk].double()
        eb = e[x0:x0 + chunk] if ax == 0 else e
        d = blk - eb
        num += float((d * d).sum())
        den += float((eb * eb).expand_as(blk).sum())
    return math.sqrt(num / den)


def rms(flat, chunk=1 << 26):
    s = 0.0
    for i in range(0, flat.numel(), chunk):
        b = flat[i:i + chunk].double()
        s += float((b * b).sum())
    return math.sqrt(s / flat.numel())


@pytest.mark.parametrize("ax", [0, 1, 2])
def test_fullsize_planar_pm_force(ax):
    p = WORKLOAD
    n, n_p = p.nmesh1d, p.np1d
    N, M = n_p ** 3, n ** 3
    st = C.State(p)
    C.cola_prepare(p, st)
    u1 = profile(n_p, p.box, seed=ax)
    st.disp_f.zero_()
    fill_planar(st.disp_f[ax], u1, ax, n_p)
    F = torch.empty(3, N, dtype=torch.float32, device="cuda")
    mesh = torch.empty(5, M, dtype=torch.float32, device="cuda")
    a = 0.75
    C.cola_pm_force(p, st, a, F, mesh)
    torch.cuda.synchronize()
    pl = planar_pm(u1.astype(np.float32).astype(np.float64), to_oracle(p), a)
    # the fixed-point deposit makes every cell of a plane bitwise equal
    v, _ = planar_view(mesh[0], ax, n)
    others = tuple(d for d in range(3) if d != ax)
    assert float((torch.amax(v, dim=others) - torch.amin(v, dim=others)).abs().max()) == 0.0
    e = dict(rho=relrms_planar(mesh[0], pl["rho"], ax, n),
             src=relrms_planar(mesh[1], pl["src"], ax, n),
             f=relrms_planar(mesh[2 + ax], pl["force"], ax, n),
             fp=relrms_planar(F[ax], pl["fp"], ax, n_p))
    scale_mesh, scale_p = rms(mesh[2 + ax]), rms(F[ax])
    e["f_across"] = max(rms(mesh[2 + o]) for o in others) / scale_mesh
    e["fp_across"] = max(rms(F[o]) for o in others) / scale_p
    record(f"fullsize_planar_pm_force_ax{ax}", **e)
    assert e["rho"] < 1e-5 and e["src"] < 1e-4 and e["f"] < 1e-5 and e["fp"] < 1e-5, e
    assert e["f_across"] < 1e-5 and e["fp_across"] < 1e-5, e


# Radix-3 meshes at the sizes of the serving mix (n_p = 384, 192, 96 on 768^3, 384^3,
# 192^3 meshes, L = 2 n_p Mpc/h): f(R) with its potential screening and two sources,
# screened nDGP with one combined source, LCDM; and f(R) on the largest radix-3 mesh,
# 1536^3 (about 170 GB of device memory with the test's mesh outputs).
RADIX3 = [(C.FR_HS1, 384, 0), (C.NDGP, 192, 1), (C.LCDM, 96, 2), (C.FR_HS1, 768, 2)]


@pytest.mark.parametrize("model,n_p,ax", RADIX3)
def test_planar_pm_force_radix3_sizes(model, n_p, ax):
    p = C.Params(model=model, fr0_abs=1e-5, rc_h0=1.0, screening=1, r_smooth=1.0, np1d=n_p,
                 nmesh1d=2 * n_p, box=2.0 * n_p, z_init=19.0, n_steps=20, seed=3)
    n, N, M = p.nmesh1d, n_p ** 3, p.nmesh1d ** 3
    st = C.State(p)
    C.cola_prepare(p, st)
    u1 = profile(n_p, p.box, seed=11 + ax)
    st.disp_f.zero_()
    fill_planar(st.disp_f[ax], u1, ax, n_p)
    F = torch.empty(3, N, dtype=torch.float32, device="cuda")
    mesh = torch.empty(5, M, dtype=torch.float32, device="cuda")
    a = 0.8
    C.cola_pm_force(p, st, a, F, mesh)
    torch.cuda.synchronize()
    pl = planar_pm(u1.astype(np.float32).astype(np.float64), to_oracle(p), a)
    e = dict(rho=relrms_planar(mesh[0], pl["rho"], ax, n),
             src=relrms_planar(mesh[1], pl["src"], ax, n),
             f=relrms_planar(mesh[2 + ax], pl["force"], ax, n),
             fp=relrms_planar(F[ax], pl["fp"], ax, n_p))
    record(f"planar_pm_force_radix3_model{model}_np{n_p}", **e)
    assert e["rho"] < 1e-5 and e["src"] < 1e-4 and e["f"] < 1e-5 and e["fp"] < 1e-5, e


def test_fullsize_planar_step():
    """One cola_step (step 20 of 30) of the benchmark workload on a planar state: u, v,
    Psi1, Psi2 along x as functions of the lattice index ix."""
    p = WORKLOAD
    n_p, N = p.np1d, p.np1d ** 3
    st = C.State(p)
    C.cola_prepare(p, st)
    u1 = profile(n_p, p.box, seed=5).astype(np.float32).astype(np.float64)
    v1 = (0.2 * profile(n_p, p.box, seed=6)).astype(np.float32).astype(np.float64)
    psi1 = (0.6 * profile(n_p, p.box, seed=7)).astype(np.float32).astype(np.float64)
    psi2 = (-0.1 * profile(n_p, p.box, seed=8)).astype(np.float32).astype(np.float64)
    st.disp_f.zero_()
    st.vel_f.zero_()
    fill_planar(st.disp_f[0], u1, 0, n_p)
    fill_planar(st.vel_f[0], v1, 0, n_p)
    # per-particle LPT store of k-independent growth: Psi1 [3][N] at 0, Psi2 at disp_bytes
    lptf = st.lpt.view(torch.float32)
    off2 = st.sizes["disp_bytes"] // 4
    P1, P2 = lptf[:3 * N].view(3, N), lptf[off2:off2 + 3 * N].view(3, N)
    P1.zero_()
    P2.zero_()
    fill_planar(P1[0], psi1, 0, n_p)
    fill_planar(P2[0], psi2, 0, n_p)
    i = 20
    st.c.next_step = i
    C.cola_step(p, st, i)
    torch.cuda.synchronize()
    assert st.next_step == i + 1
    u_or, v_or = planar_step(u1, v1, psi1, psi2, to_oracle(p), i)
    cell = p.box / p.nmesh1d
    e = dict(u_cells=relrms_planar(st.disp_f[0], u_or, 0, n_p) * rms_np(u_or) / cell,
             v=relrms_planar(st.vel_f[0], v_or, 0, n_p),
             u_across_cells=max(rms(st.disp_f[1]), rms(st.disp_f[2])) / cell)
    record("fullsize_planar_step", **e)
    assert e["u_cells"] < 1e-3 and e["v"] < 1e-5 and e["u_across_cells"] < 1e-3, e


def rms_np(x):
    return float(np.sqrt(np.mean(np.asarray(x, dtype=np.float64) ** 2)))


def test_fullsize_white_noise_samples():
    """The 512^3 particle-grid white noise at 20000 sampled grid points equals the
    oracle's SplitMix64 / Box-Muller value there (integer stream exact; FP32 Box-Muller)."""
    p = WORKLOAD
    N = p.np1d ** 3
    out = torch.empty(N, dtype=torch.float32, device="cuda")
    C.cola_white_noise(p, out)
    torch.cuda.synchronize()
    j = np.unique(np.random.default_rng(3).integers(0, N, 20000)).astype(np.uint64)
    j = np.concatenate([j, np.array([0, N - 1], dtype=np.uint64)])
    u0 = to_unit(splitmix64(p.seed, 2 * j))
    u1 = to_unit(splitmix64(p.seed, 2 * j + np.uint64(1)))
    ref = np.sqrt(-2.0 * np.log(u0)) * np.cos(2.0 * np.pi * u1)
    g = out[torch.from_numpy(j.astype(np.int64)).cuda()].cpu().numpy().astype(np.float64)
    err = np.max(np.abs(g - ref) / np.maximum(1.0, np.abs(ref)))
    record("fullsize_white_noise", max_err=err)
    assert err < 2e-5


def test_fullsize_scale_dependent_growth_table_samples():
    """f(R) F5 on the 512^3 particle grid (196609 distinct |nu|^2 per slice): sampled
    entries of three slices against the oracle's ODE solution at those k."""
    p = WORKLOAD.with_(model=C.FR_HS1, fr0_abs=1e-5)
    st = C.State(p)
    C.cola_prepare(p, st)
    po = to_oracle(p)
    model = Model(po)
    n2 = np.array([0, 1, 2, 3, 17, 250, 4096, 33333, 100000, 196608])
    k = 2.0 * np.pi * np.sqrt(n2.astype(np.float64)) / p.box
    a_grid = po.a_ini + np.arange(p.n_steps + 1) * (1.0 - po.a_ini) / p.n_steps
    G = solve_growth(k, a_grid, po.omega_m, model.mu, model.gamma2_orth, po.a_ini)
    worst = 0.0
    for i in (0, 11, p.n_steps):
        tab = C.cola_growth_table(p, st, i)
        assert tab.shape == (3 * (p.np1d // 2) ** 2 + 1, 6)
        ref = G[i]
        got = tab[n2]
        rel = np.abs(got - ref) / np.maximum(np.abs(ref), 1e-300)
        rel[ref == 0] = np.abs(got[ref == 0])
        worst = max(worst, float(rel.max()))
    record("fullsize_growth_table", max_rel=worst)
    assert worst < 1e-10


def test_maximum_size_planar_forces():
    """The largest supported configuration, 1024^3 particles on a 2048^3 mesh (64-bit
    element offsets in every FFT pass): per-particle planar forces of nDGP with Vainshtein
    screening against the oracle's 1D reduction.  Skipped if the device has too little
    free memory for the ~265 GB state."""
    p = WORKLOAD.with_(np1d=1024, nmesh1d=2048, box=2048.0)
    n_p, N = p.np1d, p.np1d ** 3
    sizes = C.cola_query_sizes(p)
    gc.collect()
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    need = sizes["total_bytes"] + 12 * N + 5 * 256 + (4 << 30)
    if free < need:
        pytest.skip(f"needs {need / 1e9:.0f} GB of device memory, {free / 1e9:.0f} GB free")
    st = C.State(p)
    C.cola_prepare(p, st)
    u1 = profile(n_p, p.box, seed=9)
    st.disp_f.zero_()
    fill_planar(st.disp_f[0], u1, 0, n_p)
    F = torch.empty(3, N, dtype=torch.float32, device="cuda")
    a = 0.9
    C.cola_pm_force(p, st, a, F, None)
    torch.cuda.synchronize()
    pl = planar_pm(u1.astype(np.float32).astype(np.float64), to_oracle(p), a)
    e = dict(fp=relrms_planar(F[0], pl["fp"], 0, n_p),
             fp_across=max(rms(F[1]), rms(F[2])) / rms(F[0]))
    record("maximum_size_planar_forces", **e)
    assert e["fp"] < 1e-5 and e["fp_across"] < 1e-5, e


def _sparse_modes(n, box, rng):
    """Five particle-grid modes (nu_x, nu_y, nu_z), 0 < nu_z < n/2: a low mode, an x- and a
    y-Nyquist mode (their i k_x / i k_y factor is zero), the largest |nu|^2 with a
    non-zero gradient, and a mode next to k = 0; amplitudes make each field O(1) Mpc/h."""
    h = n // 2
    nus = [(3, 5, 7), (-h, 2, 9), (h - 1, -(h - 1), h - 1), (0, -h, 3), (-1, 0, 1)]
    out = []
    for nu in nus:
        k = 2 * np.pi * math.sqrt(sum(v * v for v in nu)) / box
        a1, a2 = (rng.standard_normal(2) + 1j * rng.standard_normal(2)) * n ** 3 / k
        out.append((nu, a1, a2))
    return out


@pytest.mark.parametrize("n_p", [512, 1024])
def test_fullsize_scale_dependent_lpt_step(n_p):
    """One cola_step of F5 with scale-dependent growth at 512^3 particles / 1024^3 cells and
    at 1024^3 / 2048^3 (the headline size; skipped when the device lacks the memory) with
    the particles on the lattice (u = v = 0, so the density is exactly uniform and the PM
    force exactly zero) and phi1_k, phi2_k zero except at five modes.  The step then gives
    v = -dtau_kick L''(q, a_i) and u = dtau_drift v + Delta_i(q): the per-step LPT synthesis
    (App. A) through the particle-grid transforms and the gather, compared particle by
    particle with the oracle's direct summation over the modes with its FP64 growth factors
    (every particle at 512^3; every particle of every eighth lattice plane at 1024^3)."""
    p = C.Params(model=C.FR_HS1, fr0_abs=1e-5, screening=1, growth_mode=0, np1d=n_p,
                 nmesh1d=2 * n_p, box=2.0 * n_p, z_init=19.0, n_steps=20, seed=1)
    N = n_p ** 3
    sizes = C.cola_query_sizes(p)
    gc.collect()
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    need = sizes["total_bytes"] + (4 << 30)
    if free < need:
        pytest.skip(f"needs {need / 1e9:.0f} GB of device memory, {free / 1e9:.0f} GB free")
    st = C.State(p)
    C.cola_prepare(p, st)
    st.disp_f.zero_()
    st.vel_f.zero_()
    st.lpt.zero_()
    # phi1_k at byte 0, phi2_k at half of lpt_bytes: padded half-complex particle-grid
    # fields, element (ix, iy, iz) at ix * plane + iy * pitch + iz (complex values)
    pitch = (n_p // 2 + 1 + 15) // 16 * 16
    plane = n_p * pitch + 16
    lptc = st.lpt.view(torch.float32).view(-1, 2)
    off2 = sizes["lpt_bytes"] // 2 // 8
    rng = np.random.default_rng(n_p)
    modes = _sparse_modes(n_p, p.box, rng)
    for nu, a1, a2 in modes:
        e = (nu[0] % n_p) * plane + (nu[1] % n_p) * pitch + nu[2]
        lptc[e] = torch.tensor([a1.real, a1.imag], dtype=torch.float32)
        lptc[off2 + e] = torch.tensor([a2.real, a2.imag], dtype=torch.float32)
    i = 7
    st.c.next_step = i
    C.cola_step(p, st, i)
    torch.cuda.synchronize()
    # oracle: growth factors at the modes' k, the time grid, direct summation
    from oracle.cola import time_grid
    from oracle.lpt import lpt_field_sparse
    po = to_oracle(p)
    model = Model(po)
    a_grid, kick, drift = time_grid(po)
    ks = np.array([2 * np.pi * math.sqrt(sum(v * v for v in nu)) / p.box for nu, _, _ in modes])
    G = solve_growth(ks, a_grid[i:i + 2], po.omega_m, model.mu, model.gamma2_orth, po.a_ini)
    G0, G1 = G[0], G[1]
    lpp = [(nu, G0[m, 2] * complex(np.complex64(a1)) + G0[m, 5] * complex(np.complex64(a2)))
           for m, (nu, a1, a2) in enumerate(modes)]
    dlt = [(nu, (G1[m, 0] - G0[m, 0]) * complex(np.complex64(a1))
            + (G1[m, 3] - G0[m, 3]) * complex(np.complex64(a2)))
           for m, (nu, a1, a2) in enumerate(modes)]
    step = 1 if n_p <= 512 else 8
    chunk = 32 if n_p <= 512 else 8
    num_u = den_u = num_v = den_v = 0.0
    u3 = st.disp_f.view(3, n_p, n_p, n_p)
    v3 = st.vel_f.view(3, n_p, n_p, n_p)
    for x0 in range(0, n_p, chunk * step):
        planes = np.arange(x0, min(n_p, x0 + chunk * step), step)
        L2 = lpt_field_sparse(lpp, n_p, p.box, planes)
        D = lpt_field_sparse(dlt, n_p, p.box, planes)
        v_or = -kick[i] * L2
        u_or = drift[i] * v_or + D
        sel = torch.from_numpy(planes).cuda()
        ug = u3[:, sel].cpu().numpy().astype(np.float64)
        vg = v3[:, sel].cpu().numpy().astype(np.float64)
        num_u += float(((ug - u_or) ** 2).sum())
        den_u += float((u_or ** 2).sum())
        num_v += float(((vg - v_or) ** 2).sum())
        den_v += float((v_or ** 2).sum())
    e = dict(u=math.sqrt(num_u / den_u), v=math.sqrt(num_v / den_v),
             u_rms=math.sqrt(den_u / (3 * N / step)))
    record(f"fullsize_scale_dependent_lpt_step_np{n_p}", **e)
    assert e["u_rms"] > 1e-3   # the modes move the particles
    assert e["u"] < 1e-5 and e["v"] < 1e-5, e


def test_fullsize_initial_conditions_512():
    """cola_make_ic of F5 with scale-dependent growth at 512^3 particles (the 8-column
    particle-grid tiles of the Hessian, potential and LPT transforms) against the oracle's
    2LPT fields on the same seeded white noise: u = Psi1 - (3/7) Psi2 at every particle."""
    from oracle import fftlib
    from oracle.lpt import initial_fields
    from oracle.spectrum import InitialSpectrum
    p = C.Params(model=C.FR_HS1, fr0_abs=1e-5, screening=1, growth_mode=0, np1d=512,
                 nmesh1d=1024, box=1024.0, z_init=19.0, n_steps=20, seed=1)
    st = C.State(p)
    C.cola_make_ic(p, st)
    torch.cuda.synchronize()
    u = st.disp_f.cpu().numpy()
    del st
    gc.collect()
    torch.cuda.empty_cache()
    po = to_oracle(p)
    fftlib.set_workers(min(16, len(__import__("os").sched_getaffinity(0))))
    try:
        f = initial_fields(po, InitialSpectrum(po))
    finally:
        fftlib.set_workers(1)
    num = den = 0.0
    for c in range(3):
        ref = (f["psi1"][c] - (3.0 / 7.0) * f["psi2"][c]).reshape(-1)
        d = u[c].astype(np.float64) - ref
        num += float(d @ d)
        den += float(ref @ ref)
    e = dict(u=math.sqrt(num / den), u_rms=math.sqrt(den / u.size))
    record("fullsize_initial_conditions_512", **e)
    assert e["u"] < 1e-5, e


def test_fullsize_power_spectrum_1024():
    """P(k) on a 1024^3 mesh: a 512^3-particle F5 state after its initial conditions (the
    scale-dependent workload at half the headline size).  The GPU's own density mesh (rho
    from cola_pm_force) goes through the oracle's FP64 FFT and shell binning, and
    cola_power_spectrum (the same deposit, bitwise, then the FP32 FFT and FP64 shell sums)
    must agree per bin to 0.1 % up to half the mesh Nyquist frequency, with the same mode
    counts."""
    from oracle import fftlib
    from oracle.pk import power_spectrum_mesh
    p = C.Params(model=C.FR_HS1, fr0_abs=1e-5, np1d=512, nmesh1d=1024, box=1024.0, n_steps=20,
                 seed=11)
    st = C.State(p)
    C.cola_make_ic(p, st)
    n, nb = p.nmesh1d, p.nmesh1d // 4 + 1
    k, P, nm = C.cola_power_spectrum(p, st, nbins=nb)
    M = n ** 3
    mesh = torch.empty(5, M, dtype=torch.float32, device="cuda")
    C.cola_pm_force(p, st, 0.05, None, mesh)
    torch.cuda.synchronize()
    rho = mesh[0].cpu().numpy()
    del mesh, st
    gc.collect()
    torch.cuda.empty_cache()
    delta = rho.astype(np.float64).reshape(n, n, n)
    delta -= 1.0
    del rho
    w0 = fftlib.workers()
    fftlib.set_workers(16)
    try:
        ko, Po, nmo = power_spectrum_mesh(delta, p.box, nb)
    finally:
        fftlib.set_workers(w0)
    del delta
    assert np.array_equal(nm[1:], nmo[1:].astype(np.int64))
    e_p = float(np.max(np.abs(P[1:] / Po[1:] - 1)))
    e_k = float(np.max(np.abs(k[1:] / ko[1:] - 1)))
    record("fullsize_pk_1024", pk=e_p, k=e_k)
    assert e_p < 1e-3, f"P(k) {e_p:.2e}"
    assert e_k < 1e-6, f"k {e_k:.2e}"
