"""Serving loop on the GPU: each run's result is the same alone and in the mix.

Four requests of different models and sizes (LCDM, F5 on a radix-3 mesh, screened nDGP,
the symmetron) arrive at staggered times and are interleaved on two streams by the
request loop, all states resident at once.  Each is then run alone on the default
stream.  Final displacements and velocities must agree bit for bit: the deposit sums in
integers, and no kernel keeps state between calls or depends on what else is running.
"""

import pytest

from paper_1703_00879_amd import cola as C
from paper_1703_00879_amd.serve import GpuEngine, Request, Server, summarize

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

REQS = [
    dict(model=C.LCDM, np1d=32, nmesh1d=64, box=64.0, n_steps=5, seed=1),
    dict(model=C.FR_HS1, fr0_abs=1e-5, np1d=24, nmesh1d=48, box=48.0, n_steps=4, seed=2),
    dict(model=C.NDGP, rc_h0=1.0, np1d=32, nmesh1d=64, box=64.0, n_steps=6, seed=3),
    dict(model=C.SYMMETRON, np1d=16, nmesh1d=32, box=32.0, n_steps=5, seed=4),
]


def _alone(p):
    st = C.State(p)
    C.cola_make_ic(p, st)
    for i in range(p.n_steps):
        C.cola_step(p, st, i)
    torch.cuda.synchronize()
    return st.disp_f.clone(), st.vel_f.clone()


def test_results_identical_alone_and_in_the_mix():
    params = [C.Params(**kw) for kw in REQS]
    reqs = [Request(p, arrival=0.002 * j, rid=j) for j, p in enumerate(params)]
    res = Server(GpuEngine(n_streams=2), hbm_budget=8 << 30, max_active=4,
                 keep_states=True).run(reqs)
    torch.cuda.synchronize()
    s = summarize(res)
    assert s["runs"] == 4 and s["p99_s"] > 0
    for p, r in zip(params, res):
        d0, v0 = _alone(p)
        assert r.state.next_step == p.n_steps
        assert torch.equal(r.state.disp_f, d0), p
        assert torch.equal(r.state.vel_f, v0), p
        assert torch.isfinite(d0).all()


def test_sixteen_requests_with_overlapping_arrivals():
    """Sixteen requests drawn like the serving workload (n_p in {128, 256, 384} with
    n_mesh = 2 n_p and L = 2 n_p Mpc/h, 10-30 steps, LCDM / f(R) / nDGP), arriving every
    50 ms while earlier ones run: at most six admitted at once on four streams, later
    ones admitted as slots free up.  Every result equals the same run alone, bit for bit."""
    import numpy as np
    rng = np.random.default_rng(77)
    params = []
    for j in range(16):
        n = int(rng.choice([128, 256, 384]))
        m = int(rng.integers(6))
        kw = dict(np1d=n, nmesh1d=2 * n, box=2.0 * n, z_init=19.0, n_steps=int(rng.integers(10, 31)),
                  seed=5000 + j, screening=1)
        if m == 0:
            kw.update(model=C.LCDM)
        elif m <= 3:
            kw.update(model=C.FR_HS1, fr0_abs=(1e-6, 1e-5, 1e-4)[m - 1])
        else:
            kw.update(model=C.NDGP, rc_h0=(0.5, 1.0)[m - 4])
        params.append(C.Params(**kw))
    reqs = [Request(p, arrival=0.05 * j, rid=j) for j, p in enumerate(params)]
    eng = GpuEngine(n_streams=4)
    res = Server(eng, hbm_budget=200 << 30, max_active=6, keep_states=True).run(reqs)
    torch.cuda.synchronize()
    admitted_late = sum(1 for r in res if r.admitted > r.arrival + 1e-3)
    overlapped = sum(1 for a in res for b in res if a is not b and a.admitted < b.finished
                     and b.admitted < a.finished)
    assert overlapped > 0   # runs shared the device
    for p, r in zip(params, res):
        d0, v0 = _alone(p)
        assert r.state.next_step == p.n_steps
        assert torch.equal(r.state.disp_f, d0), p
        assert torch.equal(r.state.vel_f, v0), p
        del d0, v0
    print(f"16 requests: {admitted_late} waited for a slot; {overlapped // 2} overlapping pairs")
