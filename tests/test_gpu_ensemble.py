"""Ensembles stepped as captured HIP graphs (cola_ensemble_*) against the same runs stepped
alone with cola_step: every member's final displacements and velocities must be bitwise
equal (the same kernels and per-step values; the deposit sums in integers).  The members
differ in model, size (radix-2 and radix-3 meshes) and step count, and one starts
mid-run, so the ensemble re-captures its graph as members finish."""

import numpy as np
import pytest

from paper_1703_00879_amd import cola as C

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MIX = [
    dict(model=C.LCDM, np1d=16, nmesh1d=32, box=32.0, n_steps=3, seed=21),
    dict(model=C.FR_HS1, fr0_abs=1e-5, np1d=24, nmesh1d=48, box=48.0, n_steps=5, seed=22),
    dict(model=C.NDGP, rc_h0=1.0, np1d=32, nmesh1d=64, box=64.0, n_steps=4, seed=23),
    dict(model=C.SYMMETRON, np1d=16, nmesh1d=32, box=32.0, n_steps=6, seed=24),
    dict(model=C.FR_HS1, fr0_abs=1e-6, growth_mode=1, np1d=16, nmesh1d=32, box=40.0, n_steps=5,
         seed=25),
]


def _final(st):
    torch.cuda.synchronize()
    return st.disp_f.cpu().numpy().copy(), st.vel_f.cpu().numpy().copy()


@pytest.mark.parametrize("n_streams", [1, 3])
def test_ensemble_graph_equals_runs_alone(n_streams):
    ps = [C.Params(**kw) for kw in MIX]
    alone = []
    for p in ps:
        st = C.State(p)
        C.cola_make_ic(p, st)
        for i in range(p.n_steps):
            C.cola_step(p, st, i)
        alone.append(_final(st))
    states = [C.State(p) for p in ps]
    for p, st in zip(ps, states):
        C.cola_make_ic(p, st)
    C.cola_step(ps[1], states[1], 0)   # a member that starts mid-run
    ens = C.Ensemble(ps, states)
    ens.run(n_streams=n_streams)
    ens.close()
    for j, (p, st) in enumerate(zip(ps, states)):
        assert st.next_step == p.n_steps
        u, v = _final(st)
        assert np.isfinite(u).all()
        assert np.array_equal(u, alone[j][0]), f"member {j} displacements"
        assert np.array_equal(v, alone[j][1]), f"member {j} velocities"


def test_ensemble_rejects_members_without_initial_conditions():
    p = C.Params(**MIX[0])
    st = C.State(p)
    C.cola_prepare(p, st)
    ens = C.Ensemble([p], [st])
    with pytest.raises(C.ColaError) as e:
        ens.run()
    assert e.value.status == -3
    ens.close()
