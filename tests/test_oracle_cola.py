"""Pins of the oracle's COLA integration (Sec. 2, App. A): the LCDM limit of the
scale-dependent path, special cases, linear growth of tiny modes against the
growth ODE, and the time grid."""

import numpy as np
import pytest

from oracle import Params, MODEL_LCDM, MODEL_FR, MODEL_NDGP
from oracle.background import tau_between
from oracle.cola import Run, time_grid
from oracle.growth import solve_growth
from oracle.lpt import phi1_from_delta_k, displacement
from oracle.models import Model


def test_time_grid_telescopes():
    p = Params(omega_m=1.0, n_steps=7, z_init=19.0)
    a, kick, drift = time_grid(p)
    assert a[0] == pytest.approx(0.05) and a[-1] == pytest.approx(1.0)
    tau = lambda x: 2 * (a[0] ** -0.5 - x ** -0.5)   # noqa: E731  (EdS closed form)
    assert drift.sum() == pytest.approx(tau(1.0), rel=1e-12)
    assert kick.sum() == pytest.approx(tau(0.5 * (a[-2] + a[-1])), rel=1e-12)
    assert kick[0] == pytest.approx(tau(0.5 * (a[0] + a[1])), rel=1e-12)


def test_lcdm_limit_kspace_lpt_equals_standard_cola():
    # Sec. 7: the scale-dependent solver run for LCDM reproduces standard COLA.
    # Growth factors that do not depend on k, applied per mode in Fourier space,
    # equal the per-particle Psi1, Psi2 scaled by D(a).
    for model in (MODEL_LCDM, MODEL_NDGP):
        p = Params(model=model, np1d=16, nmesh1d=32, box=100.0, n_steps=4)
        std = Run(p).run()
        ksp = Run(p, kspace_lpt=True).run()
        assert ksp.kdep and not std.kdep
        scale = np.abs(std.u).max()
        assert np.allclose(ksp.u, std.u, rtol=0, atol=1e-10 * scale)
        assert np.allclose(ksp.v, std.v, rtol=0, atol=1e-10 * np.abs(std.v).max())


def test_initial_displacement_is_2lpt():
    p = Params(model=MODEL_FR, np1d=16, nmesh1d=32, box=100.0, n_steps=2)
    r = Run(p)
    want = r.psi1 - 3.0 / 7.0 * r.psi2
    assert np.allclose(r.u, want, rtol=0, atol=1e-12 * np.abs(want).max())
    assert np.all(r.v == 0)


def test_zero_amplitude_stays_on_lattice():
    p = Params(model=MODEL_NDGP, np1d=8, nmesh1d=16, box=50.0, n_steps=3)
    z = np.zeros((3, 8, 8, 8))
    zk = np.zeros((8, 8, 5), complex)
    r = Run(p, lpt=dict(phi1_k=zk, phi2_k=zk, psi1=z, psi2=z)).run()
    assert np.all(r.u == 0) and np.all(r.v == 0)


def _tiny_mode_run(p, nu, amp=1e-6):
    n, L = p.np1d, p.box
    x = np.arange(n) * L / n
    X, _, _ = np.meshgrid(x, x, x, indexing="ij")
    k = 2 * np.pi * nu / L
    phi1 = phi1_from_delta_k(np.fft.rfftn(amp * np.cos(k * X)), n, L)
    lpt = dict(phi1_k=phi1, phi2_k=np.zeros_like(phi1), psi1=displacement(phi1, n, L),
               psi2=np.zeros((3, n, n, n)))
    r = Run(p, lpt=lpt).run()
    psi = lpt["psi1"].reshape(3, -1)
    grown = (r.u[0] @ psi[0]) / (psi[0] @ psi[0])
    m = Model(p)
    D1 = solve_growth(np.array([k]), np.array([1.0]), p.omega_m, m.mu, m.gamma2_orth,
                      p.a_ini)[0, 0, 0]
    return grown, D1


@pytest.mark.parametrize("box", [25.0, 200.0])
def test_tiny_mode_grows_with_scale_dependent_D1(box):
    # A tiny single mode follows 1LPT when residual forces vanish, so after the run its
    # amplitude is D1(k, a=1) up to the PM discreteness factor at nu = 1 (mesh = particle
    # grid), which is the same for every model.  The MG/LCDM ratio then isolates
    # mu(k, a): at k = 0.25 h/Mpc F5 grows 9 % more than LCDM, at k = 0.031 h/Mpc 0.5 %.
    base = Params(np1d=32, nmesh1d=32, box=box, n_steps=10, screening=0)
    g_l, D_l = _tiny_mode_run(base.with_(model=MODEL_LCDM), 1)
    assert g_l / D_l == pytest.approx(1.0, abs=0.015)
    for model in (MODEL_FR, MODEL_NDGP):
        g, D = _tiny_mode_run(base.with_(model=model), 1)
        assert g / D == pytest.approx(1.0, abs=0.015)
        assert (g / g_l) / (D / D_l) == pytest.approx(1.0, abs=1e-3)
    if box == 25.0:
        _, D_f = _tiny_mode_run(base.with_(model=MODEL_FR), 1)
        assert D_f / D_l > 1.08


def test_planar_step_equals_3d_step():
    """Two steps of Run.step on a planar configuration (displacement, Psi1 and Psi2 along
    x, functions of the lattice index ix) equal planar_step on the 1D profiles."""
    from oracle.pm import lagrangian_index
    from oracle.planar import planar_step
    p = Params(model=MODEL_NDGP, rc_h0=1.0, np1d=16, nmesh1d=32, box=64.0, n_steps=6)
    q = np.arange(p.np1d) * p.box / p.np1d
    psi1 = 3.0 * np.sin(2 * np.pi * q / p.box) + 0.5 * np.sin(2 * np.pi * 3 * q / p.box)
    psi2 = -0.7 * np.sin(2 * np.pi * 2 * q / p.box)
    ix = lagrangian_index(p.np1d)[0]
    P1 = np.zeros((3, p.n_part))
    P2 = np.zeros((3, p.n_part))
    P1[0], P2[0] = psi1[ix], psi2[ix]
    r = Run(p, lpt=dict(psi1=P1, psi2=P2))
    u1 = r.G[0, 0, 0] * psi1 + r.G[0, 0, 3] * psi2
    v1 = np.zeros(p.np1d)
    for i in range(2):
        r.step()
        u1, v1 = planar_step(u1, v1, psi1, psi2, p, i)
        scale = np.abs(u1).max()
        assert np.abs(r.u[0] - u1[ix]).max() < 1e-11 * scale
        assert np.abs(r.v[0] - v1[ix]).max() < 1e-11 * np.abs(v1).max()
        assert np.abs(r.u[1:]).max() < 1e-11 * scale and np.abs(r.v[1:]).max() < 1e-11 * scale
