"""Pins of the oracle's power spectrum estimator and of the modified-gravity boost
on large scales (Sec. 7)."""

import numpy as np
import pytest

from oracle import Params, MODEL_LCDM, MODEL_FR, MODEL_NDGP
from oracle.cola import Run
from oracle.growth import solve_growth
from oracle.models import Model
from oracle.pk import power_spectrum, power_spectrum_mesh, shell_index
from oracle.pm import cic_deposit


def test_shell_index_exact():
    n2 = np.arange(0, 20000)
    want = np.array([int(np.floor(np.sqrt(m) + 0.5)) for m in n2])
    assert np.array_equal(shell_index(n2), want)


def test_shot_noise_of_uniform_random_particles():
    # Poisson particles: <|delta_k|^2> = (M^2/N) C1(k), C1 = prod_i (1 - 2/3 sin^2(pi nu_i/n))
    # for CIC (aliased window sum), so the estimator returns (L^3/N) C1/W^2 per mode.
    n, L, N = 32, 100.0, 200_000
    rng = np.random.default_rng(2)
    s = rng.uniform(0, n, size=(3, N))
    rho = cic_deposit(s, n, n ** 3 / N)
    k, P, nm = power_spectrum_mesh(rho - 1.0, L, n // 2)
    from oracle.lpt import kvec
    _, (nx, ny, nz) = kvec(n, L)
    C1 = ((1 - 2 / 3 * np.sin(np.pi * nx / n) ** 2) * (1 - 2 / 3 * np.sin(np.pi * ny / n) ** 2)
          * (1 - 2 / 3 * np.sin(np.pi * nz / n) ** 2))
    W = (np.sinc(nx / n) * np.sinc(ny / n) * np.sinc(nz / n)) ** 2
    expect_mode = np.broadcast_to(L ** 3 / N * C1 / W ** 2, (n, n, n // 2 + 1))
    wt = np.broadcast_to(np.where((nz > 0) & (nz < n // 2), 2.0, 1.0), expect_mode.shape)
    b = shell_index(np.broadcast_to(nx * nx + ny * ny + nz * nz, expect_mode.shape))
    sel = b < n // 2
    expect = (np.bincount(b[sel], weights=(wt * expect_mode)[sel], minlength=n // 2)
              / np.bincount(b[sel], weights=wt[sel], minlength=n // 2))
    # each bin averages ~nm/2 independent exponential variates
    for i in range(2, n // 2):
        assert P[i] / expect[i] == pytest.approx(1.0, abs=5.0 / np.sqrt(nm[i] / 2))


@pytest.mark.slow
def test_unscreened_boost_follows_linear_growth_on_large_scales():
    # Sec. 7: the boost P_MG / P_LCDM from the same initial conditions; on the largest
    # scales it must approach [D1_MG(k,1) / D1_LCDM(1)]^2 from the growth ODE.
    base = Params(np1d=32, nmesh1d=64, box=200.0, n_steps=10, screening=0)
    rl = Run(base.with_(model=MODEL_LCDM)).run()
    _, Pl, _ = power_spectrum(rl.u, base)
    Dl = solve_growth(np.array([0.0]), np.array([1.0]), 0.3, lambda k, a: np.ones_like(k),
                      lambda k, a: np.zeros_like(k), base.a_ini)[0, 0, 0]
    for model in (MODEL_FR, MODEL_NDGP):
        p = base.with_(model=model)
        r = Run(p).run()
        k, P, _ = power_spectrum(r.u, p)
        m = Model(p)
        D = solve_growth(k[1:4], np.array([1.0]), 0.3, m.mu, m.gamma2_orth, p.a_ini)[0, :, 0]
        assert np.allclose((P[1:4] / Pl[1:4]) / (D / Dl) ** 2, 1.0, atol=0.015)
        # with screening the enhancement is smaller (Sec. 7.1)
        rs = Run(p.with_(screening=1)).run()
        _, Ps, _ = power_spectrum(rs.u, p)
        assert np.all(Ps[1:6] / Pl[1:6] < P[1:6] / Pl[1:6])
        assert np.all(Ps[1:6] / Pl[1:6] > 0.99)
