"""Pins of the oracle's k-Mouflage gradient screening (App. B) with the kinetic function
P(X) = -1 + X + K0 X^m: the X* equation P_X(X*)^2 X* = R against the closed-form roots of
the cubic it becomes for m = 2, its unscreened and deep-screening limits, the screened
source of a plane wave against the closed-form gradient of its potential, and the
unscreened force (1 + 2 beta^2) F_Newton (C = 2 beta^2, massless field)."""

import numpy as np
import pytest

from oracle.background import kappa
from oracle.models import Model, eps_kmouflage, km_mu, km_px, km_xstar
from oracle.params import H0_OVER_C, MODEL_KMOUFLAGE, Params
from oracle.pm import force_mesh, screened_source


def test_xstar_is_the_cubic_root_for_m2():
    k0 = 0.7
    R = np.array([1e-9, 1e-3, 0.5, 3.0, 1e4, 1e9])
    X = km_xstar(R, k0, 2)
    for r, x in zip(R, X):
        # (1 + 2 K0 X)^2 X = R  <=>  4 K0^2 X^3 + 4 K0 X^2 + X - R = 0
        roots = np.roots([4 * k0 * k0, 4 * k0, 1.0, -r])
        real = roots[np.abs(roots.imag) < 1e-9 * max(1.0, abs(roots).max())].real
        assert x == pytest.approx(real[real > 0].max(), rel=1e-12)
    assert km_xstar(np.array([0.0]), k0, 2)[0] == 0.0


def test_screening_limits():
    k0, m = 2.0, 3
    # unscreened: P_X(0) = 1
    assert eps_kmouflage(np.array([0.0, 1e-12]), k0, m, 1.0) == pytest.approx([1.0, 1.0], abs=1e-11)
    # deep: X* -> (R/(m K0)^2)^(1/(2m-1)), eps -> 1/(m K0 X*^(m-1))
    g = np.array([1e8])
    R = g[0] ** 2
    Xa = (R / (m * k0) ** 2) ** (1.0 / (2 * m - 1))
    assert km_xstar(np.array([R]), k0, m)[0] == pytest.approx(Xa, rel=1e-3)
    assert eps_kmouflage(g, k0, m, 1.0)[0] == pytest.approx(1.0 / (m * k0 * Xa ** (m - 1)), rel=2e-3)
    # linear growth: mu = 1 + 2 beta^2 / P_X(X(a))
    p = Params(model=MODEL_KMOUFLAGE, km_beta=0.6, km_k0=k0, km_m=m, km_x0=0.3, km_xn=-1.5)
    assert km_mu(0.5, p) == pytest.approx(1 + 0.72 / (1 + m * k0 * (0.3 * 0.5 ** -1.5) ** 2), rel=1e-14)


def _wave(n, L, A):
    x = np.arange(n) * L / n
    X = np.meshgrid(x, x, x, indexing="ij")
    k = 2 * np.pi * 3 / L
    return A * np.cos(k * X[0]), k, X


def test_plane_wave_screened_source_and_unscreened_force():
    n, L, a = 16, 64.0, 0.8
    p = Params(model=MODEL_KMOUFLAGE, nmesh1d=n, box=L, km_beta=0.5, km_k0=1.5, km_m=3,
               km_lambda=3e6)
    d, k, X = _wave(n, L, 20.0)
    # Phi = -kappa A cos(kx)/k^2 -> |grad Phi| = kappa A |sin(kx)| / k (code units)
    grad = kappa(a, p.omega_m) * 20.0 * np.abs(np.sin(k * X[0])) / k * H0_OVER_C ** 2 / a ** 2
    eps = eps_kmouflage(grad, p.km_k0, p.km_m, p.km_lambda)
    assert eps.min() < 0.5   # really screened somewhere
    S = screened_source(d, np.fft.rfftn(d), p, a, Model(p))
    assert np.allclose(S, d * eps, rtol=1e-10, atol=1e-12 * 20.0)
    # tiny lambda: unscreened, F = (1 + 2 beta^2) F_Newton
    q = p.with_(km_lambda=1e-6)
    F, _ = force_mesh(d, q, a, Model(q))
    Fn = -kappa(a, p.omega_m) * 20.0 * np.sin(k * X[0]) / k   # -dPhi/dx
    assert np.allclose(F[0], (1 + 2 * 0.25) * Fn, rtol=1e-10, atol=1e-10 * np.abs(Fn).max())
    assert np.abs(F[1]).max() < 1e-12 * np.abs(Fn).max()
