"""Pins of the oracle's initial conditions: the white-noise generator, the initial
power spectrum, and the 1LPT/2LPT potentials (Secs. 3-4)."""

import os

import numpy as np
import pytest
from scipy import stats

from oracle import Params
from oracle.lpt import (kvec, phi1_from_delta_k, phi2_from_phi1, displacement,
                        grad_factor, nyquist_masks, delta_k_from_noise, n2_grid)
from oracle.rng import splitmix64, white_noise
from oracle.spectrum import InitialSpectrum, eh_nowiggle_T, tophat_W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_vectors():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "splitmix64_vectors.txt"))
            if l.strip() and not l.startswith("#")]
    for seed, k, out in rows:
        assert int(splitmix64(int(seed), np.array([int(k)], dtype=np.uint64))[0]) == int(out)


def test_white_noise_statistics():
    g = white_noise(7, 64).ravel()
    assert abs(g.mean()) < 5.0 / np.sqrt(g.size)
    assert g.var() == pytest.approx(1.0, abs=5 * np.sqrt(2.0 / g.size))
    assert stats.kstest(g, "norm").pvalue > 1e-3
    # neighbouring points are uncorrelated
    assert abs(np.corrcoef(g[:-1], g[1:])[0, 1]) < 5.0 / np.sqrt(g.size)
    assert not np.array_equal(white_noise(7, 8), white_noise(8, 8))


def test_transfer_function_limits():
    p = Params()
    T = lambda k: eh_nowiggle_T(k, p.omega_m, p.omega_b, p.h, p.t_cmb)   # noqa: E731
    assert T(1e-7) == pytest.approx(1.0, abs=1e-6)
    assert np.all(np.diff(T(np.logspace(-4, 2, 200))) < 0)
    # large-q asymptote ln(2e + 1.8 q) / (C0 q^2) with C0 -> 14.2 (EH98 eq. 29)
    k = 1e4
    s = 44.5 * np.log(9.83 / (p.omega_m * p.h ** 2)) / np.sqrt(1 + 10 * (p.omega_b * p.h ** 2) ** 0.75)
    fb = p.omega_b / p.omega_m
    omh2 = p.omega_m * p.h ** 2
    alpha = 1 - 0.328 * np.log(431 * omh2) * fb + 0.38 * np.log(22.3 * omh2) * fb ** 2
    q = k * (p.t_cmb / 2.7) ** 2 / (p.omega_m * p.h * alpha)
    assert T(k) * 14.2 * q * q / np.log(1.8 * q) == pytest.approx(1.0, rel=2e-2)
    assert s > 0


def test_sigma8_normalisation_independent_quadrature():
    p = Params()
    sp = InitialSpectrum(p)
    lnk = np.linspace(np.log(1e-5), np.log(1e2), 2_000_001)
    k = np.exp(lnk)
    f = k ** 3 * sp.P_today(k) * tophat_W(8.0 * k) ** 2 / (2 * np.pi ** 2)
    sig2 = np.sum((f[1:] + f[:-1]) * 0.5 * np.diff(lnk))
    assert np.sqrt(sig2) == pytest.approx(p.sigma8, rel=1e-6)
    # P_ini = P_today / D1(a=1)^2 with the LCDM growth normalised at a_ini
    assert sp.P_ini(0.1) * sp.D1_today ** 2 == pytest.approx(sp.P_today(0.1), rel=1e-14)


def test_initial_delta_power_matches_spectrum():
    # <|delta_k|^2> = N^2 P_ini / L^3 shell by shell (chi^2 with 2 dof per complex mode)
    p = Params(np1d=64, box=256.0)
    sp = InitialSpectrum(p)
    dk = delta_k_from_noise(white_noise(p.seed, 64), p, sp)
    (kx, ky, kz), _ = kvec(64, p.box)
    k = np.sqrt(kx * kx + ky * ky + kz * kz)
    N = 64 ** 3
    ratio = np.abs(dk) ** 2 / (N * N * np.where(k > 0, sp.P_ini(np.maximum(k, 1e-9)), 1) / p.box ** 3)
    nyq = nyquist_masks(64)
    inner = (k > 0) & ~(nyq[0] | nyq[1] | nyq[2]) & (np.broadcast_to(kz, k.shape) > 0)
    r = ratio[inner]
    assert r.mean() == pytest.approx(1.0, abs=5 / np.sqrt(r.size))
    assert dk[0, 0, 0] == 0


def _plane_wave_delta_k(n, L, waves):
    x = np.arange(n) * L / n
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    d = np.zeros((n, n, n))
    for amp, kvec_, fn in waves:
        d += amp * fn(kvec_[0] * X + kvec_[1] * Y + kvec_[2] * Z)
    return d, np.fft.rfftn(d), (X, Y, Z)


def test_1lpt_divergence_is_minus_delta():
    n, L = 32, 100.0
    rng = np.random.default_rng(1)
    d = rng.standard_normal((n, n, n))
    dk = np.fft.rfftn(d)
    psi = displacement(phi1_from_delta_k(dk, n, L), n, L)
    div_k = sum(np.fft.rfftn(psi[ax]) * grad_factor(n, L, ax) for ax in range(3))
    nyq = nyquist_masks(n)
    inner = ~(nyq[0] | nyq[1] | nyq[2]) & (n2_grid(n) > 0)
    inner = np.broadcast_to(inner, dk.shape)
    assert np.allclose(-div_k[inner], dk[inner], rtol=1e-12, atol=1e-10 * np.abs(dk).max())


def test_2lpt_single_plane_wave_has_no_second_order():
    n, L = 32, 100.0
    k1 = 2 * np.pi * 3 / L
    _, dk, _ = _plane_wave_delta_k(n, L, [(0.3, (k1, 0, 0), np.cos)])
    phi2 = phi2_from_phi1(phi1_from_delta_k(dk, n, L), n, L)
    assert np.abs(phi2).max() < 1e-14 * np.abs(dk).max()


def test_2lpt_two_orthogonal_waves_closed_form():
    # delta = A1 cos(k1 x) + A2 cos(k2 y): phi1 = A1 cos(k1 x)/k1^2 + A2 cos(k2 y)/k2^2,
    # S = phi11 phi22 = A1 A2 cos(k1 x) cos(k2 y),
    # Psi2 = A1 A2/(k1^2 + k2^2) (k1 sin(k1 x) cos(k2 y), k2 cos(k1 x) sin(k2 y), 0)
    n, L = 32, 100.0
    A1, A2 = 0.2, -0.35
    k1, k2 = 2 * np.pi * 2 / L, 2 * np.pi * 5 / L
    _, dk, (X, Y, Z) = _plane_wave_delta_k(n, L, [(A1, (k1, 0, 0), np.cos),
                                                 (A2, (0, k2, 0), np.cos)])
    phi1 = phi1_from_delta_k(dk, n, L)
    psi2 = displacement(phi2_from_phi1(phi1, n, L), n, L)
    c = A1 * A2 / (k1 * k1 + k2 * k2)
    want = np.stack([c * k1 * np.sin(k1 * X) * np.cos(k2 * Y),
                     c * k2 * np.cos(k1 * X) * np.sin(k2 * Y), np.zeros_like(X)])
    assert np.allclose(psi2, want, atol=1e-12 * np.abs(want).max())
    psi1 = displacement(phi1, n, L)
    want1 = np.stack([-A1 / k1 * np.sin(k1 * X), -A2 / k2 * np.sin(k2 * Y), np.zeros_like(X)])
    assert np.allclose(psi1, want1, atol=1e-12 * np.abs(want1).max())


def test_sparse_lpt_field_equals_the_transform():
    # direct summation over a few stored modes equals the FFT synthesis of the same
    # half-complex fields (App. A), Nyquist modes included
    from oracle.lpt import lpt_field_sparse, lpt_field_scale_dependent
    n, L = 16, 40.0
    rng = np.random.default_rng(5)
    modes = [((3, -5, 2), None), ((-8, 2, 5), None), ((7, -8, 7), None), ((0, 1, 1), None)]
    phi1 = np.zeros((n, n, n // 2 + 1), complex)
    phi2 = np.zeros_like(phi1)
    sparse = []
    X1 = rng.uniform(0.5, 2.0, 3 * (n // 2) ** 2 + 1)
    X2 = rng.uniform(-1.0, 0.0, X1.size)
    for nu, _ in modes:
        a, b = rng.standard_normal(2) + 1j * rng.standard_normal(2)
        phi1[nu[0] % n, nu[1] % n, nu[2]] = a
        phi2[nu[0] % n, nu[1] % n, nu[2]] = b
        n2 = nu[0] ** 2 + nu[1] ** 2 + nu[2] ** 2
        sparse.append((nu, X1[n2] * a + X2[n2] * b))
    ref = lpt_field_scale_dependent(phi1, phi2, X1, X2, n, L, lambda n2: n2)
    planes = np.arange(n)
    got = lpt_field_sparse(sparse, n, L, planes)
    assert np.max(np.abs(got - ref)) < 1e-13 * np.max(np.abs(ref))
    assert np.abs(ref).max() > 0
