"""Pins of the oracle's particle-mesh force (Secs. 2 and 6): CIC invariants,
closed-form plane-wave forces, brute-force DFT, screening limits, momentum
conservation and a direct (Ewald) sum on a tiny periodic box."""

import numpy as np
import pytest
from scipy.special import erfc

from oracle import Params, MODEL_LCDM, MODEL_FR, MODEL_NDGP
from oracle.background import kappa
from oracle.models import Model, fr_mu, fr_fR_abs, dgp_beta, eps_vainshtein, vainshtein_x, window
from oracle.params import H0_OVER_C
from oracle.pm import cic_deposit, cic_gather, force_mesh, pm_force, screened_source


# ----------------------------------------------------------------------------- CIC
def test_cic_mass_conservation_and_node_cases():
    n = 16
    rng = np.random.default_rng(0)
    s = rng.uniform(-20, 40, size=(3, 1000))
    rho = cic_deposit(s, n, 0.37)
    assert rho.sum() == pytest.approx(0.37 * 1000, rel=1e-13)
    # on a node: all mass in that cell
    rho = cic_deposit(np.array([[3.0], [5.0], [15.0]]), n, 2.0)
    assert rho[3, 5, 15] == 2.0 and rho.sum() == 2.0
    # half-way along x: split evenly
    rho = cic_deposit(np.array([[3.5], [5.0], [1.0]]), n, 1.0)
    assert rho[3, 5, 1] == 0.5 and rho[4, 5, 1] == 0.5
    # periodic wrap at both ends
    rho = cic_deposit(np.array([[n - 0.25], [-1.0], [2 * n]]), n, 1.0)
    assert rho[n - 1, n - 1, 0] == pytest.approx(0.25) and rho[0, n - 1, 0] == pytest.approx(0.75)


@pytest.mark.parametrize("nm", [16, 32])
def test_cic_lattice_is_uniform(nm):
    # Lagrangian points at cell centres: the undisplaced lattice is uniform for
    # n_m = n_p and n_m = 2 n_p
    p = Params(np1d=16, nmesh1d=nm, box=64.0)
    from oracle.pm import density_contrast
    d, _ = density_contrast(np.zeros((3, p.n_part)), p)
    assert np.abs(d).max() < 1e-14


def test_cic_gather_is_exact_for_linear_fields():
    n = 16
    j = np.arange(n, dtype=float)
    X, Y, Z = np.meshgrid(j, j, j, indexing="ij")
    f = 0.3 * X - 1.2 * Y + 2.0 * Z + 0.5
    rng = np.random.default_rng(1)
    s = rng.uniform(1, n - 2, size=(3, 500))
    g = cic_gather([f], s, n)[0]
    assert np.allclose(g, 0.3 * s[0] - 1.2 * s[1] + 2.0 * s[2] + 0.5, rtol=1e-13)


# ----------------------------------------------------------------------------- plane waves
def _wave(n, L, nu, amp):
    x = np.arange(n) * L / n
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    k = 2 * np.pi * np.asarray(nu) / L
    ph = k[0] * X + k[1] * Y + k[2] * Z
    return amp * np.cos(ph), np.sin(ph), k


@pytest.mark.parametrize("nu", [(1, 0, 0), (0, 3, 0), (2, -1, 5), (0, 0, 7)])
def test_plane_wave_newtonian_force(nu):
    # delta = A cos(k.x): Phi = -kappa A cos / k^2, F = -grad Phi = -kappa A k sin / k^2
    p = Params(model=MODEL_LCDM, nmesh1d=16, box=64.0)
    a = 0.5
    d, sn, k = _wave(16, p.box, nu, 0.1)
    F, _ = force_mesh(d, p, a)
    k2 = k @ k
    for ax in range(3):
        want = -kappa(a, p.omega_m) * 0.1 * k[ax] * sn / k2
        assert np.allclose(F[ax], want, atol=1e-12 * kappa(a, p.omega_m) * 0.1 / np.sqrt(k2))


@pytest.mark.parametrize("nu", [(1, 0, 0), (3, 4, 0), (6, 6, 6)])
def test_plane_wave_fifth_force_unscreened(nu):
    # unscreened f(R): F_total = mu(k, a) F_Newton; nDGP: (1 + 1/(3 beta)) F_Newton
    a = 0.7
    for model, factor in [
            (Params(model=MODEL_FR, screening=0, nmesh1d=16, box=64.0),
             lambda k: fr_mu(k, a, 0.3, 1e-5)),
            (Params(model=MODEL_NDGP, screening=0, nmesh1d=16, box=64.0, rc_h0=1.0),
             lambda k: 1 + 1 / (3 * dgp_beta(a, 0.3, 1.0)))]:
        d, sn, k = _wave(16, model.box, nu, 0.05)
        F, S = force_mesh(d, model, a)
        kk = np.sqrt(k @ k)
        fac = factor(kk)
        for ax in range(3):
            want = -kappa(a, 0.3) * 0.05 * k[ax] * sn / kk ** 2 * fac
            assert np.allclose(F[ax], want, atol=1e-12 * 0.05 * kappa(a, 0.3) / kk)
        assert np.array_equal(S, d)


def test_fr_screening_tiny_amplitude_is_unscreened():
    a = 0.6
    pu = Params(model=MODEL_FR, screening=0, nmesh1d=16, box=64.0)
    ps = pu.with_(screening=1)
    d, _, _ = _wave(16, 64.0, (1, 2, 0), 1e-6)
    Fu, _ = force_mesh(d, pu, a)
    Fs, S = force_mesh(d, ps, a)
    assert np.allclose(Fs, Fu, rtol=0, atol=1e-14 * np.abs(Fu).max())
    assert np.allclose(S, d, rtol=1e-14)


def test_fr_screening_deep_potential_closed_form():
    # Phi_code = -kappa A cos/k^2 exactly; Phi_N = Phi (H0/c)^2 / a^2;
    # S = delta * min(1, |3 f_R(a) / (2 Phi_N)|) point by point (Sec. 6.1)
    a = 0.8
    p = Params(model=MODEL_FR, screening=1, nmesh1d=16, box=64.0, fr0_abs=1e-6)
    A = 30.0
    d, _, k = _wave(16, p.box, (1, 0, 0), A)
    phi_n = -kappa(a, 0.3) * d / (k @ k) * H0_OVER_C ** 2 / a ** 2
    eps = np.minimum(1.0, np.abs(1.5 * fr_fR_abs(a, 0.3, 1e-6) / phi_n))
    assert eps.min() < 0.5  # really screened somewhere
    S = screened_source(d, np.fft.rfftn(d), p, a, Model(p))
    assert np.allclose(S, d * eps, rtol=1e-10, atol=1e-12 * A)


def test_ndgp_screening_plane_wave_closed_form():
    # delta_R = W(kR) A cos exactly for a plane wave; eps from x(delta_R) (Sec. 6.2)
    a = 0.9
    for filt in (0, 1, 2):
        p = Params(model=MODEL_NDGP, screening=1, nmesh1d=16, box=32.0, rc_h0=2.0,
                   r_smooth=1.5, filter=filt)
        d, _, k = _wave(16, p.box, (2, 1, 0), 3.0)
        kk = np.sqrt(k @ k)
        dR = window(kk * p.r_smooth, filt) * d
        beta = dgp_beta(a, 0.3, 2.0)
        eps = eps_vainshtein(vainshtein_x(dR, a, 0.3, 2.0, beta))
        S = screened_source(d, np.fft.rfftn(d), p, a, Model(p))
        assert np.allclose(S, d * eps, rtol=1e-12, atol=1e-13)


# ----------------------------------------------------------------------------- brute force
def _dft_matrix(n, sign):
    j = np.arange(n)
    return np.exp(sign * 2j * np.pi * np.outer(j, j) / n)


def _brute_force_force(delta, p, a):
    """Full complex DFT by explicit matrices (no FFT), same Green's functions,
    screening evaluated in real space from the brute-force potential."""
    n, L = delta.shape[0], p.box
    Fw, Bw = _dft_matrix(n, -1), _dft_matrix(n, +1)

    def fwd(x):
        return np.einsum("ai,bj,ck,ijk->abc", Fw, Fw, Fw, x.astype(complex))

    def inv(x):
        return np.einsum("ai,bj,ck,ijk->abc", Bw, Bw, Bw, x) / n ** 3

    nu = np.fft.fftfreq(n, 1.0 / n)
    K = np.meshgrid(*(2 * np.pi * nu / L,) * 3, indexing="ij")
    NU = np.meshgrid(nu, nu, nu, indexing="ij")
    k2 = K[0] ** 2 + K[1] ** 2 + K[2] ** 2
    inv_k2 = np.where(k2 > 0, 1 / np.where(k2 > 0, k2, 1), 0)
    kap = kappa(a, p.omega_m)
    m = Model(p)
    dk = fwd(delta)
    tot = -kap * dk * inv_k2
    if m.has_fifth_force:
        S = delta
        if p.screening and p.model == MODEL_FR:
            Phi = inv(-kap * dk * inv_k2).real * H0_OVER_C ** 2 / a ** 2
            from oracle.models import eps_chameleon
            S = delta * eps_chameleon(Phi, fr_fR_abs(a, p.omega_m, p.fr0_abs))
        elif p.screening and p.model == MODEL_NDGP:
            dR = inv(dk * window(np.sqrt(k2) * p.r_smooth, p.filter)).real
            b = dgp_beta(a, p.omega_m, p.rc_h0)
            S = delta * eps_vainshtein(vainshtein_x(dR, a, p.omega_m, p.rc_h0, b))
        Sk = fwd(S)
        den = k2 + m.a2m2(a)
        tot = tot + np.where(k2 > 0, -m.coupling(a) * kap / np.where(k2 > 0, den, 1), 0) * Sk
    out = []
    for ax in range(3):
        kk = np.where(NU[ax] == -n // 2, 0.0, K[ax])
        f = inv(-1j * kk * tot)
        assert np.abs(f.imag).max() < 1e-10 * max(np.abs(f.real).max(), 1e-300)
        out.append(f.real)
    return np.stack(out)


@pytest.mark.parametrize("model,screen", [(MODEL_LCDM, 0), (MODEL_FR, 0), (MODEL_FR, 1),
                                          (MODEL_NDGP, 0), (MODEL_NDGP, 1)])
def test_force_mesh_matches_brute_force_dft(model, screen):
    p = Params(model=model, screening=screen, nmesh1d=8, box=16.0, fr0_abs=3e-7, rc_h0=3.0,
               r_smooth=2.0)
    rng = np.random.default_rng(11)
    delta = rng.standard_normal((8, 8, 8)) * 3.0
    a = 0.9
    F, _ = force_mesh(delta, p, a)
    Fb = _brute_force_force(delta, p, a)
    assert np.allclose(F, Fb, rtol=0, atol=1e-12 * np.abs(Fb).max())


# ----------------------------------------------------------------------------- invariants
@pytest.mark.parametrize("model", [MODEL_LCDM, MODEL_FR, MODEL_NDGP])
def test_momentum_conservation_unscreened(model):
    p = Params(model=model, screening=0, np1d=8, nmesh1d=16, box=32.0)
    rng = np.random.default_rng(5)
    u = rng.normal(0, 2.0, size=(3, p.n_part))
    Fp, _ = pm_force(u, p, 0.5)
    assert np.abs(Fp.sum(axis=1)).max() < 1e-12 * np.abs(Fp).sum(axis=1).max()


def _ewald_force(r, L, alpha_L=2.0, nreal=3, nk=8):
    """Periodic force per unit (kappa m cell^3 / 4 pi) on a test point at r from a unit
    point mass at the origin in a box L with neutralising background (Ewald split)."""
    al = alpha_L / L
    F = np.zeros(3)
    rng_ = range(-nreal, nreal + 1)
    for i in rng_:
        for j in rng_:
            for k in rng_:
                rn = r + L * np.array([i, j, k])
                d = np.linalg.norm(rn)
                F -= (erfc(al * d) / d ** 2 + 2 * al / np.sqrt(np.pi) * np.exp(-al * al * d * d) / d) * rn / d
    rngk = range(-nk, nk + 1)
    for i in rngk:
        for j in rngk:
            for k in rngk:
                if i == j == k == 0:
                    continue
                kv = 2 * np.pi * np.array([i, j, k]) / L
                k2 = kv @ kv
                F -= 4 * np.pi / L ** 3 * kv / k2 * np.exp(-k2 / (4 * al * al)) * np.sin(kv @ r)
    return F


@pytest.mark.parametrize("r", [8.0, 12.0])
def test_pair_force_vs_ewald(r):
    # Poisson in code units: nabla^2 Phi = kappa delta, so a particle of mass m (in
    # mean-cell units) is a point source of strength kappa m cell^3.  The PM pair force
    # (source deposited alone, force gathered at the test point) averaged over random
    # placements and directions must reproduce the periodic Newtonian force within the
    # scatter that the mesh causes at 8-12 cells.
    n, L = 32, 32.0
    p = Params(model=MODEL_LCDM, np1d=2, nmesh1d=n, box=L)
    rng = np.random.default_rng(0)
    ratios, errs = [], []
    for _ in range(32):
        src = rng.uniform(0, n, 3)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        rho = cic_deposit(src[:, None], n, 1.0)
        F, _ = force_mesh(rho - rho.mean(), p, 1.0)
        got = cic_gather(F, (src + r * d)[:, None], n)[:, 0]
        want = kappa(1.0, p.omega_m) * p.cell ** 3 / (4 * np.pi) * _ewald_force(r * d * p.cell, L)
        ratios.append(got @ d / (want @ d))
        errs.append(np.linalg.norm(got - want) / np.linalg.norm(want))
    assert np.mean(ratios) == pytest.approx(1.0, abs=0.02)
    assert np.median(errs) < 0.03


# ----------------------------------------------------------------------------- planar reduction
from oracle.pm import lagrangian_index  # noqa: E402
from oracle.planar import planar_pm  # noqa: E402


def _planar_profile(n_p, box, seed):
    """Per-plane displacements: two sine modes plus seeded jitter (Mpc/h)."""
    q = np.arange(n_p) * box / n_p
    rng = np.random.default_rng(seed)
    return (2.5 * np.sin(2 * np.pi * 2 * q / box) + 0.8 * np.cos(2 * np.pi * 5 * q / box + 0.3)
            + 0.4 * rng.standard_normal(n_p))


PLANAR_CASES = {
    "lcdm_r2": dict(model=MODEL_LCDM, np1d=16, nmesh1d=32, box=64.0),
    "ndgp_gauss_r2": dict(model=MODEL_NDGP, rc_h0=1.0, np1d=16, nmesh1d=32, box=32.0),
    "ndgp_tophat_r2": dict(model=MODEL_NDGP, rc_h0=2.0, filter=1, r_smooth=2.0, np1d=16,
                           nmesh1d=32, box=40.0),
    "fr_screened_r1": dict(model=MODEL_FR, fr0_abs=1e-7, np1d=24, nmesh1d=24, box=60.0),
    "fr_unscreened_r2": dict(model=MODEL_FR, fr0_abs=1e-5, screening=0, np1d=12, nmesh1d=24,
                             box=48.0),
    "symmetron_r2": dict(model=3, sym_beta=1.0, sym_mass=2997.92458, sym_astar=0.5, np1d=16,
                         nmesh1d=32, box=32.0),
}


@pytest.mark.parametrize("name", list(PLANAR_CASES))
def test_planar_reduction_equals_3d_oracle(name):
    """Particles displaced along one axis by a function of their lattice index along it:
    the 3D oracle's density, screened source and force meshes and per-particle forces
    equal the 1D planar computation broadcast over the other two axes, with zero force
    across the axis -- for each of the three axes."""
    p = Params(**PLANAR_CASES[name])
    n, N = p.nmesh1d, p.n_part
    u1 = _planar_profile(p.np1d, p.box, seed=sorted(PLANAR_CASES).index(name))
    idx = lagrangian_index(p.np1d)
    a = 0.8
    pl = planar_pm(u1, p, a)
    scale = np.abs(pl["force"]).max()
    assert scale > 0
    for ax in range(3):
        u = np.zeros((3, N))
        u[ax] = u1[idx[ax]]
        Fp, m = pm_force(u, p, a)
        shape = [n if i == ax else 1 for i in range(3)]
        b = lambda prof: np.broadcast_to(prof.reshape(shape), (n, n, n))  # noqa: E731
        assert np.abs(m["rho"] - b(pl["rho"])).max() < 1e-12
        assert np.abs(m["src"] - b(pl["src"])).max() < 1e-12
        assert np.abs(m["force"][ax] - b(pl["force"])).max() < 1e-11 * scale
        assert np.abs(Fp[ax] - pl["fp"][idx[ax]]).max() < 1e-11 * scale
        for o in range(3):
            if o != ax:
                assert np.abs(m["force"][o]).max() < 1e-11 * scale
                assert np.abs(Fp[o]).max() < 1e-11 * scale
