"""Pins of the oracle's background, model functions and growth factors against closed
forms, limits and cross-checks between independent passages of the paper."""

import numpy as np
import pytest
from scipy import integrate

from oracle import Params, MODEL_FR, MODEL_NDGP
from oracle.background import E, tau_between, omega_m_of_a
from oracle.growth import solve_growth
from oracle.models import (Model, fr_a2m2, fr_fR_abs, fr_gamma2E, fr_mu, fr_X, fr_Y,
                           dgp_beta, dgp_gamma2E_orth, eps_vainshtein, eps_chameleon)
from oracle.params import H0_OVER_C

ONE = lambda k, a: np.ones_like(k)      # noqa: E731
ZERO = lambda k, a: np.zeros_like(k)    # noqa: E731


def test_tau_eds_closed_form():
    # EdS: d tau = da / a^(3/2)  ->  tau = 2 (a0^-1/2 - a^-1/2)
    for a0, a1 in [(0.05, 1.0), (0.1, 0.37), (0.5, 0.9)]:
        assert tau_between(a0, a1, 1.0) == pytest.approx(2 * (a0 ** -0.5 - a1 ** -0.5),
                                                         rel=1e-12)


def test_growth_eds_lcdm_closed_form():
    # EdS, mu = 1: D1 = a/a_ini, D2 = -(3/7) D1^2 exactly (Sec. 3.2)
    ai = 0.05
    a = np.array([0.05, 0.1, 0.3, 0.77, 1.0])
    G = solve_growth(np.array([0.0]), a, 1.0, ONE, ZERO, ai)[:, 0, :]
    D1 = a / ai
    assert np.allclose(G[:, 0], D1, rtol=1e-10, atol=0)
    assert np.allclose(G[:, 3], -3.0 / 7.0 * D1 ** 2, rtol=1e-10, atol=0)
    # tau-derivatives: dD1/dtau = a^{3/2}/a_ini, D1'' = (3/2) a^2/a_ini
    assert np.allclose(G[:, 1], a ** 1.5 / ai, rtol=1e-10)
    assert np.allclose(G[:, 2], 1.5 * a ** 2 / ai, rtol=1e-12)


def _eds_const_mu(mu, a, ai):
    """Closed form for EdS with constant mu: D1 = sum c_s (a/ai)^p_s,
    p(p + 1/2) = (3/2) mu; D2 from the particular solutions of the D1^2 source plus
    the homogeneous solution fixed by D2 = -3/7, dD2/dtau = -(6/7) a_i^{1/2}."""
    disc = np.sqrt(1 + 24 * mu)
    p = np.array([(-1 + disc) / 4, (-1 - disc) / 4])
    # D1(ai) = 1, dD1/dtau(ai) = ai^{1/2}  with d(a^p)/dtau = p a^(p+1/2)
    cp = (1 - p[1]) / (p[0] - p[1])
    c = np.array([cp, 1 - cp])
    x = a / ai
    D1 = c[0] * x ** p[0] + c[1] * x ** p[1]
    # particular solution of D'' - (3/2) mu a D = -(3/2) mu a D1^2:
    # for a source term s x^q (x = a/ai): A x^q with A [q(q+1/2) - 3mu/2] = -(3/2) mu s
    part = np.zeros_like(x)
    dpart0 = 0.0
    part0 = 0.0
    for i in range(2):
        for j in range(2):
            q = p[i] + p[j]
            s = c[i] * c[j]
            A = -1.5 * mu * s / (q * (q + 0.5) - 1.5 * mu)
            part += A * x ** q
            part0 += A
            dpart0 += A * q
    # homogeneous b_s x^p_s with  part0 + sum b = -3/7,  dpart0 + sum b p = -6/7
    M = np.array([[1, 1], [p[0], p[1]]])
    b = np.linalg.solve(M, [-3 / 7 - part0, -6 / 7 - dpart0])
    D2 = part + b[0] * x ** p[0] + b[1] * x ** p[1]
    return D1, D2


@pytest.mark.parametrize("mu", [4.0 / 3.0, 1.1, 0.9])
def test_growth_eds_constant_mu_closed_form(mu):
    ai = 0.05
    a = np.array([0.08, 0.2, 0.5, 1.0])
    G = solve_growth(np.array([0.0]), a, 1.0, lambda k, aa: np.full_like(k, mu), ZERO, ai)
    D1, D2 = _eds_const_mu(mu, a, ai)
    assert np.allclose(G[:, 0, 0], D1, rtol=1e-10)
    assert np.allclose(G[:, 0, 3], D2, rtol=1e-10)


def test_growth_lcdm_growing_plus_decaying_mode():
    # LCDM: the two solutions of D'' = kappa D are the growing mode
    # D+ = E(a) int_0^a da'/(a' E)^3 (Heath 1977) and the decaying mode D- = E(a).
    om, ai = 0.3, 0.05
    a = np.array([0.05, 0.2, 0.6, 1.0])

    def Dp(x):
        v, _ = integrate.quad(lambda t: 1.0 / (t * E(t, om)) ** 3, 0.0, x, epsabs=0,
                              epsrel=1e-13, limit=200)
        return E(x, om) * v

    def dDp_dtau(x):      # d/dtau = a^3 E d/da
        h = 1e-5 * x
        return x ** 3 * E(x, om) * (Dp(x + h) - Dp(x - h)) / (2 * h)

    def dDm_dtau(x):      # dE/da = -1.5 om a^-4 / E
        return x ** 3 * E(x, om) * (-1.5 * om * x ** -4 / E(x, om))

    # fit alpha D+ + beta D- to D1 = 1, D1' = a_i^2 E(a_i)
    Mx = np.array([[Dp(ai), E(ai, om)], [dDp_dtau(ai), dDm_dtau(ai)]])
    al, be = np.linalg.solve(Mx, [1.0, ai ** 2 * E(ai, om)])
    want = np.array([al * Dp(x) + be * E(x, om) for x in a])
    G = solve_growth(np.array([0.0]), a, om, ONE, ZERO, ai)
    assert np.allclose(G[:, 0, 0], want, rtol=1e-8)


def test_growth_lcdm_second_order_omega_scaling():
    # Bouchet et al. (1995): D2 ~= -(3/7) Omega_m^{-1/143} D1^2 for LCDM
    om, ai = 0.3, 0.05
    G = solve_growth(np.array([0.0]), np.array([1.0]), om, ONE, ZERO, ai)[0, 0]
    assert G[3] / (-3.0 / 7.0 * G[0] ** 2) == pytest.approx(om ** (-1.0 / 143.0), abs=5e-4)


def test_fr_growth_limits():
    # k -> 0: LCDM growth; k -> infinity: constant mu = 4/3 (Sec. 5.1).  EdS background
    # (Omega_m = 1) so that the large-k limit has a closed form.
    p = Params(model=MODEL_FR, omega_m=1.0, fr0_abs=1e-5)
    m = Model(p)
    ai = 0.05
    a = np.array([0.3, 1.0])
    G = solve_growth(np.array([1e-7, 1e9]), a, 1.0, m.mu, m.gamma2_orth, ai)
    assert np.allclose(G[:, 0, 0], a / ai, rtol=1e-9)
    assert np.allclose(G[:, 0, 3], -3 / 7 * (a / ai) ** 2, rtol=1e-9)
    D1, D2 = _eds_const_mu(4.0 / 3.0, a, ai)
    assert np.allclose(G[:, 1, 0], D1, rtol=1e-8)
    assert np.allclose(G[:, 1, 3], D2, rtol=1e-8)


def _solve_exact_D2(k, k1, k2, cos, om, mu_fn, g2E_fn, ai, a_out):
    """Exact second-order kernel D2(k, k1, k2, a) of eq. (fofrexact) for one triangle,
    with D1(k1), D1(k2) integrated alongside (test helper, k-independent mu only)."""
    c2 = cos * cos

    def rhs(a, y):
        D1a, dD1a, D1b, dD1b, D2, dD2 = y
        kap = 1.5 * om * a
        mk, m1 = mu_fn(k, a), mu_fn(k1, a)
        g2 = g2E_fn(a) * (1 - c2)
        src = -kap * mk * D1a * D1b * (1 - (2 * m1 - mk) / mk * c2
                                       + 2 * a ** 4 * E(a, om) ** 2 / (kap * mk) * g2)
        f = 1.0 / (a ** 3 * E(a, om))
        return [dD1a * f, kap * m1 * D1a * f, dD1b * f, kap * mu_fn(k2, a) * D1b * f,
                dD2 * f, (kap * mk * D2 + src) * f]

    g0 = ai ** 2 * E(ai, om)
    y0 = [1, g0, 1, g0, -3 / 7 * (1 - c2), -6 / 7 * (1 - c2) * g0]
    s = integrate.solve_ivp(rhs, (ai, a_out), y0, method="DOP853", rtol=1e-12, atol=1e-14)
    return s.y[4, -1]


@pytest.mark.parametrize("model", ["lcdm", "ndgp"])
def test_approximate_D2_exact_for_scale_independent_models(model):
    # Sec. 4.2: the approximation is exact for gamma_2 = 0, and for
    # gamma_2 = f(a)(1 - cos^2) with mu = mu(a) (nDGP): D2_exact = (1 - cos^2) D2_hat.
    om, ai = 0.3, 0.05
    if model == "lcdm":
        mu_fn = lambda k, a: 1.0            # noqa: E731
        g2E = lambda a: 0.0                 # noqa: E731
        m = Model(Params())
    else:
        p = Params(model=MODEL_NDGP, rc_h0=0.5)
        m = Model(p)
        mu_fn = lambda k, a: float(m.mu(np.array([k]), a)[0])    # noqa: E731
        g2E = lambda a: dgp_gamma2E_orth(a, om, 0.5)              # noqa: E731
    Dhat = solve_growth(np.array([0.0]), np.array([1.0]), om, m.mu, m.gamma2_orth, ai)[0, 0, 3]
    rng = np.random.default_rng(3)
    for _ in range(3):
        k1, k2 = rng.uniform(0.05, 2.0, 2)
        cos = rng.uniform(-0.95, 0.95)
        k = np.sqrt(k1 * k1 + k2 * k2 + 2 * k1 * k2 * cos)
        D2 = _solve_exact_D2(k, k1, k2, cos, om, mu_fn, g2E, ai, 1.0)
        assert D2 == pytest.approx((1 - cos * cos) * Dhat, rel=1e-9)


def test_fr_phi_crit_integral_equals_fR():
    # App. C: Phi_crit(a) = (9 Om / (2 beta)) int_0^a beta / ((m^2/H0^2) a'^4) da' with
    # beta = 1/sqrt(6) and the HS m^2(a) reduces to (3/2)|f_R(a)| of Sec. 5.1.
    om, fr0 = 0.3, 1e-5
    for a in (0.2, 0.5, 1.0):
        def integrand(x):
            m2_over_H02 = fr_a2m2(x, om, fr0) / (x * x * H0_OVER_C ** 2)
            return 1.0 / (m2_over_H02 * x ** 4)
        I, _ = integrate.quad(integrand, 0.0, a, epsabs=0, epsrel=1e-13, limit=200)
        assert 4.5 * om * I == pytest.approx(1.5 * fr_fR_abs(a, om, fr0), rel=1e-10)


def test_fr_gamma2_matches_general_m_beta_form():
    # App. C gives gamma_2^E = m^2 (dm^2/da) beta^2 Om / (2 H0^4 Pi Pi Pi) k^2/(a^4 H^2),
    # Pi = (k/(a H0))^2 + m^2/H0^2; with HS beta = 1/sqrt(6) and m^2(a) it must equal
    # the f(R) gamma_2^E of Sec. 5.1.
    om, fr0 = 0.3, 1e-5
    for a in (0.3, 1.0):
        def m2(x):   # m^2/H0^2
            return fr_a2m2(x, om, fr0) / (x * x * H0_OVER_C ** 2)
        h = 1e-6 * a
        dm2 = (m2(a + h) - m2(a - h)) / (2 * h)
        for k, k1, k2 in [(0.1, 0.2, 0.15), (1.0, 0.7071, 0.7071), (3.0, 1.0, 2.5)]:
            Pi = lambda q: (q / (a * H0_OVER_C)) ** 2 + m2(a)     # noqa: E731
            H = E(a, om) * H0_OVER_C
            gen = m2(a) * dm2 * (1 / 6) * om / (2 * Pi(k) * Pi(k1) * Pi(k2)) * k * k / (a ** 4 * H * H)
            assert fr_gamma2E(k, k1, k2, a, om, fr0) == pytest.approx(gen, rel=1e-7)


def test_fr_mu_limits_and_compton_scale():
    om, fr0 = 0.3, 1e-5
    assert fr_mu(1e-9, 1.0, om, fr0) == pytest.approx(1.0, abs=1e-12)
    assert fr_mu(1e9, 1.0, om, fr0) == pytest.approx(4.0 / 3.0, rel=1e-12)
    # mu = 1 + 1/6 exactly where k = a m
    am = np.sqrt(fr_a2m2(1.0, om, fr0))
    assert fr_mu(am, 1.0, om, fr0) == pytest.approx(1 + 1 / 6, rel=1e-14)
    assert fr_X(1.0, om) == pytest.approx(fr_Y(om))


def test_dgp_beta_hdot_reading():
    # beta = 1 + 2 r_c H (1 + Hdot/(3 H^2)), Hdot = dH/dt = a H dH/da (cosmic time),
    # evaluated by finite differences of the background, independently of the
    # closed form used in the model.
    om, rc = 0.3, 1.0
    for a in (0.1, 0.5, 1.0):
        h = 1e-6 * a
        dHda = (E(a + h, om) - E(a - h, om)) / (2 * h)
        Hdot = a * E(a, om) * dHda
        want = 1 + 2 * rc * E(a, om) * (1 + Hdot / (3 * E(a, om) ** 2))
        assert dgp_beta(a, om, rc) == pytest.approx(want, rel=1e-9)
    assert omega_m_of_a(1.0, om) == pytest.approx(om)


def test_screening_factor_limits():
    # Vainshtein: eps -> 1 for x -> 0, eps sqrt(x) -> 2 for x -> infinity (Sec. 6.2)
    assert eps_vainshtein(1e-12) == pytest.approx(1.0, abs=1e-12)
    assert eps_vainshtein(1e12) * 1e6 == pytest.approx(2.0, rel=1e-5)
    # the printed closed form 2(sqrt(1+x)-1)/x agrees away from x = 0
    x = np.array([0.1, 1.0, 30.0])
    assert np.allclose(eps_vainshtein(x), 2 * (np.sqrt(1 + x) - 1) / x, rtol=1e-14)
    # chameleon: unscreened for shallow potentials, |3 fR/(2 Phi)| for deep ones
    fR = 1e-5
    assert np.all(eps_chameleon(np.array([1e-9, -1e-8, 0.0]), fR) == 1.0)
    deep = np.array([-1e-4, 3e-4])
    assert np.allclose(eps_chameleon(deep, fR), np.abs(1.5 * fR / deep), rtol=1e-15)


# ----------------------------------------------------------------------------- triangles
from oracle import MODEL_LCDM, MODEL_NDGP  # noqa: E402
from oracle.triangle import (approx_d2_triangle, cos_theta, fig1_triangles,  # noqa: E402
                             solve_d2_triangle)


def _random_triangles(n, seed):
    rng = np.random.default_rng(seed)
    k1 = rng.uniform(0.01, 3.0, n)
    k2 = rng.uniform(0.01, 3.0, n)
    c = rng.uniform(-0.99, 0.99, n)
    return np.sqrt(k1 * k1 + k2 * k2 + 2 * k1 * k2 * c), k1, k2


@pytest.mark.parametrize("model", [MODEL_LCDM, MODEL_NDGP])
def test_triangle_growth_exact_where_the_approximation_is(model):
    """LCDM and nDGP: mu does not depend on k and gamma_2 is proportional to
    (1 - cos^2 theta), so the exact triangle D2 equals D2_hat (1 - cos^2 theta) (Sec. 4.2)."""
    p = Params(model=model, rc_h0=0.5)
    k, k1, k2 = _random_triangles(40, seed=model)
    a = [p.a_ini, 0.3, 1.0]
    ex = solve_d2_triangle(k, k1, k2, a, p)
    ap = approx_d2_triangle(k, k1, k2, a, p)
    assert np.max(np.abs(ex / ap - 1.0)) < 1e-9
    c = cos_theta(k, k1, k2)
    assert np.allclose(ex[0], -3.0 / 7.0 * (1.0 - c * c), rtol=1e-14, atol=0)


@pytest.mark.parametrize("fr0", [1e-5, 1e-6])
def test_fig1_ratios_of_exact_to_approximate_d2(fr0):
    """Fig. 1 and its discussion (Sec. 4.2): for F5 and F6 at a = 1 the approximation
    agrees with the exact D2 to a few per cent up to k = 5 h/Mpc for equilateral and
    orthogonal triangles; for squeezed triangles it departs by up to ~10 % at
    k >~ 1 h/Mpc; all configurations agree on large scales."""
    p = Params(model=MODEL_FR, fr0_abs=fr0)
    ks = np.geomspace(0.01, 5.0, 25)
    r = {}
    for cfg in ("equilateral", "orthogonal", "squeezed"):
        k, k1, k2 = fig1_triangles(ks, cfg)
        r[cfg] = solve_d2_triangle(k, k1, k2, [1.0], p)[0] / approx_d2_triangle(k, k1, k2, [1.0], p)[0]
    for cfg in r:
        assert np.all(np.abs(r[cfg][ks <= 0.05] - 1.0) < 5e-3), cfg
    assert np.max(np.abs(r["equilateral"] - 1.0)) < 0.02
    assert np.max(np.abs(r["orthogonal"] - 1.0)) < 0.03
    sq = np.abs(r["squeezed"][ks >= 1.0] - 1.0)
    assert 0.03 < sq.max() < 0.13
    # the squeezed departure grows with k: the long mode k2 has LCDM-like growth
    assert np.all(np.diff(r["squeezed"][ks >= 0.5]) < 0)


# ----------------------------------------------------------------------------- symmetron
from oracle import MODEL_SYMMETRON  # noqa: E402
from oracle.models import (eps_potential, sym_a2m2, sym_beta2, sym_dm2_da, sym_gamma2E,  # noqa: E402
                           sym_m2, sym_mu, sym_phi_crit)

SYM = Params(model=MODEL_SYMMETRON, sym_beta=1.0, sym_mass=2997.92458, sym_astar=0.5)


def test_symmetron_phi_crit_is_the_app_c_integral():
    """Phi_crit(a) = (9 Om/(2 beta(a))) int_{a_*}^a beta/((m^2/H0^2) a'^4) da' (App. C),
    evaluated by quadrature with the (a' - a_*)^(-1/2) endpoint singularity as a weight."""
    p, ast = SYM, SYM.sym_astar
    for a in (0.55, 0.8, 1.0):
        def f(x):   # beta/(m^2 a^4) with (x - a_*)^(-1/2) taken out
            return (p.sym_beta * x ** 1.5
                    / (p.sym_mass ** 2 * x ** 4 * np.sqrt(x * x + x * ast + ast * ast)))
        I, _ = integrate.quad(f, ast, a, weight="alg", wvar=(-0.5, 0.0), epsabs=0, epsrel=1e-13)
        phi = 4.5 * p.omega_m / np.sqrt(sym_beta2(a, p)) * I
        assert phi == pytest.approx(sym_phi_crit(p), rel=1e-11)


def test_symmetron_mu_limits_and_switch_on():
    p = SYM
    for a in (0.2, 0.5):            # beta = m = 0 up to a_*
        assert sym_mu(np.array([0.01, 1.0, 100.0]), a, p) == pytest.approx(1.0, abs=0)
        assert sym_gamma2E(np.array([1.0]), 0.7, 0.7, a, p)[0] == 0.0
        assert Model(p).coupling(a) == 0.0
    a = 0.8
    s = 1 - (0.5 / a) ** 3
    assert sym_mu(1e-9, a, p) == pytest.approx(1.0, abs=1e-12)
    assert sym_mu(1e9, a, p) == pytest.approx(1 + 2 * s, rel=1e-12)
    am = np.sqrt(sym_a2m2(a, p))
    assert sym_mu(am, a, p) == pytest.approx(1 + s, rel=1e-14)   # k = a m
    assert Model(p).coupling(a) == pytest.approx(2 * s, rel=1e-14)


def test_symmetron_gamma2_matches_general_m_beta_form():
    # App. C: gamma_2^E = m^2 (dm^2/da) beta^2 Om / (2 H0^4 Pi Pi Pi) k^2/(a^4 H^2), with
    # dm^2/da taken here by finite differences of m^2(a)
    p = SYM
    for a in (0.6, 1.0):
        h = 1e-6 * a
        dm2 = (sym_m2(a + h, p) - sym_m2(a - h, p)) / (2 * h)
        assert dm2 == pytest.approx(sym_dm2_da(a, p), rel=1e-8)
        for k, k1, k2 in [(0.1, 0.2, 0.15), (1.0, 0.7071, 0.7071), (3.0, 1.0, 2.5)]:
            Pi = lambda q: (q / (a * H0_OVER_C)) ** 2 + sym_m2(a, p)     # noqa: E731
            H = E(a, p.omega_m) * H0_OVER_C
            gen = sym_m2(a, p) * dm2 * sym_beta2(a, p) * p.omega_m / (2 * Pi(k) * Pi(k1) * Pi(k2)) \
                * k * k / (a ** 4 * H * H)
            assert float(sym_gamma2E(k, k1, k2, a, p)) == pytest.approx(gen, rel=1e-7)


def test_symmetron_growth_lcdm_until_astar_then_scale_dependent():
    p = SYM
    model = Model(p)
    k = np.array([1e-4, 0.1, 1.0, 5.0])
    a = np.array([p.a_ini, 0.3, 0.5, 0.75, 1.0])
    G = solve_growth(k, a, p.omega_m, model.mu, model.gamma2_orth, p.a_ini)
    L = solve_growth(k, a, p.omega_m, ONE, ZERO, p.a_ini)
    assert np.max(np.abs(G[:3] / L[:3] - 1)) < 1e-10          # a <= a_*: LCDM (solver tol.)
    assert np.all(np.diff(G[-1, :, 0]) > 0)                  # enhanced growth on small scales
    assert G[-1, 0, 0] == pytest.approx(L[-1, 0, 0], rel=1e-6)   # k << a m: LCDM


def test_potential_screening_limits():
    pc = sym_phi_crit(SYM)
    assert np.all(eps_potential(np.array([1e-3, -1e-3]) * pc, pc) == 1.0)
    deep = np.array([1e3, -3e4]) * pc
    assert eps_potential(deep, pc) == pytest.approx(np.abs(pc / deep), rel=1e-15)
    assert eps_potential(np.array([0.0]), pc)[0] == 1.0


def test_symmetron_growth_resolves_the_switch_on():
    """Just after a_* the symmetron's gamma_2 term has a narrow peak for small k (its
    width in s = 1 - (a_*/a)^3 scales as (k/(a_* m_*))^2).  The oracle restarts its
    adaptive integration at a_*; a fixed-step RK4 in ln a whose steps grow geometrically
    from 1e-10 after a_* must agree with it, for the fundamental mode of a 1024 Mpc/h box."""
    from oracle.growth import growth_table
    p = SYM.with_(np1d=16, nmesh1d=32, box=1024.0, n_steps=4)
    model = Model(p)
    a_grid = p.a_ini + np.arange(5) * (1 - p.a_ini) / 4
    G, _ = growth_table(p, model, a_grid)
    k = 2 * np.pi * np.sqrt(np.arange(G.shape[1], dtype=float)) / p.box
    om = p.omega_m

    def rhs(lna, y):
        a = np.exp(lna)
        kap, Ea = 1.5 * om * a, E(a, om)
        mu, g2 = model.mu(k, a), model.gamma2_orth(k, a)
        f = 1 / (a * a * Ea)
        return np.array([y[1] * f, kap * mu * y[0] * f, y[3] * f,
                         (kap * mu * y[2] - kap * mu * y[0] ** 2 - 2 * a ** 4 * Ea * Ea * g2 * y[0] ** 2) * f])

    g0 = p.a_ini ** 2 * E(p.a_ini, om)
    y = np.array([np.ones_like(k), g0 + 0 * k, -3 / 7 + 0 * k, -6 / 7 * g0 + 0 * k])
    lna, lk = np.log(p.a_ini), np.log(p.sym_astar)
    for i in range(1, 5):
        l1 = np.log(a_grid[i])
        while lna < l1 - 1e-15:
            h = 1e-3 if lna < lk - 1e-15 else min(1e-3, 1e-10 + 0.02 * (lna - lk))
            if lna < lk < lna + h:
                h = lk - lna
            h = min(h, l1 - lna)
            k1 = rhs(lna, y)
            k2 = rhs(lna + h / 2, y + h / 2 * k1)
            k3 = rhs(lna + h / 2, y + h / 2 * k2)
            k4 = rhs(lna + h, y + h * k3)
            y, lna = y + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4), lna + h
        assert np.max(np.abs(y[0] / G[i, :, 0] - 1)) < 1e-10
        assert np.max(np.abs(y[2] / G[i, :, 3] - 1)) < 1e-10
