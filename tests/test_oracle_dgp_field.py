"""Pins of the oracle's nDGP second-order pieces against the nDGP field equation itself
(Sec. 6.2, eq. ndgpfieldeq):

    nabla^2 phi + C_nl [(nabla^2 phi)^2 - (nabla_i nabla_j phi)^2] = kappa delta / (3 beta),

written here once with the nonlinear coefficient read as C_nl = 2 (r_c H0)^2 / (3 beta a^4)
(time unit 1/H0, c = 1).  Two independent solutions of that one equation fix two printed
results the oracle uses:

(i)  the O(A1 A2) response to two plane waves, solved on a periodic mesh with spectral
     derivatives, gives gamma_2^E of Sec. 5.2 in the normalisation of eq. eulerian
     (oracle.models.dgp_gamma2E);
(ii) the spherically symmetric solution for a top-hat, integrated numerically in r,
     gives eps = phi'/phi'_lin, which must equal eps_vainshtein(vainshtein_x(delta_bar))
     with the mean overdensity delta_bar inside r (oracle.models.vainshtein_x).

With the printed coefficient 2 r_c^2 / a^4 both results come out 3 beta times the printed
gamma_2^E and x; the tests record that as well, since it is why the coefficient is read
with the 1/(3 beta).
"""

import numpy as np
import pytest
from scipy import integrate

from oracle.background import E
from oracle.models import dgp_beta, dgp_gamma2E, eps_vainshtein, vainshtein_x
from oracle.params import READ_X_NO_A3, READ_X_TOTAL_DENSITY

OM = 0.3


def c_nl(a, rc, printed=False):
    """Coefficient of the nonlinear term of the nDGP field equation (see module doc)."""
    b = dgp_beta(a, OM, rc)
    return 2.0 * rc * rc / a ** 4 if printed else 2.0 * rc * rc / (3.0 * b * a ** 4)


# ----------------------------------------------------------------------------- (i) gamma_2^E
def _two_wave_response(m1, m2, a, rc, n=16, L=50.0, A1=0.7, A2=1.3, printed=False):
    """Amplitude of cos((k1 + k2).x) in nabla^2 phi at second order, divided by A1 A2, for
    delta = A1 cos(k1.x) + A2 cos(k2.x) on an n^3 periodic mesh."""
    x = np.arange(n) * L / n
    X = np.meshgrid(x, x, x, indexing="ij")
    k1 = 2 * np.pi * np.asarray(m1) / L
    k2 = 2 * np.pi * np.asarray(m2) / L
    delta = A1 * np.cos(sum(k1[i] * X[i] for i in range(3))) \
        + A2 * np.cos(sum(k2[i] * X[i] for i in range(3)))
    b = dgp_beta(a, OM, rc)
    kap = 1.5 * OM * a
    nu = np.fft.fftfreq(n, 1.0 / n)
    K = np.meshgrid(*(2 * np.pi * nu / L,) * 3, indexing="ij")
    ksq = K[0] ** 2 + K[1] ** 2 + K[2] ** 2
    # first order: nabla^2 phi1 = kappa delta / (3 beta)
    phi1_k = np.where(ksq > 0, -kap / (3 * b) * np.fft.fftn(delta) / np.where(ksq > 0, ksq, 1), 0)
    lap = np.fft.ifftn(-ksq * phi1_k).real
    Q = lap * lap
    for i in range(3):
        for j in range(3):
            hij = np.fft.ifftn(-K[i] * K[j] * phi1_k).real
            Q -= hij * hij
    # second order: nabla^2 phi2 = -C_nl Q
    lap2 = -c_nl(a, rc, printed) * Q
    idx = tuple(int(v) % n for v in (np.asarray(m1) + np.asarray(m2)))
    amp = 2.0 * np.fft.fftn(lap2)[idx].real / n ** 3
    return amp / (A1 * A2)


@pytest.mark.parametrize("m1,m2", [((1, 0, 0), (0, 2, 0)), ((1, 1, 0), (2, 0, 1)),
                                   ((2, 0, 0), (1, 1, 0)), ((0, 1, 2), (1, 0, -1))])
@pytest.mark.parametrize("a,rc", [(0.3, 1.0), (0.7, 0.5), (1.0, 1.0), (1.0, 3.0)])
def test_gamma2E_is_the_second_order_response_of_the_field_equation(m1, m2, a, rc):
    # eq. eulerian: nabla^2 Phi contains a^4 H^2 A1 A2 gamma_2^E(k1, k2) cos((k1 + k2).x)
    # for the pair of waves; Phi_N is linear in delta, so only phi contributes.
    v1, v2 = np.asarray(m1, float), np.asarray(m2, float)
    cos2 = (v1 @ v2) ** 2 / ((v1 @ v1) * (v2 @ v2))
    measured = _two_wave_response(m1, m2, a, rc) / (a ** 4 * E(a, OM) ** 2)
    assert measured == pytest.approx(dgp_gamma2E(a, OM, rc, cos2), rel=1e-10)
    if cos2 < 1e-12:   # the orthogonal case is the one the growth equations use
        assert measured < 0
    # the printed coefficient gives 3 beta times the printed gamma_2^E
    printed = _two_wave_response(m1, m2, a, rc, printed=True) / (a ** 4 * E(a, OM) ** 2)
    assert printed / measured == pytest.approx(3 * dgp_beta(a, OM, rc), rel=1e-10)


def test_gamma2E_vanishes_for_parallel_waves():
    # (1 - cos^2 theta): collinear waves give no second-order field
    assert abs(_two_wave_response((1, 0, 0), (2, 0, 0), 1.0, 1.0)) < 1e-12 * abs(
        _two_wave_response((1, 0, 0), (0, 2, 0), 1.0, 1.0))


# ----------------------------------------------------------------------------- (ii) Vainshtein
def test_spherical_reduction_of_the_nonlinear_operator():
    # (nabla^2 phi)^2 - (nabla_i nabla_j phi)^2 = (2 / r^2) d/dr (r phi'^2) for phi(r):
    # checked at a point by a finite-difference Hessian of phi = exp(-r^2/2) in 3D
    phi = lambda x: np.exp(-0.5 * (x @ x))   # noqa: E731
    x0 = np.array([0.4, -0.3, 0.5])
    h = 1e-3
    H = np.zeros((3, 3))
    for i in range(3):
        for j in range(3):
            ei, ej = np.eye(3)[i] * h, np.eye(3)[j] * h
            H[i, j] = (phi(x0 + ei + ej) - phi(x0 + ei - ej) - phi(x0 - ei + ej)
                       + phi(x0 - ei - ej)) / (4 * h * h)
    lhs = np.trace(H) ** 2 - np.sum(H * H)
    r = np.sqrt(x0 @ x0)
    dphi = lambda s: -s * np.exp(-0.5 * s * s)   # noqa: E731
    d_r_dphi2 = (((r + h) * dphi(r + h) ** 2) - ((r - h) * dphi(r - h) ** 2)) / (2 * h)
    assert lhs == pytest.approx(2 / r ** 2 * d_r_dphi2, rel=1e-5)


def _tophat_eps(delta0, R, r_eval, a, rc, printed=False):
    """eps(r) = phi'/phi'_lin of the spherical solution for delta = delta0 inside R.

    In spherical symmetry the field equation is (r^2 y + 2 C_nl r y^2)' = r^2 s(r),
    y = phi', s = kappa delta / (3 beta).  With y = r g it reads
    d g / d ln r = (s - 3 g - 6 C_nl g^2) / (1 + 4 C_nl g), integrated numerically from
    r = 1e-8 R (any starting g is attracted as r^3 to the regular solution)."""
    b = dgp_beta(a, OM, rc)
    s0 = 1.5 * OM * a * delta0 / (3 * b)
    C = c_nl(a, rc, printed)

    def rhs(lnr, g, s):
        return (s - 3 * g - 6 * C * g * g) / (1 + 4 * C * g)

    lo = np.log(1e-8 * R)
    r_in = np.sort([r for r in r_eval if r <= R])
    r_out = np.sort([r for r in r_eval if r > R])
    res = {}
    s1 = integrate.solve_ivp(rhs, (lo, np.log(R)), [s0 / 3], args=(s0,), method="DOP853",
                             rtol=1e-13, atol=1e-30, dense_output=True)
    for r in r_in:
        res[r] = s1.sol(np.log(r))[0] * r
    if len(r_out):
        s2 = integrate.solve_ivp(rhs, (np.log(R), np.log(r_out[-1])), s1.y[:, -1], args=(0.0,),
                                 method="DOP853", rtol=1e-13, atol=1e-30, dense_output=True)
        for r in r_out:
            res[r] = s2.sol(np.log(r))[0] * r
    # linear solution: r^2 y_lin = int_0^r r'^2 s = s0 min(r, R)^3 / 3
    return np.array([res[r] / (s0 * min(r, R) ** 3 / (3 * r * r)) for r in r_eval])


@pytest.mark.parametrize("delta0", [-0.6, 1e-3, 0.5, 30.0, 2000.0])
@pytest.mark.parametrize("a,rc", [(0.25, 1.0), (0.6, 0.5), (1.0, 1.0), (1.0, 3.0)])
def test_vainshtein_eps_is_the_spherical_solution(delta0, a, rc):
    R = 2.0
    r_eval = [0.3, 1.0, 2.0, 3.0, 8.0]
    eps = _tophat_eps(delta0, R, r_eval, a, rc)
    b = dgp_beta(a, OM, rc)
    dbar = np.array([delta0 * min(1.0, (R / r) ** 3) for r in r_eval])
    want = eps_vainshtein(vainshtein_x(dbar, a, OM, rc, b))
    assert eps == pytest.approx(want, rel=1e-9)
    # underdense regions are anti-screened, overdense ones screened
    assert np.all(eps > 1) if delta0 < 0 else np.all(eps <= 1)


def test_vainshtein_readings():
    a, rc = 0.5, 1.0
    b = dgp_beta(a, OM, rc)
    # mean density is unscreened under the field-equation reading
    assert eps_vainshtein(vainshtein_x(0.0, a, OM, rc, b)) == 1.0
    # the printed rho/rho_bar reading screens it
    assert eps_vainshtein(vainshtein_x(0.0, a, OM, rc, b, READ_X_TOTAL_DENSITY)) < 0.99
    # the spherical solution with the printed coefficient is the x of that coefficient:
    # 3 beta times larger
    eps_p = _tophat_eps(5.0, 2.0, [1.0], a, rc, printed=True)[0]
    x = vainshtein_x(5.0, a, OM, rc, b)
    assert eps_p == pytest.approx(eps_vainshtein(3 * b * x), rel=1e-9)
    # without a^-3 the two readings differ exactly by a^3
    assert vainshtein_x(2.0, a, OM, rc, b, READ_X_NO_A3) == pytest.approx(
        a ** 3 * vainshtein_x(2.0, a, OM, rc, b), rel=1e-15)
    # 1 + x > 0 for every delta_bar >= -1 and every a (beta^2 a^3 > (r_c H0)^2 Om)
    for aa in np.geomspace(0.01, 1.0, 40):
        for r in (0.25, 1.0, 5.0):
            bb = dgp_beta(aa, OM, r)
            assert 1 + vainshtein_x(-1.0, aa, OM, r, bb) > 1.0 / 9.0
            assert 1 + vainshtein_x(-5.0, aa, OM, r, bb) > 1.0 / 9.0   # clamped at -1
