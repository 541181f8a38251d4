"""Pins of the tabulated general {m(a), beta(a)} model (App. C) in the oracle.

* Hu-Sawicki f(R) is the {m, beta} model with beta = 1/sqrt(6) and the Sec. 5.1 m^2(a)
  (App. C): tabulated on 64 knots, the general model reproduces the f(R) mu, gamma_2^E,
  a^2 m^2, C = 1/3, the growth factors, and Phi_crit = (3/2)|f_R(a)| (App. C's worked
  case), to the accuracy of the cubic splines.
* Constant beta and m: the Phi_crit integral has the closed form
  (3 Om / (2 m^2/H0^2)) (a_0^-3 - a^-3), and the splines are exact.
* mu -> 1 for k -> 0 and 1 + 2 beta^2 for k -> infinity.
"""

import numpy as np
import pytest

from oracle.growth import solve_growth
from oracle.models import Model, fr_a2m2, fr_fR_abs, fr_gamma2E, fr_mu
from oracle.params import H0_OVER_C, MODEL_FR, MODEL_MBETA, Params

OM, FR0 = 0.3, 1e-5


def hs_tables(n=64, a_lo=0.01, a_hi=2.0):
    lna = np.linspace(np.log(a_lo), np.log(a_hi), n)
    a = np.exp(lna)
    m2 = fr_a2m2(a, OM, FR0) / (a * a * H0_OVER_C ** 2)
    return Params(model=MODEL_MBETA, omega_m=OM, mb_lna=tuple(lna),
                  mb_beta=tuple(np.full(n, 1 / np.sqrt(6.0))), mb_m2=tuple(m2))


def test_fr_as_tabulated_m_beta_model():
    p = hs_tables()
    m = Model(p)
    k = np.array([0.01, 0.1, 0.5, 2.0, 8.0])
    for a in (0.05, 0.3, 0.77, 1.0):
        assert m.mu(k, a) == pytest.approx(fr_mu(k, a, OM, FR0), rel=1e-5)
        assert m.a2m2(a) == pytest.approx(float(fr_a2m2(a, OM, FR0)), rel=1e-5)
        assert m.coupling(a) == pytest.approx(1.0 / 3.0, rel=1e-14)
        kk = k / np.sqrt(2.0)
        assert m.gamma2_orth(k, a) == pytest.approx(fr_gamma2E(k, kk, kk, a, OM, FR0), rel=1e-3)
        # App. C: the integral gives (3/2)|f_R(a)| (from a_0 = 0.01, where the rest is
        # below 1e-10 of it)
        assert m.phi_crit(a) == pytest.approx(1.5 * float(fr_fR_abs(a, OM, FR0)), rel=1e-5)
    # growth factors of the two descriptions
    pf = Params(model=MODEL_FR, omega_m=OM, fr0_abs=FR0)
    mf = Model(pf)
    kq = np.array([0.02, 0.3, 1.5])
    a_out = np.array([0.5, 1.0])
    Gm = solve_growth(kq, a_out, OM, m.mu, m.gamma2_orth, p.a_ini)
    Gf = solve_growth(kq, a_out, OM, mf.mu, mf.gamma2_orth, pf.a_ini)
    assert np.allclose(Gm, Gf, rtol=1e-5, atol=0)


def test_constant_m_beta_phi_crit_closed_form():
    lna = np.linspace(np.log(0.02), np.log(1.1), 6)
    beta, m2 = 0.7, 4.0e6
    p = Params(model=MODEL_MBETA, omega_m=OM, mb_lna=tuple(lna), mb_beta=(beta,) * 6,
               mb_m2=(m2,) * 6)
    m = Model(p)
    a0 = np.exp(lna[0])
    for a in (0.05, 0.5, 1.0):
        want = 1.5 * OM / m2 * (a0 ** -3 - a ** -3)
        assert m.phi_crit(a) == pytest.approx(want, rel=1e-11)
        assert m.coupling(a) == pytest.approx(2 * beta * beta, rel=1e-14)
        assert m.mb.dm2_da(a) == pytest.approx(0.0, abs=1e-9 * m2)
        # mu limits and gamma_2 vanishing with dm^2/da
        assert m.mu(np.array([1e-9]), a)[0] == pytest.approx(1.0, abs=1e-12)
        assert m.mu(np.array([1e9]), a)[0] == pytest.approx(1 + 2 * beta * beta, rel=1e-12)
        assert np.all(np.abs(m.gamma2_orth(np.array([0.1, 1.0]), a)) < 1e-20)
