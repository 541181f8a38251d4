"""Exact second-order growth of a Fourier-space triangle, and the approximation the COLA
path uses in its place (Sec. 4.2; Fig. 1).

THIS MODULE IS TEST INFRASTRUCTURE (see the package header).

A triangle is k = k1 + k2 with cos(theta) = k1.k2/(k1 k2) = (k^2 - k1^2 - k2^2)/(2 k1 k2).
Primes are d/dtau and kappa = 1.5 Omega_m a. Per triangle:

  D1''(q) = kappa mu(q, a) D1(q)                                    for q = k1, k2   (Sec. 4.1)
  D2'' = kappa mu(k) D2 - kappa mu(k) D1(k1) D1(k2)
         x [1 - (2 mu(k1) - mu(k))/mu(k) cos^2(theta) + 2 a^4 H^2 gamma_2/(kappa mu(k))]
                                                                    (Sec. 4.2, exact D2 equation)
  gamma_2 = gamma_2^E(k, k1, k2, a) + (3/2) Omega_m(a) [mu(k) - mu(k1)] k1.k2/k2^2   (Sec. 4)

The initial conditions at a_ini are the EdS values: D1 = 1, D1' = (a^-1 da/dtau), and
D2 = -(3/7)(1 - cos^2 theta), D2' = -(6/7)(1 - cos^2 theta)(a^-1 da/dtau).

The terms that single out k1 are taken as printed. For the triangles of Fig. 1 they
reduce to symmetric values: equilateral, orthogonal, and squeezed with k = k1.

The approximation is D2_hat(k, a)(1 - cos^2 theta), with D2_hat from growth.solve_growth
(the approximate D2 equation, gamma_2 at k1 = k2 = k/sqrt2). Fig. 1 plots the ratio of the
exact D2 to it. The approximation is exact for LCDM and nDGP, where mu does not depend on
k and gamma_2 is proportional to (1 - cos^2 theta) (Sec. 4.2).
"""

import numpy as np

from .background import E, kappa, dlna_dtau, omega_m_of_a
from .growth import _integrate_pieces, growth_breaks, solve_growth
from .models import Model, fr_gamma2E, dgp_gamma2E_orth, sym_gamma2E
from .params import MODEL_FR, MODEL_NDGP, MODEL_SYMMETRON, MODEL_MBETA


def cos_theta(k, k1, k2):
    return (k * k - k1 * k1 - k2 * k2) / (2.0 * k1 * k2)


def gamma2E(model, k, k1, k2, a):
    """gamma_2^E of the model at the triangle (Secs. 5.1-5.2, App. C); zero for LCDM and
    for runs with LCDM growth factors."""
    k, k1, k2 = (np.asarray(x, dtype=np.float64) for x in (k, k1, k2))
    if model.lcdm_growth or model.kind not in (MODEL_FR, MODEL_NDGP, MODEL_SYMMETRON, MODEL_MBETA):
        return np.zeros_like(k)
    if model.kind == MODEL_MBETA:
        return model.mb.gamma2E(k, k1, k2, a)
    if model.kind == MODEL_FR:
        return fr_gamma2E(k, k1, k2, a, model.om, model.p.fr0_abs)
    if model.kind == MODEL_SYMMETRON:
        return sym_gamma2E(k, k1, k2, a, model.p)
    c = cos_theta(k, k1, k2)
    return dgp_gamma2E_orth(a, model.om, model.p.rc_h0) * (1.0 - c * c)


def solve_d2_triangle(k, k1, k2, a_out, p, rtol=1e-12, atol=1e-14):
    """Exact D2(k, k1, k2, a) at the scale factors a_out (ascending, >= a_ini), shape
    (len(a_out), n) for n triangles given by the arrays k, k1, k2 [h/Mpc]."""
    model = Model(p)
    om = p.omega_m
    k, k1, k2 = (np.atleast_1d(np.asarray(x, dtype=np.float64)) for x in (k, k1, k2))
    n = k.size
    c = cos_theta(k, k1, k2)
    c2 = c * c
    k1dotk2_over_k2sq = k1 * c / k2

    def rhs(a, y):
        D1a, dD1a, D1b, dD1b, D2, dD2 = (y[i * n:(i + 1) * n] for i in range(6))
        kap = kappa(a, om)
        mu, mu1, mu2 = model.mu(k, a), model.mu(k1, a), model.mu(k2, a)
        g2 = gamma2E(model, k, k1, k2, a) + 1.5 * omega_m_of_a(a, om) * (mu - mu1) * k1dotk2_over_k2sq
        Ea = E(a, om)
        src = 1.0 - (2.0 * mu1 - mu) / mu * c2 + 2.0 * a ** 4 * Ea * Ea * g2 / (kap * mu)
        dd2 = kap * mu * D2 - kap * mu * D1a * D1b * src
        f = 1.0 / (a ** 3 * Ea)
        return np.concatenate([dD1a * f, kap * mu1 * D1a * f, dD1b * f, kap * mu2 * D1b * f,
                               dD2 * f, dd2 * f])

    g0 = dlna_dtau(p.a_ini, om)
    y0 = np.concatenate([np.ones(n), np.full(n, g0), np.ones(n), np.full(n, g0),
                         -3.0 / 7.0 * (1.0 - c2), -6.0 / 7.0 * (1.0 - c2) * g0])
    a_out = np.atleast_1d(np.asarray(a_out, dtype=np.float64))
    out = np.empty((a_out.size, n))
    need = a_out > p.a_ini
    if np.any(need):
        ys = iter(_integrate_pieces(rhs, y0, p.a_ini, a_out[need], growth_breaks(p, model), rtol,
                                    atol))
    for i in range(a_out.size):
        y = next(ys) if need[i] else y0
        out[i] = y[4 * n:5 * n]
    return out


def approx_d2_triangle(k, k1, k2, a_out, p, rtol=1e-12, atol=1e-14):
    """The approximation D2_hat(k, a)(1 - cos^2 theta), shape (len(a_out), n)."""
    model = Model(p)
    k, k1, k2 = (np.atleast_1d(np.asarray(x, dtype=np.float64)) for x in (k, k1, k2))
    c = cos_theta(k, k1, k2)
    G = solve_growth(k, np.atleast_1d(a_out), p.omega_m, model.mu, model.gamma2_orth, p.a_ini,
                     rtol=rtol, atol=atol, breaks=growth_breaks(p, model))
    return G[:, :, 3] * (1.0 - c * c)


def fig1_triangles(k, config, squeeze=1e-3):
    """(k, k1, k2) of the Fig. 1 configurations: equilateral k = k1 = k2, orthogonal
    k1 = k2 = k/sqrt2, squeezed k1 = k with k2 = squeeze * k."""
    k = np.asarray(k, dtype=np.float64)
    if config == "equilateral":
        return k, k.copy(), k.copy()
    if config == "orthogonal":
        return k, k / np.sqrt(2.0), k / np.sqrt(2.0)
    if config == "squeezed":
        return k, k.copy(), squeeze * k
    raise ValueError(config)
