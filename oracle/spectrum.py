"""Initial linear power spectrum of the Gaussian initial conditions.

The paper reads its initial conditions from external simulations (Sec. 7); the
synthetic stand-in used here is a Gaussian random field with the Eisenstein & Hu
(1998) "no-wiggle" transfer function, normalised to sigma_8 of linear LCDM at
z = 0 and scaled back to a_ini with the LCDM growth factor of the growth ODE
(mu = 1), so every model starts from the same initial field.

Eisenstein & Hu 1998 (ApJ 496, 605), zero-baryon-oscillation fit:
  s       = 44.5 ln(9.83/(Om h^2)) / sqrt(1 + 10 (Ob h^2)^(3/4))  Mpc        (their eq. 26)
  alpha_G = 1 - 0.328 ln(431 Om h^2) f_b + 0.38 ln(22.3 Om h^2) f_b^2      (eq. 31)
  Gamma   = Om h [alpha_G + (1 - alpha_G)/(1 + (0.43 k s)^4)], k in 1/Mpc   (eq. 30)
  q       = (k / h Mpc^-1) Theta_2.7^2 / Gamma                              (eq. 28)
  T0      = L0 / (L0 + C0 q^2), L0 = ln(2e + 1.8 q), C0 = 14.2 + 731/(1 + 62.5 q)  (eq. 29)
"""

import numpy as np
from scipy import integrate

from .growth import solve_growth


def eh_nowiggle_T(k, om, ob, h, tcmb):
    """Transfer function T(k), k in h/Mpc."""
    k = np.asarray(k, dtype=np.float64)
    theta = tcmb / 2.7
    omh2 = om * h * h
    obh2 = ob * h * h
    fb = ob / om
    s = 44.5 * np.log(9.83 / omh2) / np.sqrt(1.0 + 10.0 * obh2 ** 0.75)
    alpha = 1.0 - 0.328 * np.log(431.0 * omh2) * fb + 0.38 * np.log(22.3 * omh2) * fb * fb
    gamma = om * h * (alpha + (1.0 - alpha) / (1.0 + (0.43 * k * h * s) ** 4))
    q = k * theta * theta / gamma
    L0 = np.log(2.0 * np.e + 1.8 * q)
    C0 = 14.2 + 731.0 / (1.0 + 62.5 * q)
    return L0 / (L0 + C0 * q * q)


def tophat_W(x):
    x = np.asarray(x, dtype=np.float64)
    return np.where(x > 1e-4, 3.0 * (np.sin(x) - x * np.cos(x)) / np.maximum(x, 1e-4) ** 3,
                    1.0 - x * x / 10.0)


def _sigma_R_sq_unnormalised(p, R=8.0):
    """(2 pi^2)^-1 int k^2 k^ns T^2(k) W^2(kR) dk over 1e-5 < k < 1e2 h/Mpc (the range
    beyond contributes below 1e-10 relative), integrated in ln k on panels narrower
    than one oscillation of the window."""
    def f(lnk):
        k = np.exp(lnk)
        return k ** 3 * k ** p.n_s * eh_nowiggle_T(k, p.omega_m, p.omega_b, p.h, p.t_cmb) ** 2 \
            * tophat_W(k * R) ** 2 / (2.0 * np.pi ** 2)
    edges = np.linspace(np.log(1e-5), np.log(1e2), 2001)
    tot = 0.0
    for lo, hi in zip(edges[:-1], edges[1:]):
        v, _ = integrate.quad(f, lo, hi, epsabs=1e-24, epsrel=1e-12, limit=50)
        tot += v
    return tot


def lcdm_D1_today(p):
    """D1 of the LCDM growth ODE (mu = 1), normalised to 1 at a_ini, at a = 1."""
    G = solve_growth(np.array([0.0]), np.array([1.0]), p.omega_m,
                     lambda k, a: np.ones_like(k), lambda k, a: np.zeros_like(k), p.a_ini)
    return float(G[0, 0, 0])


class InitialSpectrum:
    """P_ini(k) = A k^ns T^2(k) / D1_LCDM(a=1)^2, with A fixed by sigma_8."""

    def __init__(self, p):
        self.p = p
        self.A = p.sigma8 ** 2 / _sigma_R_sq_unnormalised(p)
        self.D1_today = lcdm_D1_today(p)

    def P_today(self, k):
        k = np.asarray(k, dtype=np.float64)
        p = self.p
        return self.A * k ** p.n_s * eh_nowiggle_T(k, p.omega_m, p.omega_b, p.h, p.t_cmb) ** 2

    def P_ini(self, k):
        return self.P_today(k) / self.D1_today ** 2
