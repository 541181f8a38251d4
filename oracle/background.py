"""Flat LCDM background and the super-comoving time (Sec. 2; App. B fiducial H(a)).

Time unit 1/H0: H(a) = E(a) = sqrt(Omega_m a^-3 + Omega_L), Omega_L = 1 - Omega_m.
Super-comoving time: d tau = dt / a^2 = da / (a^3 E(a)).
"""

import numpy as np
from scipy import integrate


def E(a, om):
    return np.sqrt(om * np.asarray(a, dtype=np.float64) ** -3 + (1.0 - om))


def omega_m_of_a(a, om):
    a = np.asarray(a, dtype=np.float64)
    return om * a ** -3 / E(a, om) ** 2


def kappa(a, om):
    """kappa = 4 pi G rho_bar a^4 = (3/2) Omega_m H0^2 a (Sec. 2), H0 = 1."""
    return 1.5 * om * np.asarray(a, dtype=np.float64)


def dtau_da(a, om):
    return 1.0 / (a ** 3 * E(a, om))


def tau_between(a0, a1, om):
    """tau(a1) - tau(a0) = int_{a0}^{a1} da / (a^3 E), adaptive quadrature."""
    if a1 == a0:
        return 0.0
    val, _ = integrate.quad(dtau_da, a0, a1, args=(om,), epsabs=0.0, epsrel=1e-13,
                            limit=500)
    return val


def dlna_dtau(a, om):
    """(1/a) da/dtau = a^2 E(a): the initial growth rate of the EdS growing mode
    used for D1'(tau_ini) (Sec. 3.1)."""
    return a ** 2 * E(a, om)
