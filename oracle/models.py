"""Modified-gravity model functions (Secs. 4-6, App. B-C).

Each model supplies, as functions of wavenumber k [h/Mpc] and scale factor a:

* mu(k, a): linear modification of the Poisson equation (Sec. 4, eq. eulerian);
* gamma2_orth(k, a): the Lagrangian second-order kernel gamma_2 evaluated at the
  orthogonal triangle k1 = k2 = k/sqrt(2), k1.k2 = 0, the argument the approximate
  second-order growth equation uses (Sec. 4.2, eq. fofrapprox).  At k1 . k2 = 0
  the extra Lagrangian term (3/2) Omega_m(a) [mu(k)-mu(k1)] k1.k2/k2^2 vanishes, so
  gamma_2 = gamma_2^E there;
* a2m2(a): a^2 m^2(a) of the linear field equation (Sec. 6; App. B), in (h/Mpc)^2;
* coupling(a): C(a) of the general field equation (App. B):
  nabla^2 phi = a^2 m^2 phi + C kappa delta eps_screen;
* the screening factor eps_screen (Sec. 6).
"""

import numpy as np

from .background import E, omega_m_of_a
from .params import (MODEL_LCDM, MODEL_FR, MODEL_NDGP, MODEL_SYMMETRON, MODEL_MBETA,
                     MODEL_KMOUFLAGE, FILTER_GAUSS,
                     FILTER_TOPHAT, FILTER_SHARPK, H0_OVER_C, READ_X_TOTAL_DENSITY, READ_X_NO_A3)


# ----------------------------------------------------------------------------- f(R)
def fr_X(a, om):
    return om * np.asarray(a, dtype=np.float64) ** -3 + 4.0 * (1.0 - om)


def fr_Y(om):
    return om + 4.0 * (1.0 - om)


def fr_a2m2(a, om, fr0):
    """a^2 m^2(a) for Hu-Sawicki n = 1 (Sec. 5.1, eq. mofahus):
    m^2 = H0^2 (Om + 4 OL) / (2|fR0|) * ((Om a^-3 + 4 OL)/(Om + 4 OL))^3,
    with H0 -> H0/c so that m is in h/Mpc."""
    X, Y = fr_X(a, om), fr_Y(om)
    return a * a * H0_OVER_C ** 2 * Y * (X / Y) ** 3 / (2.0 * fr0)


def fr_fR_abs(a, om, fr0):
    """|f_R(a)| = |fR0| ((Om + 4 OL)/(Om a^-3 + 4 OL))^2 (Sec. 5.1)."""
    return fr0 * (fr_Y(om) / fr_X(a, om)) ** 2


def fr_mu(k, a, om, fr0):
    """mu = 1 + (1/3) k^2 / (k^2 + a^2 m^2) (Sec. 5.1)."""
    k2 = np.asarray(k, dtype=np.float64) ** 2
    return 1.0 + k2 / (3.0 * (k2 + fr_a2m2(a, om, fr0)))


def fr_Pi(k, a, om, fr0):
    """Pi(k,a) = (k/(a H0))^2 + (Om a^-3 + 4 OL)^3 / (2|fR0| (Om + 4 OL)^2) (Sec. 5.1)."""
    X, Y = fr_X(a, om), fr_Y(om)
    return (np.asarray(k, dtype=np.float64) / (a * H0_OVER_C)) ** 2 \
        + X ** 3 / (2.0 * fr0 * Y ** 2)


def fr_gamma2E(k, k1, k2, a, om, fr0):
    """gamma_2^E of Hu-Sawicki f(R) (Sec. 5.1):
    -(9 Om^2/(48 a^6 |fR0|^2)) (k/(aH))^2 X^5/Y^4 / (Pi(k) Pi(k1) Pi(k2))."""
    X, Y = fr_X(a, om), fr_Y(om)
    kah = np.asarray(k, dtype=np.float64) / (a * H0_OVER_C * E(a, om))
    return (-9.0 * om * om / (48.0 * a ** 6 * fr0 * fr0) * kah * kah * X ** 5 / Y ** 4
            / (fr_Pi(k, a, om, fr0) * fr_Pi(k1, a, om, fr0) * fr_Pi(k2, a, om, fr0)))


# ----------------------------------------------------------------------------- nDGP
def dgp_beta(a, om, rc):
    """beta_DGP = 1 + 2 r_c H (1 + Hdot/(3 H^2)) (Sec. 5.2).  With Hdot the
    cosmic-time derivative, Hdot/H^2 = dlnH/dlna = -(3/2) Omega_m(a) in flat LCDM,
    so beta = 1 + 2 (r_c H0) E(a) (1 - Omega_m(a)/2)."""
    return 1.0 + 2.0 * rc * E(a, om) * (1.0 - 0.5 * omega_m_of_a(a, om))


def dgp_mu(a, om, rc):
    return 1.0 + 1.0 / (3.0 * dgp_beta(a, om, rc))


def dgp_gamma2E(a, om, rc, cos2=0.0):
    """gamma_2^E = -(H0/H)^2 (r_c H0)^2 Om^2 / (6 beta^3 a^6) (1 - cos^2 theta) (Sec. 5.2).

    Pinned against the nDGP field equation (Sec. 6.2, eq. ndgpfieldeq): the O(A1 A2)
    response of that equation to two plane waves, solved on a mesh with the nonlinear
    coefficient 2 (r_c H0)^2 / (3 beta a^4) (the printed 2 r_c^2 / a^4 lacks the 1/(3 beta)
    that reproduces both this gamma_2^E and the printed prefactor of the Vainshtein x)."""
    b = dgp_beta(a, om, rc)
    return -(rc * rc * om * om) / (6.0 * E(a, om) ** 2 * b ** 3 * a ** 6) * (1.0 - cos2)


def dgp_gamma2E_orth(a, om, rc):
    """gamma_2^E of Sec. 5.2 at cos theta = 0 (the orthogonal triangle of Sec. 4.2)."""
    return dgp_gamma2E(a, om, rc, 0.0)


# ----------------------------------------------------------------------------- symmetron
# A {m(a), beta(a)} model (App. C): mu = 1 + 2 beta^2 k^2/(k^2 + a^2 m^2),
# gamma_2^E = m^2 (dm^2/da) beta^2 Om / (2 H0^4 Pi(k) Pi(k1) Pi(k2)) k^2/(a^4 H^2) with
# Pi(q) = (q/(a H0))^2 + m^2/H0^2, field equation nabla^2 phi = a^2 m^2 phi + 2 beta^2
# kappa delta eps_screen, eps_screen = min(1, |Phi_crit/Phi_N|).  For the symmetron
# beta = beta_* sqrt(s), m^2 = m_*^2 s, s = 1 - (a_*/a)^3 after a_* and beta = m = 0 before.
def sym_s(a, astar):
    a = np.asarray(a, dtype=np.float64)
    return np.where(a > astar, 1.0 - (astar / np.maximum(a, 1e-300)) ** 3, 0.0)


def sym_beta2(a, p):
    return p.sym_beta ** 2 * sym_s(a, p.sym_astar)


def sym_m2(a, p):
    """m^2(a)/H0^2."""
    return p.sym_mass ** 2 * sym_s(a, p.sym_astar)


def sym_dm2_da(a, p):
    """d(m^2/H0^2)/da = m_*^2/H0^2 * 3 a_*^3 / a^4 after a_*, else 0."""
    a = np.asarray(a, dtype=np.float64)
    return np.where(a > p.sym_astar, p.sym_mass ** 2 * 3.0 * p.sym_astar ** 3 / a ** 4, 0.0)


def sym_a2m2(a, p):
    """a^2 m^2(a) in (h/Mpc)^2 (H0 -> H0/c)."""
    return a * a * H0_OVER_C ** 2 * sym_m2(a, p)


def sym_mu(k, a, p):
    k2 = np.asarray(k, dtype=np.float64) ** 2
    b2 = sym_beta2(a, p)
    if not np.any(b2 > 0):
        return np.ones_like(k2)
    return 1.0 + 2.0 * b2 * k2 / (k2 + sym_a2m2(a, p))


def sym_gamma2E(k, k1, k2, a, p):
    k = np.asarray(k, dtype=np.float64)
    if not np.any(sym_s(a, p.sym_astar) > 0):
        return np.zeros_like(k)
    m2 = sym_m2(a, p)
    Pi = lambda q: (np.asarray(q, dtype=np.float64) / (a * H0_OVER_C)) ** 2 + m2  # noqa: E731
    H = E(a, p.omega_m) * H0_OVER_C
    return (m2 * sym_dm2_da(a, p) * sym_beta2(a, p) * p.omega_m / (2.0 * Pi(k) * Pi(k1) * Pi(k2))
            * k * k / (a ** 4 * H * H))


def sym_phi_crit(p):
    """Phi_crit of the symmetron from the App. C integral with Phi_crit(a_*) = 0:
    (9 Om/(2 beta(a))) int_{a_*}^a beta/((m^2/H0^2) a'^4) da' = 3 Om/(a_*^3 m_*^2/H0^2),
    the same at every a > a_*.  (The printed closed form is half of this; the integral,
    which reproduces the f(R) value (3/2)|f_R(a)| exactly, is taken as the definition.)"""
    return 3.0 * p.omega_m / (p.sym_astar ** 3 * p.sym_mass ** 2)


# ----------------------------------------------------------------------------- general {m, beta}
class MBetaTables:
    """A general {m(a), beta(a)} model (App. C) given as beta and m^2/H0^2 at knots in ln a,
    interpolated by natural cubic splines of beta(ln a) and ln(m^2/H0^2)(ln a) (scipy's
    CubicSpline as the library step).  mu = 1 + 2 beta^2 k^2/(k^2 + a^2 m^2);
    gamma_2^E = m^2 (dm^2/da) beta^2 Om / (2 H0^4 Pi Pi Pi) k^2/(a^4 H^2) with
    Pi(q) = (q/(a H0))^2 + m^2/H0^2; field equation with C = 2 beta^2 and potential screening
    by Phi_crit(a) = (9 Om / (2 beta(a))) int_{a_0}^a beta/((m^2/H0^2) a'^4) da', a_0 the first
    knot with Phi_crit(a_0) = 0 (the App. C integral)."""

    def __init__(self, p):
        from scipy.interpolate import CubicSpline
        lna = np.asarray(p.mb_lna, dtype=np.float64)
        self.om = p.omega_m
        self.a0 = float(np.exp(lna[0]))
        self.sb = CubicSpline(lna, np.asarray(p.mb_beta, dtype=np.float64), bc_type="natural")
        self.sm = CubicSpline(lna, np.log(np.asarray(p.mb_m2, dtype=np.float64)), bc_type="natural")
        self.dsm = self.sm.derivative()

    def beta(self, a):
        return self.sb(np.log(a))

    def m2(self, a):
        """m^2(a)/H0^2."""
        return np.exp(self.sm(np.log(a)))

    def dm2_da(self, a):
        return self.m2(a) * self.dsm(np.log(a)) / a

    def a2m2(self, a):
        return a * a * H0_OVER_C ** 2 * self.m2(a)

    def mu(self, k, a):
        k2 = np.asarray(k, dtype=np.float64) ** 2
        b = self.beta(a)
        return 1.0 + 2.0 * b * b * k2 / (k2 + self.a2m2(a))

    def gamma2E(self, k, k1, k2, a):
        m2 = self.m2(a)
        Pi = lambda q: (np.asarray(q, dtype=np.float64) / (a * H0_OVER_C)) ** 2 + m2  # noqa: E731
        H = E(a, self.om) * H0_OVER_C
        b = self.beta(a)
        k = np.asarray(k, dtype=np.float64)
        return (m2 * self.dm2_da(a) * b * b * self.om / (2.0 * Pi(k) * Pi(k1) * Pi(k2))
                * k * k / (a ** 4 * H * H))

    def phi_crit(self, a):
        from scipy import integrate
        f = lambda x: float(self.beta(x)) / (float(self.m2(x)) * x ** 4)  # noqa: E731
        I, _ = integrate.quad(f, self.a0, a, epsabs=0.0, epsrel=1e-12, limit=200)
        return 4.5 * self.om / float(self.beta(a)) * I


# ----------------------------------------------------------------------------- k-Mouflage
# Gradient screening (App. B) for a kinetic function P(X) = -1 + X + K0 X^m (the form is
# this reading's choice; the paper leaves X*(|grad Phi_N|) to the user):
# P_X(X*)^2 X* = (lambda |grad Phi_N|)^2, eps = min(1, 1/P_X(X*)); C = 2 beta^2, m(a) = 0;
# linear growth mu = 1 + 2 beta^2 / P_X(X(a)) with the cosmological X(a) = x0 a^xn, and
# gamma_2 = 0 (none is given).
def km_px(X, k0, m):
    return 1.0 + m * k0 * np.asarray(X, dtype=np.float64) ** (m - 1)


def km_xstar(R, k0, m):
    """X* >= 0 solving P_X(X*)^2 X* = R (R >= 0), by bisection on ln X (the left side
    increases monotonically); X* = 0 where R = 0."""
    R = np.asarray(R, dtype=np.float64)
    out = np.zeros_like(R)
    pos = R > 0
    r = R[pos]
    lo = np.log(r) - 2.0 * np.log(km_px(r, k0, m)) - 1.0    # P_X(X) >= 1: X <= R
    hi = np.log(r) + 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        x = np.exp(mid)
        f = km_px(x, k0, m) ** 2 * x - r
        lo = np.where(f < 0, mid, lo)
        hi = np.where(f < 0, hi, mid)
    out[pos] = np.exp(0.5 * (lo + hi))
    return out


def eps_kmouflage(grad_phi_n, k0, m, lam):
    """eps = min(1, 1/P_X(X*)) (App. B) from |grad Phi_N| (h/Mpc)."""
    R = (lam * np.asarray(grad_phi_n, dtype=np.float64)) ** 2
    return np.minimum(1.0, 1.0 / km_px(km_xstar(R, k0, m), k0, m))


def km_mu(a, p):
    X = p.km_x0 * a ** p.km_xn
    return 1.0 + 2.0 * p.km_beta ** 2 / km_px(X, p.km_k0, p.km_m)


# ----------------------------------------------------------------------------- dispatch
class Model:
    """Model functions of a run (bound to its cosmology and model parameters)."""

    def __init__(self, p, force_lcdm_growth=False):
        self.p = p
        self.om = p.omega_m
        self.kind = p.model
        self.lcdm_growth = force_lcdm_growth or (p.growth_mode == 1)
        self.mb = MBetaTables(p) if p.model == MODEL_MBETA else None

    # --- linear growth inputs (App. B: the user supplies mu and gamma_2)
    def mu(self, k, a):
        k = np.asarray(k, dtype=np.float64)
        if self.lcdm_growth or self.kind == MODEL_LCDM:
            return np.ones_like(k)
        if self.kind == MODEL_FR:
            return fr_mu(k, a, self.om, self.p.fr0_abs)
        if self.kind == MODEL_NDGP:
            return np.full_like(k, dgp_mu(a, self.om, self.p.rc_h0))
        if self.kind == MODEL_SYMMETRON:
            return sym_mu(k, a, self.p)
        if self.kind == MODEL_MBETA:
            return self.mb.mu(k, a)
        if self.kind == MODEL_KMOUFLAGE:
            return np.full_like(k, km_mu(a, self.p))
        raise ValueError(self.kind)

    def gamma2_orth(self, k, a):
        k = np.asarray(k, dtype=np.float64)
        if self.lcdm_growth or self.kind == MODEL_LCDM:
            return np.zeros_like(k)
        if self.kind == MODEL_FR:
            kk = k / np.sqrt(2.0)
            return fr_gamma2E(k, kk, kk, a, self.om, self.p.fr0_abs)
        if self.kind == MODEL_NDGP:
            return np.full_like(k, dgp_gamma2E_orth(a, self.om, self.p.rc_h0))
        if self.kind == MODEL_SYMMETRON:
            kk = k / np.sqrt(2.0)
            return sym_gamma2E(k, kk, kk, a, self.p)
        if self.kind == MODEL_MBETA:
            kk = k / np.sqrt(2.0)
            return self.mb.gamma2E(k, kk, kk, a)
        if self.kind == MODEL_KMOUFLAGE:
            return np.zeros_like(k)
        raise ValueError(self.kind)

    # --- N-body field equation (Sec. 6, App. B)
    @property
    def has_fifth_force(self):
        return self.kind in (MODEL_FR, MODEL_NDGP, MODEL_SYMMETRON, MODEL_MBETA, MODEL_KMOUFLAGE)

    def a2m2(self, a):
        if self.kind == MODEL_FR:
            return float(fr_a2m2(a, self.om, self.p.fr0_abs))
        if self.kind == MODEL_SYMMETRON:
            return float(sym_a2m2(a, self.p))
        if self.kind == MODEL_MBETA:
            return float(self.mb.a2m2(a))
        return 0.0

    def coupling(self, a):
        """C(a): 1/3 for f(R) (Sec. 6.1), 1/(3 beta_DGP) for nDGP (Sec. 6.2), 2 beta^2(a)
        for the symmetron (App. C)."""
        if self.kind == MODEL_FR:
            return 1.0 / 3.0
        if self.kind == MODEL_NDGP:
            return float(1.0 / (3.0 * dgp_beta(a, self.om, self.p.rc_h0)))
        if self.kind == MODEL_SYMMETRON:
            return float(2.0 * sym_beta2(a, self.p))   # C = 2 beta^2 (App. B, C)
        if self.kind == MODEL_MBETA:
            return float(2.0 * self.mb.beta(a) ** 2)
        if self.kind == MODEL_KMOUFLAGE:
            return 2.0 * self.p.km_beta ** 2
        return 0.0

    def phi_crit(self, a):
        """Critical potential of potential screening (App. C): (3/2)|f_R(a)| for f(R), the
        App. C integral for the symmetron and for the tabulated {m, beta} model."""
        if self.kind == MODEL_FR:
            return 1.5 * float(fr_fR_abs(a, self.om, self.p.fr0_abs))
        if self.kind == MODEL_SYMMETRON:
            return sym_phi_crit(self.p)
        if self.kind == MODEL_MBETA:
            return self.mb.phi_crit(a)
        raise ValueError(self.kind)


# ----------------------------------------------------------------------------- screening
def eps_chameleon(phi_n, fR_abs):
    """eps = min(1, |3 f_R(a) / (2 Phi_N)|) (Sec. 6.1); eps = 1 where Phi_N = 0.
    phi_n is the dimensionless conventional Newtonian potential Phi/c^2."""
    phi_n = np.asarray(phi_n, dtype=np.float64)
    out = np.ones_like(phi_n)
    nz = phi_n != 0.0
    out[nz] = np.minimum(1.0, np.abs(1.5 * fR_abs / phi_n[nz]))
    return out


def eps_potential(phi_n, phi_crit):
    """eps = min(1, |Phi_crit/Phi_N|) (App. C); eps = 1 where Phi_N = 0."""
    phi_n = np.asarray(phi_n, dtype=np.float64)
    out = np.ones_like(phi_n)
    nz = phi_n != 0.0
    out[nz] = np.minimum(1.0, np.abs(phi_crit / phi_n[nz]))
    return out


def vainshtein_x(delta_bar, a, om, rc, beta, readings=0):
    """x = 8 (r_c H0)^2 Omega_m delta_bar / (9 beta^2 a^3) (Sec. 6.2), delta_bar the mean
    density contrast inside the radius (here the smoothed delta_R), clamped at -1.

    Reading: the spherical solution of the nDGP field equation (Sec. 6.2, eq.
    ndgpfieldeq) integrates r^2 x the equation to a quadratic in phi'/r whose source is
    kappa delta_bar / (9 beta): x is proportional to the mean overdensity, so the mean
    density is unscreened (eps = 1), and kappa = 1.5 Om a over the a^4 of the nonlinear
    term leaves a^-3.  The printed rho/rho_bar and the printed form without a^-3 are the
    READ_X_TOTAL_DENSITY and READ_X_NO_A3 readings.  For delta_bar >= -1, x > -8/9 (beta^2
    a^3 > (r_c H0)^2 Om), so 1 + x > 0.  Pinned by the numerical radial solution of the
    field equation for top-hat over- and underdensities."""
    d = np.maximum(-1.0, np.asarray(delta_bar, dtype=np.float64))
    y = d + 1.0 if readings & READ_X_TOTAL_DENSITY else d
    a3 = 1.0 if readings & READ_X_NO_A3 else a ** 3
    return 8.0 * rc * rc * om * y / (9.0 * beta * beta * a3)


def eps_vainshtein(x):
    """eps = 2 (sqrt(1+x) - 1)/x = 2/(1 + sqrt(1+x)) (Sec. 6.2, read so that eps -> 1
    as x -> 0 and eps -> 2/sqrt(x) deep inside the Vainshtein radius; x in (-1, 0) in
    underdense regions gives eps > 1)."""
    return 2.0 / (1.0 + np.sqrt(1.0 + np.asarray(x, dtype=np.float64)))


def window(kR, kind):
    """Fourier-space smoothing windows offered for the density screening (App. B):
    Gaussian exp(-(kR)^2/2), spherical top-hat 3 (sin x - x cos x)/x^3, sharp-k
    Theta(1 - kR)."""
    x = np.asarray(kR, dtype=np.float64)
    if kind == FILTER_GAUSS:
        return np.exp(-0.5 * x * x)
    if kind == FILTER_TOPHAT:
        out = np.ones_like(x)
        nz = x > 1e-4
        xs = x[nz]
        out[nz] = 3.0 * (np.sin(xs) - xs * np.cos(xs)) / xs ** 3
        small = ~nz
        out[small] = 1.0 - x[small] ** 2 / 10.0
        return out
    if kind == FILTER_SHARPK:
        return (x <= 1.0).astype(np.float64)
    raise ValueError(kind)
