"""Run parameters and unit conventions of the oracle.

Units (a reading of Sec. 2, where kappa = 4 pi G rho_bar a^4 = (3/2) Omega_m H0^2 a and
d tau = dt / a^2):

* lengths in Mpc/h, wavenumbers in h/Mpc;
* time in units of 1/H0, so H(a) = E(a) and kappa(a) = 1.5 Omega_m a;
* wherever H0 multiplies a length (m(a), Pi(k,a), k/(aH), the Newtonian
  potential compared with f_R), H0 is converted with H0/c = 1/2997.92458 h/Mpc.
"""

from dataclasses import dataclass, replace

MODEL_LCDM = 0
MODEL_FR = 1      # Hu-Sawicki f(R), n = 1 (Sec. 5.1)
MODEL_NDGP = 2    # normal-branch DGP (Sec. 5.2)
MODEL_SYMMETRON = 3   # symmetron, a {m(a), beta(a)} model with potential screening (App. C)
MODEL_MBETA = 4       # general {m(a), beta(a)} model given as tables (App. C)
MODEL_KMOUFLAGE = 5   # k-Mouflage: gradient screening (App. B)
MBETA_MAX_KNOTS = 64

FILTER_GAUSS = 0
FILTER_TOPHAT = 1
FILTER_SHARPK = 2

# Alternative readings of passages the paper leaves ambiguous (bit flags of Params.readings;
# the default 0 takes the readings stated in the module docstrings):
READ_X_TOTAL_DENSITY = 1   # Vainshtein x from rho/rho_bar = 1 + delta_R, as printed (Sec. 6.2),
                           # instead of the mean overdensity delta_R that the field equation gives
READ_X_NO_A3 = 2           # Vainshtein x without the a^-3 of the physical mean density
READ_D2_HALF_K = 4         # second-order growth source D1(k/sqrt2, a)^2, the k1 = k2 = k/sqrt2
                           # argument of gamma_2, instead of the printed D1(k, a)^2 (Sec. 4.2)
READ_ALL = READ_X_TOTAL_DENSITY | READ_X_NO_A3 | READ_D2_HALF_K

H0_OVER_C = 1.0 / 2997.92458   # h/Mpc


@dataclass(frozen=True)
class Params:
    omega_m: float = 0.3
    omega_b: float = 0.05
    h: float = 0.7
    n_s: float = 0.96
    sigma8: float = 0.8
    t_cmb: float = 2.7255
    model: int = MODEL_LCDM
    fr0_abs: float = 1e-5
    rc_h0: float = 1.0
    sym_beta: float = 1.0         # beta_* of the symmetron (App. C)
    sym_mass: float = 2997.92458  # m_*/H0 (m_* = 1 h/Mpc: a 1 Mpc/h range)
    sym_astar: float = 0.5        # a_*: beta = m = 0 before it
    # general {m(a), beta(a)} model: beta and m^2/H0^2 at knots ln a (ascending, 4 to 64
    # knots spanning [a_ini, 1]); both sides interpolate with natural cubic splines of
    # beta and of ln(m^2/H0^2) in ln a
    mb_lna: tuple = ()
    mb_beta: tuple = ()
    mb_m2: tuple = ()
    # k-Mouflage (App. B) with the kinetic function P(X) = -1 + X + K0 X^m: coupling beta,
    # K0 and m, the scale lambda (Mpc/h) of P_X(X*)^2 X* = (lambda |grad Phi_N|)^2 with
    # Phi_N the dimensionless Newtonian potential, and the cosmological X(a) = x0 a^xn
    km_beta: float = 0.5
    km_k0: float = 1.0
    km_m: int = 3
    km_lambda: float = 1e6
    km_x0: float = 0.0
    km_xn: float = 0.0
    screening: int = 1
    filter: int = FILTER_GAUSS
    r_smooth: float = 1.0
    growth_mode: int = 0          # 0: true D(k,a) of the model; 1: LCDM growth factors
    np1d: int = 32
    nmesh1d: int = 64
    box: float = 200.0
    z_init: float = 19.0
    n_steps: int = 10
    seed: int = 1
    readings: int = 0             # bit flags READ_* above

    @property
    def a_ini(self):
        return 1.0 / (1.0 + self.z_init)

    @property
    def n_part(self):
        return self.np1d ** 3

    @property
    def n_cells(self):
        return self.nmesh1d ** 3

    @property
    def cell(self):
        return self.box / self.nmesh1d

    @property
    def scale_dependent(self):
        """True when the LPT growth factors depend on k (Sec. 4): f(R), the symmetron and
        the general {m, beta} model run with their own growth factors.  LCDM and nDGP have
        k-independent D1, D2 (Sec. 5.2), and growth_mode 1 forces the LCDM factors
        (Sec. 7.1)."""
        return self.model in (MODEL_FR, MODEL_SYMMETRON, MODEL_MBETA) and self.growth_mode == 0

    def with_(self, **kw):
        return replace(self, **kw)


def is_2a3b(n):
    if n < 2 or n % 2:
        return False
    while n % 2 == 0:
        n //= 2
    while n % 3 == 0:
        n //= 3
    return n == 1
