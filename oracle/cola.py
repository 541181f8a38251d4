"""COLA time stepping about the LPT path (Sec. 2; App. A).

With x = q + u, u = Psi_LPT(q, a) + delta_x, the residual obeys
  d delta_v / dtau = -grad Phi - d^2 x_LPT / dtau^2,  d delta_x / dtau = delta_v  (Sec. 2)
and is integrated with a kick-drift leapfrog (the paper names only "a Leapfrog
integrator"; spacing and coefficients are this reading):

* a_i = a_ini + i (1 - a_ini)/n, i = 0..n (uniform in a);
* positions live at a_i, residual velocities at a_{i+1/2} = (a_i + a_{i+1})/2, with
  a_{-1/2} = a_0 and v = 0 at a_0 (particles start on the LPT path);
* step i: F = PM force at x(a_i);
    v <- v + [tau(a_{i+1/2}) - tau(a_{i-1/2})] (F - L''(q, a_i));
    u <- u + [tau(a_{i+1}) - tau(a_i)] v + [Psi_LPT(q, a_{i+1}) - Psi_LPT(q, a_i)];
* L'' = d^2 Psi_LPT/dtau^2 = D1'' Psi1 + D2'' Psi2 per mode, with D'' from the growth ODE.

u is the displacement from the Lagrangian grid point and is never wrapped; the
periodic wrap is applied only where positions meet the mesh.
"""

import numpy as np

from .background import tau_between
from .growth import growth_table, distinct_n2
from .lpt import initial_fields, lpt_field_scale_dependent
from .models import Model
from .pm import pm_force, positions_in_cells
from .spectrum import InitialSpectrum


def time_grid(p):
    n = p.n_steps
    a = p.a_ini + np.arange(n + 1) * (1.0 - p.a_ini) / n
    ah = 0.5 * (a[:-1] + a[1:])
    kick = np.empty(n)
    drift = np.empty(n)
    for i in range(n):
        a_lo = a[0] if i == 0 else ah[i - 1]
        kick[i] = tau_between(a_lo, ah[i], p.omega_m)
        drift[i] = tau_between(a[i], a[i + 1], p.omega_m)
    return a, kick, drift


class Run:
    """A COLA run of the oracle: initial conditions, growth tables, state, steps."""

    def __init__(self, p, noise=None, lpt=None, kspace_lpt=False):
        """kspace_lpt forces the scale-dependent (Fourier-space) LPT synthesis even when
        the growth factors do not depend on k (the LCDM-limit check of Sec. 7)."""
        self.p = p
        self.model = Model(p)
        self.a, self.dtau_kick, self.dtau_drift = time_grid(p)
        self.G, self.kdep = growth_table(p, self.model, self.a)
        if kspace_lpt and not self.kdep:
            self.G = np.repeat(self.G, distinct_n2(p.np1d).size, axis=1)
            self.kdep = True
        if lpt is None:
            self.spec = InitialSpectrum(p)
            lpt = initial_fields(p, self.spec, noise)
        self.lpt = lpt
        N = p.n_part
        self.psi1 = lpt["psi1"].reshape(3, N)
        self.psi2 = lpt["psi2"].reshape(3, N)
        self.u = self.lpt_displacement(self.G[0, :, 0], self.G[0, :, 3])
        self.v = np.zeros((3, N))
        self.next_step = 0

    def lpt_displacement(self, X1, X2):
        """IDFT[i k (X1 phi1_k + X2 phi2_k)] at the particles, (3, N).  For k-independent
        coefficients this is X1 Psi1 + X2 Psi2 (standard COLA)."""
        if self.kdep:
            f = lpt_field_scale_dependent(self.lpt["phi1_k"], self.lpt["phi2_k"], X1, X2,
                                          self.p.np1d, self.p.box, lambda n2: n2)
            return f.reshape(3, -1)
        return X1[0] * self.psi1 + X2[0] * self.psi2

    def step(self, i=None):
        i = self.next_step if i is None else i
        if i != self.next_step or i >= self.p.n_steps:
            raise ValueError("step out of order")
        G0, G1 = self.G[i], self.G[i + 1]
        F, _ = pm_force(self.u, self.p, self.a[i], self.model)
        Lpp = self.lpt_displacement(G0[:, 2], G0[:, 5])
        self.v = self.v + self.dtau_kick[i] * (F - Lpp)
        dlt = self.lpt_displacement(G1[:, 0] - G0[:, 0], G1[:, 3] - G0[:, 3])
        self.u = self.u + self.dtau_drift[i] * self.v + dlt
        self.next_step += 1

    def run(self, n=None):
        n = self.p.n_steps if n is None else n
        while self.next_step < n:
            self.step()
        return self

    def positions(self):
        """Wrapped comoving positions x = (q + u) mod L, (3, N)."""
        return np.mod(positions_in_cells(self.u, self.p) * self.p.cell, self.p.box)
