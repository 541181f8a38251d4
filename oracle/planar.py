"""Planar reduction of the PM force and of one COLA step (Secs. 2, 6), for checking the
full-size mesh.

THIS MODULE IS TEST INFRASTRUCTURE (see the package header).

Take particles that keep their lattice position on two axes and move along the third by a
displacement that depends only on their lattice index along that axis.  Also take a mesh
with one or two nodes per particle spacing.  The CIC weights of the unmoved lattice
coordinates then cover every node of those axes equally (weights 1/2, 1/2 from the
half-cell lattice offset), so the deposited density depends on the moving axis alone.
Every Fourier-space field of the PM step follows: delta_k, the smoothed density or
Newtonian potential of the screening step, S_k and the Green's function are all non-zero
only on that axis of k-space.  The three 3D transforms reduce to 1D transforms along it,
the force has no component across it, and its component along it depends on that
coordinate alone.

planar_pm computes these 1D profiles with the same operators as pm.force_mesh, on
n_mesh points.  A full-size mesh can thus be checked cell by cell against an FP64
computation that takes milliseconds.  planar_step does the same for one COLA step of
Run.step with k-independent growth.  Both are pinned against the 3D oracle on small meshes
in tests/test_oracle_pm.py and tests/test_oracle_cola.py.
"""

import numpy as np

from .background import kappa
from .cola import time_grid
from .growth import growth_table
from .models import (Model, eps_chameleon, eps_potential, eps_vainshtein, vainshtein_x, window,
                     fr_fR_abs, dgp_beta)
from .params import MODEL_FR, MODEL_NDGP, MODEL_SYMMETRON, MODEL_MBETA, H0_OVER_C


def _cic_1d(s, n):
    fl = np.floor(s)
    d = s - fl
    i0 = np.mod(fl.astype(np.int64), n)
    return i0, np.mod(i0 + 1, n), d


def planar_pm(u1, p, a, model=None):
    """PM force of the planar configuration with per-plane displacements u1 (n_p,), Mpc/h.

    Returns dict with the mesh profiles along the moving axis: rho (= 1 + delta), src
    (the screened source S) and force (the force component along the axis), each (n,);
    and per particle plane: s (position in cells, unwrapped) and fp (the CIC-gathered
    force), each (n_p,)."""
    model = model or Model(p)
    n, n_p, L = p.nmesh1d, p.np1d, p.box
    r = n // n_p
    if r * n_p != n or r not in (1, 2):
        raise ValueError("the planar reduction needs n_mesh = n_p or 2 n_p")
    s = np.arange(n_p) * r + 0.5 + np.asarray(u1, dtype=np.float64) / p.cell
    i0, i1, d = _cic_1d(s, n)
    # mass r^3 per particle, spread 1/r over the nodes of each unmoved axis
    rho = r * (np.bincount(i0, weights=1.0 - d, minlength=n) + np.bincount(i1, weights=d, minlength=n))
    delta = rho - 1.0
    nu = np.rint(np.fft.fftfreq(n) * n)
    k = 2.0 * np.pi / L * nu
    k2 = k * k
    inv_k2 = np.zeros(n)
    inv_k2[k2 > 0] = 1.0 / k2[k2 > 0]
    dk = np.fft.fft(delta)
    kap = kappa(a, p.omega_m)
    tot_k = -kap * dk * inv_k2
    S = delta
    if model.has_fifth_force:
        if p.screening:
            if p.model in (MODEL_FR, MODEL_SYMMETRON, MODEL_MBETA):
                phi_n = np.fft.ifft(-kap * dk * inv_k2).real * H0_OVER_C ** 2 / (a * a)
                if p.model == MODEL_FR:
                    eps = eps_chameleon(phi_n, fr_fR_abs(a, p.omega_m, p.fr0_abs))
                else:
                    eps = eps_potential(phi_n, model.phi_crit(a))
            elif p.model == MODEL_NDGP:
                dR = np.fft.ifft(dk * window(np.abs(k) * p.r_smooth, p.filter)).real
                beta = dgp_beta(a, p.omega_m, p.rc_h0)
                eps = eps_vainshtein(vainshtein_x(dR, a, p.omega_m, p.rc_h0, beta, p.readings))
            else:
                raise ValueError(p.model)
            S = delta * eps
        g5 = np.zeros(n)
        g5[k2 > 0] = -model.coupling(a) * kap / (k2[k2 > 0] + model.a2m2(a))
        tot_k = tot_k + g5 * np.fft.fft(S)
    grad = 1j * k * (nu != -(n // 2))        # i k, zero on the Nyquist mode
    force = np.fft.ifft(-grad * tot_k).real
    fp = (1.0 - d) * force[i0] + d * force[i1]
    return dict(rho=rho, src=S, force=force, s=s, fp=fp)


def planar_step(u1, v1, psi1, psi2, p, i, model=None):
    """Step i of Run.step (kick-drift about the LPT path) for the planar configuration:
    u1, v1, psi1, psi2 are the components along the moving axis per particle plane
    (n_p,).  Needs growth factors that do not depend on k.  Returns (u1, v1) after the
    step."""
    model = model or Model(p)
    a, dtk, dtd = time_grid(p)
    G, kdep = growth_table(p, model, a)
    if kdep:
        raise ValueError("planar_step needs k-independent growth factors")
    g0, g1 = G[i, 0], G[i + 1, 0]
    F = planar_pm(u1, p, a[i], model)["fp"]
    v = v1 + dtk[i] * (F - (g0[2] * psi1 + g0[5] * psi2))
    u = u1 + dtd[i] * v + (g1[0] - g0[0]) * psi1 + (g1[3] - g0[3]) * psi2
    return u, v
