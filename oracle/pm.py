"""Particle-mesh force with the screened fifth force (Secs. 2 and 6, App. B).

Steps, in the paper's order:
1. density contrast delta from the particle positions (Sec. 2): cloud-in-cell
   assignment on a vertex-centred mesh (node j at j * cell), particle mass M/N so that
   rho averages to 1, delta = rho - 1; Lagrangian points at cell centres;
2. Newtonian potential nabla^2 Phi_N = kappa delta (Sec. 2, eq. nbody):
   Phi_k = -kappa delta_k / k^2, Phi_0 = 0;
3. screening factor in real space (Sec. 6):
   * f(R): Phi_N/c^2 = Phi (H0/c)^2 / a^2 (the code potential is a^2 times the
     conventional one), eps = min(1, |3 f_R(a) / (2 Phi_N)|) (Sec. 6.1);
   * nDGP: delta_R = density smoothed with W(kR) (Gaussian by default),
     x = 8 (r_c H0)^2 Om delta_R / (9 beta^2 a^3), eps = 2/(1 + sqrt(1 + x)) (Sec. 6.2);
   screened source S = delta * eps (S = delta when screening is off);
4. linear field equation nabla^2 phi = a^2 m^2 phi + C kappa S (Sec. 6, App. B):
   phi_k = -C kappa S_k / (k^2 + a^2 m^2), phi_0 = 0;
5. force F = -grad(Phi_N + phi) (the total force of Sec. 6.1), F_k = -i k (Phi_k + phi_k)
   with i k_i zeroed on the axis-i Nyquist plane, three inverse transforms;
6. force at the particles by CIC interpolation with the same weights as step 1.
"""

import numpy as np

from . import fftlib

from .background import kappa
from .lpt import grad_factor, inv_laplacian, kvec
from .models import (Model, eps_chameleon, eps_potential, eps_vainshtein, eps_kmouflage,
                     vainshtein_x, window,
                     fr_fR_abs, dgp_beta)
from .params import MODEL_FR, MODEL_NDGP, MODEL_SYMMETRON, MODEL_MBETA, MODEL_KMOUFLAGE, H0_OVER_C


def lagrangian_index(n_p):
    """(ix, iy, iz) of particles stored in row-major Lagrangian order."""
    idx = np.arange(n_p ** 3, dtype=np.int64)
    return idx // (n_p * n_p), (idx // n_p) % n_p, idx % n_p


def positions_in_cells(u, p):
    """s = x / cell = ix * (n_m / n_p) + 1/2 + u / cell, shape (3, N), unwrapped.

    u is the displacement from the Lagrangian grid point q = ix L / n_p + cell / 2.
    The half-cell offset places every unperturbed particle at a cell centre of the PM
    mesh (the paper fixes no convention): the undisplaced lattice then deposits a
    uniform density when n_m = n_p or 2 n_p, and no particle starts on the kink of
    the CIC kernel, which keeps the force linear in small displacements."""
    ix = lagrangian_index(p.np1d)
    ratio = p.nmesh1d / p.np1d
    return np.stack([ix[c] * ratio + 0.5 + np.asarray(u[c], dtype=np.float64) / p.cell
                     for c in range(3)])


def _cic_corners(s, n):
    """Yield (flat index, weight) for the 8 CIC corners of positions s (3, N)."""
    fl = np.floor(s)
    d = s - fl
    i0 = np.mod(fl.astype(np.int64), n)
    i1 = np.mod(i0 + 1, n)
    for ox in (0, 1):
        wx = d[0] if ox else 1.0 - d[0]
        ix = i1[0] if ox else i0[0]
        for oy in (0, 1):
            wy = d[1] if oy else 1.0 - d[1]
            iy = i1[1] if oy else i0[1]
            for oz in (0, 1):
                wz = d[2] if oz else 1.0 - d[2]
                iz = i1[2] if oz else i0[2]
                yield (ix * n + iy) * n + iz, wx * wy * wz


def cic_deposit(s, n, mass):
    """rho_j = sum_p mass * W(x_p - x_j), returned as (n, n, n) float64."""
    rho = np.zeros(n ** 3)
    for flat, w in _cic_corners(s, n):
        rho += np.bincount(flat, weights=mass * w, minlength=n ** 3)
    return rho.reshape(n, n, n)


def cic_gather(fields, s, n):
    """Interpolate mesh fields (C, n, n, n) to positions s (3, N) with CIC weights."""
    flatf = [f.reshape(-1) for f in fields]
    out = np.zeros((len(fields), s.shape[1]))
    for flat, w in _cic_corners(s, n):
        for c, f in enumerate(flatf):
            out[c] += w * f[flat]
    return out


def density_contrast(u, p):
    s = positions_in_cells(u, p)
    rho = cic_deposit(s, p.nmesh1d, p.n_cells / p.n_part)
    return rho - 1.0, s


def screened_source(delta, delta_k, p, a, model):
    """S = delta * eps_screen in real space (Sec. 6); S = delta when screening is off."""
    n, L = p.nmesh1d, p.box
    if not p.screening or not model.has_fifth_force:
        return delta.copy()
    if p.model in (MODEL_FR, MODEL_SYMMETRON, MODEL_MBETA):
        Phi = fftlib.irfftn(-kappa(a, p.omega_m) * delta_k * inv_laplacian(n, L), n)
        phi_n = Phi * H0_OVER_C ** 2 / (a * a)
        if p.model == MODEL_FR:
            eps = eps_chameleon(phi_n, fr_fR_abs(a, p.omega_m, p.fr0_abs))
        else:
            eps = eps_potential(phi_n, model.phi_crit(a))
    elif p.model == MODEL_KMOUFLAGE:
        # gradient screening (App. B): |grad Phi_N| of the dimensionless Newtonian potential
        Phi_k = -kappa(a, p.omega_m) * delta_k * inv_laplacian(n, L)
        g2 = sum(fftlib.irfftn(grad_factor(n, L, ax) * Phi_k, n) ** 2 for ax in range(3))
        eps = eps_kmouflage(np.sqrt(g2) * H0_OVER_C ** 2 / (a * a), p.km_k0, p.km_m, p.km_lambda)
    elif p.model == MODEL_NDGP:
        (kx, ky, kz), _ = kvec(n, L)
        k = np.sqrt(kx * kx + ky * ky + kz * kz)
        dR = fftlib.irfftn(delta_k * window(k * p.r_smooth, p.filter), n)
        beta = dgp_beta(a, p.omega_m, p.rc_h0)
        eps = eps_vainshtein(vainshtein_x(dR, a, p.omega_m, p.rc_h0, beta, p.readings))
    else:
        raise ValueError(p.model)
    return delta * eps


def force_mesh(delta, p, a, model=None):
    """Force meshes F (3, n, n, n) = -grad(Phi_N + phi) from a density contrast mesh,
    plus the screened source S."""
    model = model or Model(p)
    n, L = p.nmesh1d, p.box
    dk = fftlib.rfftn(delta)
    inv_k2 = inv_laplacian(n, L)
    kap = kappa(a, p.omega_m)
    tot_k = -kap * dk * inv_k2
    S = delta
    if model.has_fifth_force:
        S = screened_source(delta, dk, p, a, model)
        Sk = fftlib.rfftn(S)
        (kx, ky, kz), _ = kvec(n, L)
        k2 = kx * kx + ky * ky + kz * kz
        den = k2 + model.a2m2(a)
        g5 = np.zeros(den.shape)
        nz = k2 > 0
        g5[nz] = -model.coupling(a) * kap / den[nz]
        tot_k = tot_k + g5 * Sk
    F = np.stack([fftlib.irfftn(-grad_factor(n, L, ax) * tot_k, n)
                  for ax in range(3)])
    return F, S


def pm_force(u, p, a, model=None):
    """Per-particle PM force at scale factor a for displacements u (3, N).
    Returns (F_p (3, N), meshes dict with rho = 1 + delta, src = S, force (3, n, n, n))."""
    model = model or Model(p)
    delta, s = density_contrast(u, p)
    F, S = force_mesh(delta, p, a, model)
    Fp = cic_gather(F, s, p.nmesh1d)
    return Fp, dict(rho=delta + 1.0, src=S, force=F)
