"""Shell-averaged matter power spectrum of the particles (the analysis output of
Sec. 8; the estimator's details are this reading, the paper gives none).

delta from CIC assignment on the PM mesh, DFT, then for shell b = floor(|nu| + 1/2)
(|nu|^2 is an integer, so no mode sits on a shell edge):
  P_b = < L^3 |delta_k|^2 / (M^2 W_CIC(k)^2) >,  W_CIC = prod_i sinc^2(pi nu_i / n)
  k_b = < |k| >,
averaged over the modes of the half-complex grid with weight 2 for 0 < nu_z < n/2
and 1 otherwise (so each +-k pair is counted twice, the self-conjugate planes once).
Shot noise is not subtracted.  Bins 0 .. nbins-1.
"""

import numpy as np

from . import fftlib

from .lpt import kvec
from .pm import density_contrast


def shell_index(n2):
    """b = floor(sqrt(n2) + 1/2) computed exactly for integer n2."""
    b = np.floor(np.sqrt(n2.astype(np.float64)) + 0.5).astype(np.int64)
    # exact correction: b^2 - b < n2 <= b^2 + b
    b = np.where((b > 0) & (b * b - b >= n2), b - 1, b)
    b = np.where(n2 > b * b + b, b + 1, b)
    return b


def power_spectrum_mesh(delta, L, nbins):
    n = delta.shape[0]
    M = n ** 3
    dk = fftlib.rfftn(delta)
    (kx, ky, kz), (nx, ny, nz) = kvec(n, L)
    n2 = np.broadcast_to(nx * nx + ny * ny + nz * nz, dk.shape)
    kmag = np.sqrt(np.broadcast_to(kx * kx + ky * ky + kz * kz, dk.shape))
    W = (np.sinc(nx / n) * np.sinc(ny / n) * np.sinc(nz / n)) ** 2
    P = L ** 3 * np.abs(dk) ** 2 / (M * M * np.broadcast_to(W, dk.shape) ** 2)
    wt = np.broadcast_to(np.where((nz > 0) & (nz < n // 2), 2.0, 1.0), dk.shape)
    b = shell_index(n2)
    sel = b < nbins
    nm = np.bincount(b[sel], weights=wt[sel], minlength=nbins)
    ps = np.bincount(b[sel], weights=(wt * P)[sel], minlength=nbins)
    ks = np.bincount(b[sel], weights=(wt * kmag)[sel], minlength=nbins)
    with np.errstate(invalid="ignore", divide="ignore"):
        return ks / nm, ps / nm, nm


def power_spectrum(u, p, nbins=None):
    nbins = p.nmesh1d // 2 if nbins is None else nbins
    delta, _ = density_contrast(u, p)
    return power_spectrum_mesh(delta, p.box, nbins)
