"""Lagrangian perturbation theory fields (Secs. 3-4, App. A).

Conventions (the paper fixes none of them):
* DFT: forward unnormalised with e^{-i k.x}; inverse carries 1/n^3 (numpy rfftn/irfftn).
* nu_i in [-n/2, n/2 - 1] along x and y, nu_z in [0, n/2] (half-complex), k = 2 pi nu / L.
* An odd derivative factor i k_i is set to zero on the axis-i Nyquist plane
  (nu_i = -n/2, or nu_z = n/2), as is a mixed factor k_i k_j (i != j) when either axis
  is at Nyquist; this keeps every inverse transform Hermitian.

Potentials (Sec. 3):
* 1LPT: nabla_q^2 phi1 = -delta_ini, so phi1_k = delta_k / k^2; Psi1 = grad_q phi1.
* 2LPT: nabla_q^2 phi2 = (1/2)[(nabla^2 phi1)^2 - (d_i d_j phi1)^2]
        = phi11 phi22 + phi11 phi33 + phi22 phi33 - phi12^2 - phi13^2 - phi23^2
  (eq. lcdm2lpt), so phi2_k = -S_k / k^2; Psi2 = grad_q phi2.
* Scale-dependent growth (Secs. 4.1-4.2): Psi(q, a) = IDFT[i k (D1(k,a) phi1_k +
  D2(k,a) phi2_k)], recomputed by Fourier transform whenever it is needed (App. A).
"""

import numpy as np

from . import fftlib

from .rng import white_noise


def freq(n):
    """Integer frequencies nu in FFT order for a full axis (x, y) and the half axis (z)."""
    full = np.fft.fftfreq(n, d=1.0 / n).astype(np.int64)
    half = np.arange(n // 2 + 1, dtype=np.int64)
    return full, half


def kvec(n, L):
    """Broadcastable wavevector components (kx, ky, kz) and integer frequency arrays."""
    full, half = freq(n)
    nx = full[:, None, None]
    ny = full[None, :, None]
    nz = half[None, None, :]
    f = 2.0 * np.pi / L
    return (f * nx, f * ny, f * nz), (nx, ny, nz)


def nyquist_masks(n):
    """Boolean masks (broadcastable) of the Nyquist plane of each axis."""
    _, (nx, ny, nz) = kvec(n, 1.0)
    return nx == -n // 2, ny == -n // 2, nz == n // 2


def n2_grid(n):
    _, (nx, ny, nz) = kvec(n, 1.0)
    return nx * nx + ny * ny + nz * nz


def grad_factor(n, L, axis):
    """i k_axis with the Nyquist plane of that axis zeroed (odd derivative)."""
    (kx, ky, kz), _ = kvec(n, L)
    k = (kx, ky, kz)[axis]
    nyq = nyquist_masks(n)[axis]
    return 1j * np.where(nyq, 0.0, k)


def hessian_factor(n, L, i, j):
    """-k_i k_j (the transform of d_i d_j), mixed terms zeroed on either Nyquist plane."""
    (kx, ky, kz), _ = kvec(n, L)
    k = (kx, ky, kz)
    f = -k[i] * k[j]
    if i != j:
        nyq = nyquist_masks(n)
        f = np.where(nyq[i] | nyq[j], 0.0, f)
    return f


def inv_laplacian(n, L):
    """1/k^2 with the k = 0 mode set to 0."""
    (kx, ky, kz), _ = kvec(n, L)
    k2 = kx * kx + ky * ky + kz * kz
    out = np.zeros(np.broadcast(kx, ky, kz).shape)
    nz = k2 > 0
    out[nz] = 1.0 / k2[nz]
    return out


def delta_k_from_noise(w, p, spec):
    """delta_k = W_k sqrt(N P_ini(|k|) / L^3), W = DFT(white noise); delta_0 = 0.
    With <|W_k|^2> = N this gives <|delta_k|^2> = N^2 P / L^3, the DFT of a field of
    power spectrum P sampled at N points."""
    n = p.np1d
    N = n ** 3
    Wk = fftlib.rfftn(w)
    (kx, ky, kz), _ = kvec(n, p.box)
    k = np.sqrt(kx * kx + ky * ky + kz * kz)
    amp = np.zeros(k.shape)
    nz = k > 0
    amp[nz] = np.sqrt(N * spec.P_ini(k[nz]) / p.box ** 3)
    return Wk * amp


def phi1_from_delta_k(dk, n, L):
    return dk * inv_laplacian(n, L)


def twolpt_source(phi1_k, n, L):
    """S(q) = phi11 phi22 + phi11 phi33 + phi22 phi33 - phi12^2 - phi13^2 - phi23^2,
    from the six second derivatives of phi1 taken in Fourier space (eq. lcdm2lpt)."""
    d = {}
    for i in range(3):
        for j in range(i, 3):
            d[i, j] = fftlib.irfftn(phi1_k * hessian_factor(n, L, i, j), n)
    return (d[0, 0] * d[1, 1] + d[0, 0] * d[2, 2] + d[1, 1] * d[2, 2]
            - d[0, 1] ** 2 - d[0, 2] ** 2 - d[1, 2] ** 2)


def phi2_from_phi1(phi1_k, n, L):
    S = twolpt_source(phi1_k, n, L)
    return -fftlib.rfftn(S) * inv_laplacian(n, L)


def displacement(phi_k, n, L):
    """Psi = grad_q phi, returned as (3, n, n, n) real arrays."""
    return np.stack([fftlib.irfftn(phi_k * grad_factor(n, L, ax), n)
                     for ax in range(3)])


def lpt_field_scale_dependent(phi1_k, phi2_k, X1, X2, n, L, n2_index):
    """IDFT[i k (X1(k) phi1_k + X2(k) phi2_k)] for per-|nu|^2 coefficient tables X1, X2
    (App. A: multiply the stored k-space fields by growth factors, transform back)."""
    n2 = n2_grid(n)
    c = X1[n2_index(n2)] * phi1_k + X2[n2_index(n2)] * phi2_k
    return displacement(c, n, L)


def lpt_field_sparse(modes, n, L, planes):
    """IDFT[i k (X1 phi1_k + X2 phi2_k)] of a field whose half-complex coefficients are zero
    except at the listed modes, by direct summation at the grid points of the x-planes
    `planes` (App. A's transform, evaluated mode by mode).

    modes: ((nu_x, nu_y, nu_z), c) with c = X1 phi1_k + X2 phi2_k at that mode,
    nu_x, nu_y in [-n/2, n/2 - 1] and 0 < nu_z < n/2, so each stored mode and its implicit
    conjugate partner at -nu give (1/N) (c e^{i k.q} + conj) = (2/N) Re(c e^{i k.q});
    i k_c is zero on the axis-c Nyquist plane (nu_c = -n/2).  q = L i / n at grid index i.
    Returns (3, len(planes), n, n)."""
    planes = np.asarray(planes)
    N = n ** 3
    out = np.zeros((3, planes.size, n, n))
    idx = np.arange(n)
    for (nu, c) in modes:
        nu = np.asarray(nu, dtype=np.int64)
        assert 0 < nu[2] < n // 2 and all(-n // 2 <= v < n // 2 for v in nu[:2])
        ex = np.exp(2j * np.pi * nu[0] * planes / n)
        ey = np.exp(2j * np.pi * nu[1] * idx / n)
        ez = np.exp(2j * np.pi * nu[2] * idx / n)
        ph = ex[:, None, None] * ey[None, :, None] * ez[None, None, :]
        for ax in range(3):
            if nu[ax] == -n // 2:
                continue
            k = 2.0 * np.pi * nu[ax] / L
            out[ax] += (2.0 / N) * np.real(1j * k * c * ph)
    return out


def initial_fields(p, spec, noise=None):
    """The initial potentials phi1_k, phi2_k on the particle grid (Np^3, half-complex),
    and the displacements Psi1, Psi2 at the grid points (3, n, n, n)."""
    n = p.np1d
    L = p.box
    w = white_noise(p.seed, n) if noise is None else noise
    dk = delta_k_from_noise(w, p, spec)
    phi1_k = phi1_from_delta_k(dk, n, L)
    phi2_k = phi2_from_phi1(phi1_k, n, L)
    return dict(delta_k=dk, phi1_k=phi1_k, phi2_k=phi2_k,
                psi1=displacement(phi1_k, n, L), psi2=displacement(phi2_k, n, L))
