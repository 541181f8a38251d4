"""The discrete Fourier transforms the oracle uses as library steps: scipy's pocketfft,
forward unnormalised with e^{-ikx}, inverse with 1/M.  The host timing of the oracle may
raise the thread count; the transform computed is the same for any count."""

import scipy.fft as _sf

_workers = 1


def set_workers(n):
    """Threads each transform may use (1 = serial, the default)."""
    global _workers
    _workers = max(1, int(n))


def workers():
    return _workers


def rfftn(x):
    return _sf.rfftn(x, workers=_workers)


def irfftn(xk, n):
    return _sf.irfftn(xk, s=(n, n, n), axes=(0, 1, 2), workers=_workers)
