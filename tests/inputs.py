"""Seeded synthetic inputs shared by the GPU path and the oracle in tests.

Only random-number plumbing lives here (no step of the method's arithmetic): particle
displacement fields with a chosen rms and optional clustering, as float32 so that both
sides start from bit-identical values.
"""

import numpy as np


def displacements(np1d, box, rms_cells, nmesh1d, seed, clustered=False):
    """u (3, N) float32 in Mpc/h.  Gaussian, rms `rms_cells` mesh cells per axis; with
    `clustered`, a quarter of the particles are pulled onto a few random centres so that
    many particles share cells (the z = 0 regime of the deposit)."""
    rng = np.random.default_rng(seed)
    N = np1d ** 3
    cell = box / nmesh1d
    u = rng.normal(0.0, rms_cells * cell, size=(3, N))
    if clustered:
        idx = np.arange(N)
        ix, iy, iz = idx // (np1d * np1d), (idx // np1d) % np1d, idx % np1d
        q = np.stack([ix, iy, iz]) * (box / np1d) + 0.5 * cell
        centres = rng.uniform(0, box, size=(3, 4))
        pick = rng.random(N) < 0.25
        which = rng.integers(0, 4, size=N)
        target = centres[:, which] + rng.normal(0, 0.3 * cell, size=(3, N))
        d = target - q
        d -= box * np.round(d / box)          # shortest periodic displacement
        u[:, pick] = d[:, pick]
    return u.astype(np.float32)
