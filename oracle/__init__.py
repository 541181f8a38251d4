"""FP64 CPU oracle for the COLA particle-mesh hot path with scale-dependent growth
and approximate screening (Winther, Koyama, Manera, Wright & Zhao,
"COLA with scale-dependent growth: applications to screened modified gravity
models", arXiv:1703.00879).

THIS PACKAGE IS TEST INFRASTRUCTURE, NOT PRODUCT CODE.  It is the checker the
GPU path is compared against: a plain, slow, obviously correct numpy/scipy
implementation in float64 of every step the GPU path computes.  Only the test
suite, the smoke check in ``__graft_entry__`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  The product path (``paper_1703_00879_amd``) never
imports, calls or links anything here, and this package imports nothing from
the product path.

Modules (each function cites the passage of the paper it follows):

* ``params``     -- run parameters and unit conventions
* ``background`` -- flat LCDM expansion, super-comoving time tau (Sec. 2)
* ``models``     -- mu(k,a), gamma_2, m(a), f_R(a), beta_DGP(a), screening
                    factors and smoothing windows (Secs. 5-6, App. B-C)
* ``growth``     -- D1(k,a) and the approximate D2(k,a) ODEs (Secs. 3-4)
* ``spectrum``   -- initial power spectrum (Eisenstein-Hu no-wiggle shape,
                    sigma_8 normalisation; not from the paper)
* ``rng``        -- counter-based SplitMix64 white noise
* ``lpt``        -- 1LPT/2LPT potentials and displacements (Secs. 3-4)
* ``pm``         -- CIC deposit, Poisson + screened fifth force, gather (Secs. 2, 6)
* ``cola``       -- time grid, leapfrog kick/drift about the LPT path (Sec. 2, App. A)
* ``pk``         -- shell-averaged power spectrum (Sec. 8 analysis outputs)

Parity status: every function is pinned by ``tests/test_oracle_*.py`` against
closed forms, limits, invariants or brute force, except where its docstring
says "parity unpinned".
"""

from .params import Params, MODEL_LCDM, MODEL_FR, MODEL_NDGP, MODEL_SYMMETRON  # noqa: F401
from .params import FILTER_GAUSS, FILTER_TOPHAT, FILTER_SHARPK  # noqa: F401
