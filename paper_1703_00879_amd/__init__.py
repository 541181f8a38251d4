"""MI355X-native COLA particle-mesh hot path with scale-dependent growth and approximate
screening: hand-written gfx950 HIP kernels behind the C ABI of include/cola.h, with a
thin ctypes binding (cola.py) of the same names."""

from .cola import (Params, State, ColaError, load_library, cola_query_sizes, cola_validate,  # noqa: F401
                   cola_prepare, cola_make_ic, cola_pm_force, cola_step, cola_power_spectrum,
                   cola_positions, cola_growth_table, cola_white_noise, cola_profile_enable,
                   cola_profile_reset, cola_profile_read, LCDM, FR_HS1, NDGP)
