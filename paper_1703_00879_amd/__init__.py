"""MI355X-native COLA particle-mesh hot path with scale-dependent growth and approximate
screening: hand-written gfx950 HIP kernels behind the C ABI of include/cola.h, with a
thin ctypes binding (cola.py) of the same names."""

from .cola import (Params, State, ColaError, Ensemble, load_library, cola_query_sizes,  # noqa: F401
                   cola_validate, cola_prepare, cola_make_ic, cola_pm_force, cola_step,
                   cola_step_static, cola_power_spectrum, cola_positions, cola_growth_table,
                   cola_white_noise, cola_growth_triangles, cola_step_times, cola_fft_tiles,
                   cola_autotune, cola_profile_enable, cola_profile_reset, cola_profile_read,
                   LCDM, FR_HS1, NDGP, SYMMETRON, MBETA, KMOUFLAGE, READ_X_TOTAL_DENSITY,
                   READ_X_NO_A3, READ_D2_HALF_K)
