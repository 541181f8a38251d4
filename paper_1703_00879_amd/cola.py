"""Thin ctypes binding of libcola (include/cola.h).

Argument marshalling only: every step of the COLA path runs in the library's HIP
kernels.  PyTorch supplies device memory (caller-owned buffers sized by
cola_query_sizes) and the current HIP stream.  If the shared library is missing the
import fails loudly; there is no fallback implementation.
"""

import ctypes
import os
from dataclasses import dataclass, fields, replace

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("COLA_LIBRARY") or os.path.join(_PKG, "_lib", "libcola.so")

COLA_OK = 0
LCDM, FR_HS1, NDGP, SYMMETRON, MBETA, KMOUFLAGE = 0, 1, 2, 3, 4, 5
MBETA_MAX_KNOTS = 64
SMOOTH_GAUSS, SMOOTH_TOPHAT, SMOOTH_SHARPK = 0, 1, 2
READ_X_TOTAL_DENSITY, READ_X_NO_A3, READ_D2_HALF_K = 1, 2, 4

EXPORTED = ["cola_query_sizes", "cola_validate", "cola_prepare", "cola_make_ic", "cola_pm_force",
            "cola_step", "cola_step_static", "cola_ensemble_create", "cola_ensemble_run",
            "cola_ensemble_destroy", "cola_power_spectrum", "cola_positions", "cola_growth_table",
            "cola_white_noise", "cola_growth_triangles", "cola_step_times", "cola_fft_tiles", "cola_autotune",
            "cola_profile_enable", "cola_profile_read", "cola_profile_reset",
            "cola_status_string", "cola_last_error"]


class ColaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libcola status {status}: {msg}")
        self.status = status


class _Params(ctypes.Structure):
    _fields_ = [("omega_m", ctypes.c_double), ("omega_b", ctypes.c_double), ("h", ctypes.c_double),
                ("n_s", ctypes.c_double), ("sigma8", ctypes.c_double), ("t_cmb", ctypes.c_double),
                ("fr0_abs", ctypes.c_double), ("rc_h0", ctypes.c_double),
                ("r_smooth", ctypes.c_double), ("box", ctypes.c_double),
                ("z_init", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("model", ctypes.c_int32), ("screening", ctypes.c_int32),
                ("filter", ctypes.c_int32), ("growth_mode", ctypes.c_int32),
                ("np1d", ctypes.c_int32), ("nmesh1d", ctypes.c_int32),
                ("n_steps", ctypes.c_int32), ("readings", ctypes.c_int32),
                ("sym_beta", ctypes.c_double), ("sym_mass", ctypes.c_double),
                ("sym_astar", ctypes.c_double),
                ("mb_n", ctypes.c_int32), ("mb_reserved", ctypes.c_int32),
                ("mb_lna", ctypes.c_double * MBETA_MAX_KNOTS),
                ("mb_beta", ctypes.c_double * MBETA_MAX_KNOTS),
                ("mb_m2", ctypes.c_double * MBETA_MAX_KNOTS),
                ("km_beta", ctypes.c_double), ("km_k0", ctypes.c_double),
                ("km_lambda", ctypes.c_double), ("km_x0", ctypes.c_double),
                ("km_xn", ctypes.c_double), ("km_m", ctypes.c_int32),
                ("km_reserved", ctypes.c_int32)]


class _Sizes(ctypes.Structure):
    _fields_ = [("disp_bytes", ctypes.c_size_t), ("vel_bytes", ctypes.c_size_t),
                ("lpt_bytes", ctypes.c_size_t), ("tables_bytes", ctypes.c_size_t),
                ("work_bytes", ctypes.c_size_t), ("total_bytes", ctypes.c_size_t)]


class _State(ctypes.Structure):
    _fields_ = [("disp", ctypes.c_void_p), ("vel", ctypes.c_void_p), ("lpt", ctypes.c_void_p),
                ("tables", ctypes.c_void_p), ("work", ctypes.c_void_p),
                ("next_step", ctypes.c_int32), ("prepared", ctypes.c_int32)]


@dataclass(frozen=True)
class Params:
    """Mirror of cola_params (see include/cola.h for meaning and valid ranges)."""
    omega_m: float = 0.3
    omega_b: float = 0.05
    h: float = 0.7
    n_s: float = 0.96
    sigma8: float = 0.8
    t_cmb: float = 2.7255
    fr0_abs: float = 1e-5
    rc_h0: float = 1.0
    sym_beta: float = 1.0
    sym_mass: float = 2997.92458
    sym_astar: float = 0.5
    r_smooth: float = 1.0
    box: float = 200.0
    z_init: float = 19.0
    seed: int = 1
    model: int = LCDM
    screening: int = 1
    filter: int = SMOOTH_GAUSS
    growth_mode: int = 0
    np1d: int = 32
    nmesh1d: int = 64
    n_steps: int = 10
    readings: int = 0
    # general {m(a), beta(a)} model: knots ln a, beta and m^2/H0^2 there (tuples)
    mb_lna: tuple = ()
    mb_beta: tuple = ()
    mb_m2: tuple = ()
    # k-Mouflage: P(X) = -1 + X + km_k0 X^km_m, coupling, lambda (Mpc/h), X(a) = km_x0 a^km_xn
    km_beta: float = 0.5
    km_k0: float = 1.0
    km_m: int = 3
    km_lambda: float = 1e6
    km_x0: float = 0.0
    km_xn: float = 0.0

    def with_(self, **kw):
        return replace(self, **kw)

    def _c(self):
        kw = {f.name: getattr(self, f.name) for f in fields(self) if not f.name.startswith("mb_")}
        c = _Params(**kw)
        n = len(self.mb_lna)
        if not (len(self.mb_beta) == n and len(self.mb_m2) == n and n <= MBETA_MAX_KNOTS):
            raise ValueError("mb_lna, mb_beta and mb_m2 need equal lengths <= MBETA_MAX_KNOTS")
        c.mb_n = n
        for i in range(n):
            c.mb_lna[i], c.mb_beta[i], c.mb_m2[i] = self.mb_lna[i], self.mb_beta[i], self.mb_m2[i]
        return c


_lib = None


def load_library(path=LIB_PATH):
    """Load libcola.so once; raise if it is missing (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libcola not built: {path} missing (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    P, S, St = ctypes.POINTER(_Params), ctypes.POINTER(_Sizes), ctypes.POINTER(_State)
    vp, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "cola_query_sizes": [P, S], "cola_validate": [P], "cola_prepare": [P, St, vp],
        "cola_make_ic": [P, St, vp], "cola_pm_force": [P, St, d, vp, vp, vp],
        "cola_step": [P, St, i32, vp], "cola_step_static": [P, St, i32, vp],
        "cola_ensemble_create": [i32, P, vp, vp], "cola_ensemble_run": [vp, i32, vp],
        "cola_ensemble_destroy": [vp],
        "cola_power_spectrum": [P, St, i32, vp, vp, vp, vp],
        "cola_positions": [P, St, vp, vp],
        "cola_growth_table": [P, St, i32, vp, i64, vp, vp],
        "cola_white_noise": [P, i32, vp, vp], "cola_growth_triangles": [P, i32, vp, d, vp, vp],
        "cola_step_times": [P, i32, vp],
        "cola_fft_tiles": [i32, i32, i32, vp], "cola_autotune": [P, St, vp, vp],
        "cola_profile_enable": [i32],
        "cola_profile_read": [vp, vp, vp, i32, vp], "cola_profile_reset": [],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int32
    lib.cola_status_string.argtypes = [ctypes.c_int32]
    lib.cola_status_string.restype = ctypes.c_char_p
    lib.cola_last_error.argtypes = []
    lib.cola_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(st):
    if st != COLA_OK:
        raise ColaError(st, _lib.cola_last_error().decode())


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(stream)
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


# ----------------------------------------------------------------------------- entry points
def cola_validate(p):
    lib = load_library()
    _check(lib.cola_validate(ctypes.byref(p._c())))


def cola_query_sizes(p):
    lib = load_library()
    s = _Sizes()
    _check(lib.cola_query_sizes(ctypes.byref(p._c()), ctypes.byref(s)))
    return {f[0]: int(getattr(s, f[0])) for f in _Sizes._fields_}


class State:
    """Caller-owned device buffers of one run (torch uint8 tensors, 256-byte aligned)
    plus the cola_state struct pointing at them."""

    def __init__(self, p, device="cuda:0"):
        import torch
        self.p = p
        self.sizes = cola_query_sizes(p)
        self._keep = []
        self.c = _State()
        for name in ("disp", "vel", "lpt", "tables", "work"):
            nbytes = self.sizes[name + "_bytes"]
            buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
            off = (-buf.data_ptr()) % 256
            view = buf[off:off + nbytes]
            self._keep.append(buf)
            setattr(self, name, view)
            setattr(self.c, name, view.data_ptr())
        self.c.next_step = -1
        self.c.prepared = 0
        N = p.np1d ** 3
        self.disp_f = self.disp.view(torch.float32)[:3 * N].view(3, N)
        self.vel_f = self.vel.view(torch.float32)[:3 * N].view(3, N)

    @property
    def next_step(self):
        return self.c.next_step


def cola_prepare(p, state, stream=None):
    _check(load_library().cola_prepare(ctypes.byref(p._c()), ctypes.byref(state.c), _stream(stream)))


def cola_make_ic(p, state, stream=None):
    _check(load_library().cola_make_ic(ctypes.byref(p._c()), ctypes.byref(state.c), _stream(stream)))


def cola_pm_force(p, state, a, force_out=None, mesh_out=None, stream=None):
    _check(load_library().cola_pm_force(ctypes.byref(p._c()), ctypes.byref(state.c), float(a),
                                        _ptr(force_out), _ptr(mesh_out), _stream(stream)))


def cola_step(p, state, i, stream=None):
    _check(load_library().cola_step(ctypes.byref(p._c()), ctypes.byref(state.c), int(i),
                                    _stream(stream)))


def cola_step_static(p, state, i, stream=None):
    _check(load_library().cola_step_static(ctypes.byref(p._c()), ctypes.byref(state.c), int(i),
                                           _stream(stream)))


class Ensemble:
    """Runs stepped together as captured HIP graphs (cola_ensemble_*): the parameter and
    state arrays are marshalled once; run() advances every member to z = 0."""

    def __init__(self, params, states):
        lib = load_library()
        self.states = list(states)
        self._p = (_Params * len(params))(*[q._c() for q in params])
        self._st = (ctypes.POINTER(_State) * len(states))(*[ctypes.pointer(st.c) for st in states])
        self.h = ctypes.c_void_p(0)
        _check(lib.cola_ensemble_create(len(params), self._p, self._st, ctypes.byref(self.h)))

    def run(self, n_streams=8, stream=None):
        _check(load_library().cola_ensemble_run(self.h, int(n_streams), _stream(stream)))

    def close(self):
        if self.h:
            _check(load_library().cola_ensemble_destroy(self.h))
            self.h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cola_power_spectrum(p, state, nbins=None, stream=None):
    nbins = p.nmesh1d // 2 if nbins is None else nbins
    k = np.zeros(nbins)
    P = np.zeros(nbins)
    n = np.zeros(nbins, dtype=np.int64)
    _check(load_library().cola_power_spectrum(
        ctypes.byref(p._c()), ctypes.byref(state.c), int(nbins), k.ctypes.data_as(ctypes.c_void_p),
        P.ctypes.data_as(ctypes.c_void_p), n.ctypes.data_as(ctypes.c_void_p), _stream(stream)))
    return k, P, n


def cola_positions(p, state, xyz_out, stream=None):
    _check(load_library().cola_positions(ctypes.byref(p._c()), ctypes.byref(state.c), _ptr(xyz_out),
                                         _stream(stream)))


def cola_growth_table(p, state, i, stream=None):
    n_k = 3 * (p.np1d // 2) ** 2 + 1
    out = np.zeros(n_k * 6)
    nk = ctypes.c_int64(0)
    _check(load_library().cola_growth_table(
        ctypes.byref(p._c()), ctypes.byref(state.c), int(i), out.ctypes.data_as(ctypes.c_void_p),
        out.size, ctypes.byref(nk), _stream(stream)))
    return out[:nk.value * 6].reshape(nk.value, 6)


def cola_white_noise(p, dst, grid=0, stream=None):
    _check(load_library().cola_white_noise(ctypes.byref(p._c()), int(grid), _ptr(dst),
                                           _stream(stream)))


def cola_growth_triangles(p, tri, a, out, stream=None):
    """tri: device float64 (n, 3) of (|k|, |k1|, |k2|) [h/Mpc]; out: device float64 (n, 2)."""
    n = int(tri.shape[0])
    _check(load_library().cola_growth_triangles(ctypes.byref(p._c()), n, _ptr(tri), float(a),
                                                _ptr(out), _stream(stream)))


def cola_step_times(p, i):
    """(a_i, a_{i+1}, kick interval, drift interval) of step i in FP64 (host only)."""
    out = (ctypes.c_double * 4)()
    _check(load_library().cola_step_times(ctypes.byref(p._c()), int(i), out))
    return tuple(out)


def cola_fft_tiles(n, fwd=-1, inv=-1):
    """Set the Y-pass tile widths of n-point transforms (4, 8, 16; 0 = default; -1 = keep);
    returns the widths in use as (forward, inverse)."""
    cur = (ctypes.c_int32 * 2)()
    _check(load_library().cola_fft_tiles(int(n), int(fwd), int(inv), cur))
    return cur[0], cur[1]


def cola_autotune(p, state, stream=None):
    """Time the Y-pass tile widths on the state's work buffer and keep the fastest; returns
    (mesh fwd, mesh inv, particle-grid fwd, particle-grid inv)."""
    out = (ctypes.c_int32 * 4)()
    _check(load_library().cola_autotune(ctypes.byref(p._c()), ctypes.byref(state.c), out,
                                        _stream(stream)))
    return tuple(out)


def cola_profile_enable(on=True):
    _check(load_library().cola_profile_enable(1 if on else 0))


def cola_profile_reset():
    _check(load_library().cola_profile_reset())


def cola_profile_read(cap=128):
    names = (ctypes.c_char * 48 * cap)()
    ms = (ctypes.c_double * cap)()
    cnt = (ctypes.c_int64 * cap)()
    n = ctypes.c_int32(0)
    _check(load_library().cola_profile_read(names, ms, cnt, cap, ctypes.byref(n)))
    return {names[i].value.decode(): (ms[i], cnt[i]) for i in range(min(n.value, cap))}
