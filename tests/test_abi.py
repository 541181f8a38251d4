"""The C-ABI library loads and exports every entry point declared in include/cola.h;
host-only calls (sizes, validation, error strings) work without a GPU."""

import ctypes
import os
import re

import pytest

from paper_1703_00879_amd import cola as C


def _declared(root):
    txt = open(os.path.join(root, "include", "cola.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(cola_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol(root):
    lib = C.load_library()
    names = _declared(root)
    assert "cola_make_ic" in names and "cola_step" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(C.EXPORTED) == set(names)


def test_query_sizes_and_layout():
    p = C.Params(model=C.NDGP, np1d=512, nmesh1d=1024, box=1024.0, n_steps=30)
    s = C.cola_query_sizes(p)
    N = 512 ** 3
    assert s["disp_bytes"] == s["vel_bytes"] >= 12 * N
    assert s["lpt_bytes"] >= 24 * N                     # Psi1, Psi2 per particle
    up = lambda x: -(-x // 256) * 256                   # noqa: E731
    mesh = up(1024 * (1024 * 528 + 16) * 8)             # padded half-complex mesh
    ntiles = (1024 // 16) ** 3                          # 16^3-cell deposit tiles
    nblk = -(-ntiles // 1024)
    bins = -(-(17 * ntiles + 2 * nblk + 64) * 4 // 256) * 256
    # six mesh slots + tile counters; the sorted CIC records (12 B each) fit in slot 5
    assert 12 * N <= mesh and s["work_bytes"] == 6 * mesh + bins
    assert s["total_bytes"] == sum(v for k, v in s.items() if k != "total_bytes")
    # scale-dependent f(R) stores phi1_k, phi2_k; its per-step LPT work (three
    # particle-grid fields and the interleaved L'' and Delta arrays) lies over mesh slots
    # 0-2 when it fits there, as it does at n_mesh = 2 n_p
    sf = C.cola_query_sizes(p.with_(model=C.FR_HS1))
    pg = up(512 * (512 * 272 + 16) * 8)
    assert 3 * pg + 2 * up(12 * N) <= 3 * mesh
    assert sf["lpt_bytes"] == 2 * pg and sf["work_bytes"] == 6 * mesh + bins
    # at n_mesh = n_p it does not fit and gets an area of its own
    q = C.Params(model=C.FR_HS1, np1d=128, nmesh1d=128, box=128.0, n_steps=10)
    sq = C.cola_query_sizes(q)
    mq, pq = up(128 * (128 * 80 + 16) * 8), up(128 * (128 * 80 + 16) * 8)
    nt = (128 // 16) ** 3
    bq = -(-(17 * nt + 2 * (-(-nt // 1024)) + 64) * 4 // 256) * 256
    # (and the 12-byte CIC records, larger than a slot here, get their own area too)
    assert sq["work_bytes"] == 6 * mq + 3 * pq + 2 * up(12 * 128 ** 3) + bq + up(12 * 128 ** 3)


@pytest.mark.parametrize("bad", [dict(np1d=30), dict(np1d=40), dict(nmesh1d=96, np1d=64),
                                 dict(np1d=64, nmesh1d=32), dict(box=0.0), dict(n_steps=0),
                                 dict(model=1, fr0_abs=0.0), dict(model=2, rc_h0=-1.0),
                                 dict(omega_m=1.5), dict(filter=3), dict(np1d=2048, nmesh1d=2048),
                                 dict(np1d=16, nmesh1d=96)])
def test_invalid_parameters_rejected(bad):
    p = C.Params().with_(**bad)
    with pytest.raises(C.ColaError) as e:
        C.cola_validate(p)
    assert e.value.status == -1
    with pytest.raises(C.ColaError):
        C.cola_query_sizes(p)


def test_null_state_rejected_without_gpu():
    lib = C.load_library()
    p = C.Params()
    st = lib.cola_make_ic(ctypes.byref(p._c()), None, None)
    assert st == -1
    assert b"NULL" in lib.cola_last_error()
    assert lib.cola_status_string(-3) == b"call out of order"
