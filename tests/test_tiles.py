"""Host side of the Y-pass tile widths (cola_fft_tiles): the process-wide table, its
defaults and the widths that do not fit LDS or the work-group limit.  No GPU work."""

import pytest

from paper_1703_00879_amd import cola as C


@pytest.fixture(autouse=True)
def _defaults():
    yield
    for n in (32, 1024, 2048):
        C.cola_fft_tiles(n, 0, 0)


def test_defaults_are_the_lds_limited_widths():
    # widest tile whose elements fit 128 KB of LDS: 16 columns up to 1024 points, 8 at 2048
    assert C.cola_fft_tiles(32) == (16, 16)
    assert C.cola_fft_tiles(1024) == (16, 16)
    assert C.cola_fft_tiles(2048) == (8, 8)


def test_set_keep_and_restore():
    assert C.cola_fft_tiles(1024, 8, -1) == (8, 16)
    assert C.cola_fft_tiles(1024, -1, 4) == (8, 4)
    assert C.cola_fft_tiles(32) == (16, 16)   # other sizes untouched
    assert C.cola_fft_tiles(1024, 0, 0) == (16, 16)


@pytest.mark.parametrize("n,fwd,inv", [
    (2048, 16, -1),   # 256 KB of LDS
    (1024, 3, -1),
    (1024, -1, 32),
    (100, 8, 8),      # not a supported transform size
])
def test_rejected(n, fwd, inv):
    before = C.cola_fft_tiles(1024)
    with pytest.raises(C.ColaError) as e:
        C.cola_fft_tiles(n, fwd, inv)
    assert e.value.status == -1
    assert C.cola_fft_tiles(1024) == before
