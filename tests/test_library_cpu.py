"""Host-side checks of the C ABI library: it loads, exports every declared entry point,
and its host-compiled FP64 Bessel routines agree with independent evaluations."""
import os
import re

import numpy as np
import pytest
from scipy import special as sp

from paper_2005_01372_amd import lsop

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lsop.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(\w+)\s*\(", txt, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(lsop.LIB_PATH):
        pytest.fail("liblsop.so is not built (run __graft_entry__.build())")
    return lsop.load_library()


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 15
    assert set(names) == set(lsop.EXPORTS)
    for name in names:
        assert hasattr(lib, name), name


def test_header_enums_match_binding():
    txt = open(HEADER).read()
    for name, val in [("LSOP_OK", 0), ("LSOP_EINVAL", 1), ("LSOP_NOT_CONVERGED", 4), ("LSOP_DIVERGED", 5),
                      ("LSOP_ESINGULAR", 6), ("LSOP_EUNSUPPORTED", 7), ("LSOP_C64", 0), ("LSOP_C128", 1),
                      ("LSOP_MIXED", 2), ("LSOP_MODE_VHG0H", 3), ("LSOP_PC_LOWRANK", 1)]:
        assert re.search(rf"{name}\s*=\s*{val}\b", txt), name
    assert lsop.MODES == {"A": 0, "G0V": 1, "AH": 2, "VHG0H": 3}


@pytest.mark.parametrize("x", [0.01, 0.05, 0.3, 1.0, 2.404825557695773, 5.52, 7.9, 12.0, 19.999, 20.0, 20.001,
                               33.3, 100.0, 577.7, 1500.0])
def test_host_hankel0(lib, x):
    j0, y0 = lsop.bessel_host(0, x)
    h = sp.hankel1(0, x)
    scale = max(abs(h), 1e-300)
    assert abs(j0 - h.real) <= 2e-15 * scale and abs(y0 - h.imag) <= 2e-15 * scale


@pytest.mark.parametrize("x", [1e-3, 0.05, 0.177, 0.3, 1.0, 2.0])
def test_host_bessel1(lib, x):
    j1, y1 = lsop.bessel_host(1, x)
    assert abs(j1 - sp.j1(x)) <= 1e-15 * abs(sp.j1(x))
    assert abs(y1 - sp.y1(x)) <= 1e-15 * abs(sp.y1(x))


def test_host_bessel_rejects_bad_input(lib):
    with pytest.raises(lsop.LsopError):
        lsop.bessel_host(0, -1.0)
    with pytest.raises(lsop.LsopError):
        lsop.bessel_host(1, 3.0)


def test_hankel_against_mpmath_high_precision(lib):
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 40
    for x in np.geomspace(0.02, 900, 37):
        ref = complex(mp.hankel1(0, x))
        j0, y0 = lsop.bessel_host(0, float(x))
        assert abs(complex(j0, y0) - ref) <= 3e-15 * abs(ref), x
