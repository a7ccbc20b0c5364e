"""CPU-side checks of the HIP library: it loads, exports every declared
symbol, and its host-only entry points agree with the oracle."""
import ctypes as C

import numpy as np
import pytest

from oracle import green
from paper_2005_12338_amd import gf2


def test_library_exports_every_declared_symbol():
    lib = gf2.load()
    names = gf2.declared_symbols()
    assert "gf2_sigma_tau" in names and "gf2_build_B" in names and "gf2_split" in names
    assert "gf2_energy" in names
    for name in names:
        assert hasattr(lib, name), name
    assert lib.gf2_version().decode().startswith("gf2")


@pytest.mark.parametrize("ntau", [1, 2, 5, 32, 64, 128])
def test_tau_grid_matches_numpy_gauss_legendre(ntau):
    tau, w = gf2.gf2_tau_grid(50.0, ntau)
    rt, rw = green.tau_grid(50.0, ntau)
    assert np.max(np.abs(tau - rt)) < 1e-12 * 50
    assert np.max(np.abs(w - rw)) < 1e-12 * 50


def test_tau_grid_rejects_bad_arguments():
    lib = gf2.load()
    t = np.zeros(4)
    assert lib.gf2_tau_grid(-1.0, 4, t.ctypes.data_as(C.POINTER(C.c_double)),
                            t.ctypes.data_as(C.POINTER(C.c_double))) == gf2.GF2_E_ARG
    assert lib.gf2_tau_grid(1.0, 0, t.ctypes.data_as(C.POINTER(C.c_double)),
                            t.ctypes.data_as(C.POINTER(C.c_double))) == gf2.GF2_E_ARG


def test_null_context_is_an_argument_error():
    lib = gf2.load()
    assert lib.gf2_set_stream(None, None) == gf2.GF2_E_ARG
    assert lib.gf2_last_error(None) == b"null context"
