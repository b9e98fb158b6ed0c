"""CPU checks of the C-ABI library: it loads and exports every function include/dgp.h declares.

No compute call is made (there is no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dgp.h")
LIB = os.path.join(ROOT, "paper_0906_4548_amd", "libdgp.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dgp_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("dgp_deposit", "dgp_solve_field", "dgp_pm_forces", "dgp_step", "dgp_solve_field_backward"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdgp.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdgp.so not built")
def test_binding_matches_exports():
    from paper_0906_4548_amd import _lib
    assert set(_lib.EXPORTS) == set(declared_functions())


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdgp.so not built")
def test_params_init_host_only():
    # dgp_params_init is a pure host function: check it against the oracle's coefficients
    from paper_0906_4548_amd import _lib
    from oracle import cosmology as cos
    lib = _lib.load()
    p = _lib.Params()
    assert lib.dgp_params_init(ctypes.byref(p), 0.27, 0.5) == 0
    c = cos.coefficients(0.27, 0.5)
    for k in ("E", "eta", "alpha", "beta", "A", "gamma", "c2", "kappa"):
        assert abs(getattr(p, k) - getattr(c, k)) <= 1e-15 * abs(getattr(c, k))
    assert abs(p.w - 1 / 3) < 1e-16 and p.lambda_ == 1.0 and p.tol == 0.01
    assert lib.dgp_params_init(ctypes.byref(p), 1.5, 0.5) == -1
    assert b"omega_m0" in lib.dgp_last_error()
