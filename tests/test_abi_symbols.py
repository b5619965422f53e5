"""The C-ABI library loads and exports every entry point include/absorber.h declares
(no compute call: this runs without a GPU)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "absorber.h")
LIB = os.path.join(ROOT, "paper_2607_15420_amd", "libabsorber.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(absorber_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("absorber_create", "absorber_eval_cons", "absorber_eval_jac", "absorber_eval_hess",
                     "absorber_kkt_factor", "absorber_kkt_solve", "absorber_ipm_solve", "absorber_last_error"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built (python -m paper_2607_15420_amd.build)")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_marshals_params(params):
    from paper_2607_15420_amd.binding import params_struct
    s = params_struct(params)
    assert s.nu[2][0] == 1.0 and s.nu[1][0] == -1.0
    assert s.x0[15] == params["initial_point"]["T"]
    assert s.d_hi == params["bounds"]["d"][1]
