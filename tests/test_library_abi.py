"""The built C-ABI library loads and exports every symbol the header
declares (CPU only; no compute calls)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "chase_ph.h")
LIB = os.path.join(ROOT, "paper_2601_10557_amd", "libchase_ph.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(chase_ph_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["chase_ph_create", "chase_ph_filter", "chase_ph_qr", "chase_ph_oblique_rr",
              "chase_ph_residuals", "chase_ph_solve", "chase_ph_eigval_backward", "chase_ph_destroy"]:
        assert n in names


def test_library_exports_all_declared_symbols():
    assert os.path.exists(LIB), "build the library first: python -m paper_2601_10557_amd.build"
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_default_params_are_the_papers():
    """Defaults against the parameters the paper states (tests/golden/paper_parameters.txt)."""
    from paper_2601_10557_amd import _lib
    lib = _lib.load()
    p = _lib.Params()
    lib.chase_ph_default_params(ctypes.byref(p))
    vals = {}
    for line in open(os.path.join(ROOT, "tests", "golden", "paper_parameters.txt")):
        line = line.split("#")[0].strip()
        if line:
            k, v = line.split("=")
            vals[k.strip()] = float(v)
    assert p.gamma == vals["gamma"]
    assert p.max_iter == vals["max_iter"]
    assert p.deg_min == vals["deg_min"] and p.deg_max == vals["deg_max"]
    assert p.lanczos_steps % 2 == 0 and abs(p.lanczos_steps - vals["lanczos_steps_default"]) <= 1
