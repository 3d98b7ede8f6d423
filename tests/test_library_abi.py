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


def test_missing_library_fails_loudly(tmp_path):
    # no host fallback: a missing library is an import error
    from paper_2601_10557_amd import _lib
    try:
        _lib.load(str(tmp_path / "libchase_ph.so"))
    except ImportError as e:
        assert "no fallback" in str(e)
    else:
        raise AssertionError("load() of a missing library did not raise")


def _struct_fields(name):
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    body = re.search(r"typedef struct \{([^{}]*)\}\s*" + name + r"\s*;", text).group(1)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        names = decl.split(None, 1)[1] if not decl.startswith("double*") else decl[len("double*"):]
        for n in names.split(","):
            fields.append(n.strip().lstrip("*"))
    return fields


def test_ctypes_structs_match_the_header(tmp_path):
    """Field order, offsets and sizes of the ctypes mirrors against the C
    compiler's layout of the header structs."""
    import shutil
    import subprocess
    from paper_2601_10557_amd import _lib
    cc = shutil.which("gcc") or shutil.which("cc")
    assert cc, "no C compiler"
    src = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', 'int main(void) {']
    for cname, pyt in (("chase_ph_params", _lib.Params), ("chase_ph_info", _lib.Info)):
        names = _struct_fields(cname)
        assert names == [f for f, _ in pyt._fields_], (cname, names)
        src.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for n in names:
            src.append(f'printf("{cname}.{n} %zu\\n", offsetof({cname}, {n}));')
    src.append("return 0; }")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "layout"
    subprocess.run([cc, str(c), "-o", str(exe)], check=True)
    out = dict(line.rsplit(" ", 1) for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                               text=True).stdout.split("\n") if line)
    for cname, pyt in (("chase_ph_params", _lib.Params), ("chase_ph_info", _lib.Info)):
        assert int(out[cname]) == ctypes.sizeof(pyt), cname
        for f, _ in pyt._fields_:
            assert int(out[f"{cname}.{f}"]) == getattr(pyt, f).offset, (cname, f)


def test_create_rejects_invalid_tda_parameters():
    """Argument checks of chase_ph_create that run before any device call:
    the TDA mode (Alg. 1) is FP64 with a fixed degree, nex_auto needs it,
    and dB may be NULL only in it."""
    from paper_2601_10557_amd import _lib
    lib = _lib.load()

    def create(dB=1, **kw):
        p = _lib.Params()
        lib.chase_ph_default_params(ctypes.byref(p))
        p.m, p.nev, p.nex = 100, 10, 8
        for k, v in kw.items():
            setattr(p, k, v)
        h = ctypes.c_void_p()
        return lib.chase_ph_create(ctypes.byref(p), ctypes.c_void_p(1), None if dB is None else ctypes.c_void_p(dB),
                                   100, None, ctypes.byref(h))

    assert create(tda=1, precision=_lib.MIXED) == _lib.ERR_ARG
    assert create(tda=1, opt_deg=1) == _lib.ERR_ARG
    assert create(nex_auto=1) == _lib.ERR_ARG                 # without tda
    assert create(tda=1, nex_auto=1, nex=0) == _lib.ERR_ARG
    assert create(dB=None) == _lib.ERR_ARG                   # dB NULL outside the TDA mode
    assert create(tda=2) == _lib.ERR_ARG
    assert create(rr_max_sweeps=0) == _lib.ERR_ARG
