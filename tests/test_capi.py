"""CPU checks of the C-ABI library: it loads, exports every function that
include/wmg.h declares, and rejects invalid arguments in host-side
validation (before any device work)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_0912_2186_amd", "libwmg.so")
HDR = os.path.join(ROOT, "include", "wmg.h")


def declared_functions():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_]+\s*\*?\s*([a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libwmg.so not built")
    return ctypes.CDLL(LIB)


def test_header_declares_the_paper_calls():
    names = declared_functions()
    for n in ["wilson_apply", "mg_setup", "mg_solve", "mg_destroy", "mg_set_mass", "wmg_strerror"]:
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_constants_match_header(lib):
    """Every WMG_* constant of the Python binding has the value the header
    defines (flags, precisions, cycle types, error codes, profile slots)."""
    from paper_0912_2186_amd import wmg

    src = re.sub(r"/\*.*?\*/", "", open(HDR).read(), flags=re.S)
    defs = {}
    for name, val in re.findall(r"^\s*#define\s+(WMG_[A-Z0-9_]+)\s+(\(?-?[0-9][0-9a-fA-Fx]*\)?)", src, flags=re.M):
        defs[name] = int(val.strip("()"), 0)
    ours = {k: v for k, v in vars(wmg).items() if k.startswith("WMG_") and isinstance(v, int)}
    assert "WMG_Z32" in ours and "WMG_EO_SMOOTHER" in ours
    wrong = {k: (v, defs.get(k)) for k, v in ours.items() if k in defs and defs[k] != v}
    assert not wrong, wrong
    # flags are distinct bits
    flags = [defs[k] for k in ("WMG_X0_GIVEN", "WMG_COARSE_FP32", "WMG_LINKS18", "WMG_EO_SMOOTHER", "WMG_GRAPHS",
                               "WMG_SPIN_SPLIT", "WMG_COARSE_B32", "WMG_Z32")]
    assert all(f & (f - 1) == 0 for f in flags) and len(set(flags)) == len(flags)


class Geom(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int * 4)]


def test_validation_errors(lib):
    lib.wilson_apply.restype = ctypes.c_int
    lib.wilson_apply.argtypes = [ctypes.POINTER(Geom), ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p,
                                 ctypes.c_void_p, ctypes.c_void_p]
    g = Geom()
    g.L[:] = [4, 4, 4, 0]
    assert lib.wilson_apply(ctypes.byref(g), 8, 0.1, 8, 16, None) == -1
    g.L[:] = [4, 4, 4, 4]
    assert lib.wilson_apply(ctypes.byref(g), None, 0.1, 8, 16, None) == -1
    assert lib.wilson_apply(ctypes.byref(g), 8, 0.1, 16, 16, None) == -1  # aliasing
    lib.mg_setup.restype = ctypes.c_int
    lib.mg_setup.argtypes = [ctypes.POINTER(Geom), ctypes.c_void_p, ctypes.c_double, ctypes.c_int,
                             ctypes.POINTER(ctypes.c_int * 4), ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
    h = ctypes.c_void_p()
    blk = (ctypes.c_int * 4)(4, 4, 4, 3)  # does not divide 4
    assert lib.mg_setup(ctypes.byref(g), 8, 0.0, 4, ctypes.byref(blk), None, ctypes.byref(h)) == -1
    blk = (ctypes.c_int * 4)(2, 2, 2, 2)
    # Nv larger than the 6 * |block| components of one chirality half
    assert lib.mg_setup(ctypes.byref(g), 8, 0.0, 6 * 16 + 1, ctypes.byref(blk), None, ctypes.byref(h)) == -1
    assert lib.mg_setup(ctypes.byref(g), 8, 0.0, 0, ctypes.byref(blk), None, ctypes.byref(h)) == -1
    lib.wmg_strerror.restype = ctypes.c_char_p
    assert b"Nv" in lib.wmg_strerror(-1)


def test_default_params(lib):
    class P(ctypes.Structure):
        _fields_ = [("levels", ctypes.c_int), ("block", ctypes.c_int * 8), ("nvec", ctypes.c_int * 2),
                    ("setup_iters", ctypes.c_int), ("post_smooth", ctypes.c_int), ("gcr_restart", ctypes.c_int),
                    ("cycle", ctypes.c_int), ("precision", ctypes.c_int), ("nrhs_max", ctypes.c_int),
                    ("coarse_tol", ctypes.c_double), ("coarse_maxiter", ctypes.c_int),
                    ("reliable_delta", ctypes.c_double), ("maxiter", ctypes.c_int), ("seed", ctypes.c_ulonglong),
                    ("flags", ctypes.c_int)]

    p = P()
    assert lib.wmg_default_params(ctypes.byref(p)) == 0
    # Sec. 3: 4^4 aggregates, 4 post-smoothing steps, GCR(8), W-cycle
    assert list(p.block)[:4] == [4, 4, 4, 4]
    assert p.post_smooth == 4 and p.gcr_restart == 8 and p.cycle == 1


def test_bench_refuses_several_gpus():
    import subprocess
    import sys

    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_noalloc_rejects_sizes_beyond_its_array(lib):
    # host-side size check of the allocation-free entry point: returns
    # EINVAL before any device work (fake non-null pointers are never touched)
    f = lib.bicgstab_solve_noalloc
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.POINTER(Geom), ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                  ctypes.c_double, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    g = Geom()
    g.L[:] = [16, 16, 16, 8]
    assert f(ctypes.byref(g), 8, -0.1, 16, 32, 1e-10, 100, None, None) == -1
    lib.wmg_strerror.restype = ctypes.c_char_p
    assert b"fixed maximum" in lib.wmg_strerror(-1)
    g.L[:] = [8, 8, 8, 8]
    assert f(ctypes.byref(g), None, -0.1, 16, 32, 1e-10, 100, None, None) == -1


def test_mg_load_rejects_missing_and_foreign_files(lib, tmp_path):
    # file checks come before any device work (fake non-null pointers)
    f = lib.mg_load
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_char_p, ctypes.POINTER(Geom), ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p,
                  ctypes.POINTER(ctypes.c_void_p)]
    g = Geom()
    g.L[:] = [8, 8, 8, 8]
    h = ctypes.c_void_p()
    assert f(str(tmp_path / "missing").encode(), ctypes.byref(g), 8, -0.1, None, ctypes.byref(h)) == -1
    bad = tmp_path / "bad"
    bad.write_bytes(b"\0" * 4096)
    assert f(str(bad).encode(), ctypes.byref(g), 8, -0.1, None, ctypes.byref(h)) == -1
    lib.wmg_strerror.restype = ctypes.c_char_p
    assert b"not a setup file" in lib.wmg_strerror(-1)
