"""ctypes binding of ``libwmg.so`` (C ABI in ``include/wmg.h``).

Argument marshalling only: every step of the method runs in the HIP
library.  Fields are torch CUDA tensors of dtype complex128 in the canonical
layouts of ``wmg.h`` (gauge ``(V, 4, 3, 3)``, spinors ``(nrhs, V, 12)``,
coarse vectors ``(nrhs, Vc, n)``); their device pointers are handed to the
library.  Importing this module raises if the library is missing: there is
no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwmg.so")
if not os.path.exists(LIB_PATH):
    raise ImportError("libwmg.so is not built (run __graft_entry__.build() or paper_0912_2186_amd/build.py)")
_lib = ctypes.CDLL(LIB_PATH)

WMG_OK = 0
WMG_ENOTCONV = 1
WMG_EINVAL = -1
WMG_ENOMEM = -2
WMG_EHIP = -3
WMG_ERANK = -4
WMG_EBREAKDOWN = -5
WMG_FP64 = 0
WMG_MIXED = 1
WMG_VCYCLE = 0
WMG_WCYCLE = 1
WMG_X0_GIVEN = 1
WMG_COARSE_FP32 = 2
WMG_LINKS18 = 4
WMG_EO_SMOOTHER = 8
WMG_GRAPHS = 16
WMG_SPIN_SPLIT = 32
WMG_COARSE_B32 = 64
WMG_Z32 = 128


class WmgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("wmg error %d: %s" % (code, msg))
        self.code = code


class Geom(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int * 4)]


class Params(ctypes.Structure):
    _fields_ = [
        ("levels", ctypes.c_int),
        ("block", ctypes.c_int * 8),
        ("nvec", ctypes.c_int * 2),
        ("setup_iters", ctypes.c_int),
        ("post_smooth", ctypes.c_int),
        ("gcr_restart", ctypes.c_int),
        ("cycle", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("nrhs_max", ctypes.c_int),
        ("coarse_tol", ctypes.c_double),
        ("coarse_maxiter", ctypes.c_int),
        ("reliable_delta", ctypes.c_double),
        ("maxiter", ctypes.c_int),
        ("seed", ctypes.c_ulonglong),
        ("flags", ctypes.c_int),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("outer_iters", ctypes.c_int),
        ("fine_matvecs", ctypes.c_int),
        ("fine_matvecs_fp64", ctypes.c_int),
        ("coarse_iters", ctypes.c_int),
        ("reliable_updates", ctypes.c_int),
        ("converged", ctypes.c_int),
        ("true_relres", ctypes.c_double),
        ("setup_s", ctypes.c_double),
        ("solve_s", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_vp = ctypes.c_void_p
_i = ctypes.c_int
_d = ctypes.c_double
_P = ctypes.POINTER
_sig = {
    "wmg_default_params": (_i, [_P(Params)]),
    "wmg_strerror": (ctypes.c_char_p, [_i]),
    "wilson_apply": (_i, [_P(Geom), _vp, _d, _vp, _vp, _vp]),
    "mg_setup": (_i, [_P(Geom), _vp, _d, _i, _P(ctypes.c_int * 4), _P(Params), _P(_vp)]),
    "mg_solve": (_i, [_vp, _vp, _vp, _d, _i, _P(Stats)]),
    "mg_set_mass": (_i, [_vp, _d]),
    "mg_set_precision": (_i, [_vp, _i]),
    "mg_destroy": (_i, [_vp]),
    "bicgstab_solve": (_i, [_P(Geom), _vp, _d, _vp, _vp, _d, _i, _P(Stats)]),
    "bicgstab_solve_noalloc": (_i, [_P(Geom), _vp, _d, _vp, _vp, _d, _i, _P(Stats), _vp]),
    "mg_setup_batch": (_i, [_i, _P(Geom), _P(_vp), _P(_d), _i, _P(ctypes.c_int * 4), _P(Params), _P(_vp)]),
    "mg_solve_batch": (_i, [_vp, _P(_vp), _P(_vp), _d, _P(Stats)]),
    "mg_level_info": (_i, [_vp, _i, _P(ctypes.c_int * 4), _P(_i), _P(_i)]),
    "mg_set_null_vectors": (_i, [_vp, _i, _vp]),
    "mg_get_null_vectors": (_i, [_vp, _i, _vp]),
    "mg_get_prolongator": (_i, [_vp, _i, _vp]),
    "mg_get_coarse_links": (_i, [_vp, _i, _vp]),
    "mg_restrict": (_i, [_vp, _i, _vp, _vp, _i]),
    "mg_prolong": (_i, [_vp, _i, _vp, _vp, _i]),
    "mg_coarse_apply": (_i, [_vp, _i, _vp, _vp, _i, _i]),
    "mg_coarse_apply_f32": (_i, [_vp, _i, _vp, _vp, _i, _i]),
    "mg_restrict_f32": (_i, [_vp, _i, _vp, _vp, _i]),
    "mg_prolong_f32": (_i, [_vp, _i, _vp, _vp, _i]),
    "mg_apply_fine": (_i, [_vp, _i, _vp, _vp, _i]),
    "mg_smoother_residual": (_i, [_vp, _vp, _vp, _vp, _i]),
    "mg_hop_eo": (_i, [_vp, _i, _i, _d, _d, _vp, _vp, _vp, _i]),
    "mg_link_reals": (_i, [_vp]),
    "mg_save": (_i, [_vp, ctypes.c_char_p]),
    "mg_load": (_i, [ctypes.c_char_p, _P(Geom), _vp, _d, _P(Params), _P(_vp)]),
    "mg_refresh": (_i, [_vp, _vp, _i]),
    "mg_cycle": (_i, [_vp, _vp, _vp]),
    "mg_last_iters": (_i, [_vp, _P(_i), _i]),
    "mg_time_dslash": (_i, [_vp, _i, _i, _i, _P(_d)]),
    "mg_profile": (_i, [_vp, _i]),
    "wmg_tune_force": (_i, [_i]),
    "mg_profile_get": (_i, [_vp, _i, _P(_i), _P(_d), _P(_d)]),
}
KERNEL_KINDS = {"dslash_cycle": 0, "dslash_outer32": 1, "dslash_fp64": 2, "coarse_fp32": 3, "coarse_fp64": 4,
                "restrict": 5, "prolong": 6, "dslash_residual": 7}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def _check(rc: int, allow_notconv: bool = False) -> int:
    if rc == 0 or (allow_notconv and rc == WMG_ENOTCONV):
        return rc
    raise WmgError(rc, _lib.wmg_strerror(rc).decode())


def _ptr(t: torch.Tensor) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA tensor")
    if t.dtype != torch.complex128 or not t.is_contiguous():
        raise TypeError("expected a contiguous complex128 tensor")
    return t.data_ptr()


def _geom(L) -> Geom:
    g = Geom()
    for i in range(4):
        g.L[i] = int(L[i])
    return g


def default_params(**kw) -> Params:
    p = Params()
    _check(_lib.wmg_default_params(ctypes.byref(p)))
    for k, v in kw.items():
        if k == "block":
            flat = [int(a) for blk in v for a in blk]
            if len(flat) == 4:
                flat = flat + [2, 2, 2, 2]
            for i in range(8):
                p.block[i] = flat[i]
        elif k == "nvec":
            p.nvec[0] = int(v[0])
            p.nvec[1] = int(v[1] if len(v) > 1 else v[0])
        else:
            setattr(p, k, v)
    return p


def _stream_ptr(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def tune_force(choice: int) -> int:
    """Autotuner test hook: run candidate `choice` everywhere (< 0: off)."""
    return int(_lib.wmg_tune_force(int(choice)))


def wilson_apply(L, U: torch.Tensor, m: float, inp: torch.Tensor, out: torch.Tensor, stream=None) -> None:
    """Eq. 2.2, FP64, canonical layouts; enqueued on `stream` (default: torch's current)."""
    _check(_lib.wilson_apply(ctypes.byref(_geom(L)), _ptr(U), float(m), _ptr(inp), _ptr(out), _stream_ptr(stream)))


def bicgstab_solve(L, U, m, b, x, tol, maxiter=100000):
    st = Stats()
    rc = _lib.bicgstab_solve(ctypes.byref(_geom(L)), _ptr(U), float(m), _ptr(b), _ptr(x), float(tol), int(maxiter),
                             ctypes.byref(st))
    _check(rc, allow_notconv=True)
    return st.as_dict()


def bicgstab_solve_noalloc(L, U, m, b, x, tol, maxiter=100000, stream=None):
    """The allocation-free variant (work buffers in the library's fixed
    device array); runs on `stream` (default: torch's current stream)."""
    st = Stats()
    rc = _lib.bicgstab_solve_noalloc(ctypes.byref(_geom(L)), _ptr(U), float(m), _ptr(b), _ptr(x), float(tol),
                                     int(maxiter), ctypes.byref(st), _stream_ptr(stream))
    _check(rc, allow_notconv=True)
    return st.as_dict()


class MG:
    """Handle around a ``wmg_ctx``: ``mg_setup`` on construction."""

    def __init__(self, L, U: torch.Tensor, m: float, Nv: int, block=(4, 4, 4, 4), params: Params | None = None):
        torch.cuda.synchronize()
        self.L = tuple(int(v) for v in L)
        self.params = params if params is not None else default_params()
        self.h = _vp()
        blk = (ctypes.c_int * 4)(*[int(b) for b in block])
        _check(_lib.mg_setup(ctypes.byref(_geom(self.L)), _ptr(U), float(m), int(Nv), ctypes.byref(blk),
                             ctypes.byref(self.params), ctypes.byref(self.h)))

    @classmethod
    def load(cls, path: str, L, U: torch.Tensor, m: float, params: Params | None = None) -> "MG":
        """mg_load: a context rebuilt from a saved setup for links U."""
        torch.cuda.synchronize()
        obj = cls.__new__(cls)
        obj.L = tuple(int(v) for v in L)
        obj.h = _vp()
        _check(_lib.mg_load(str(path).encode(), ctypes.byref(_geom(obj.L)), _ptr(U), float(m),
                            ctypes.byref(params) if params is not None else None, ctypes.byref(obj.h)))
        obj.params = params
        return obj

    def mg_save(self, path: str) -> None:
        _check(_lib.mg_save(self.h, str(path).encode()))

    def mg_refresh(self, U: torch.Tensor, iters: int) -> None:
        torch.cuda.synchronize()
        _check(_lib.mg_refresh(self.h, _ptr(U), int(iters)))

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            _lib.mg_destroy(self.h)
            self.h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def mg_solve(self, b: torch.Tensor, x: torch.Tensor, tol: float, nrhs: int | None = None) -> dict:
        torch.cuda.synchronize()
        if nrhs is None:
            nrhs = b.shape[0] if b.dim() == 3 else 1
        st = Stats()
        rc = _lib.mg_solve(self.h, _ptr(b), _ptr(x), float(tol), int(nrhs), ctypes.byref(st))
        _check(rc, allow_notconv=True)
        return st.as_dict()

    def mg_set_mass(self, m: float) -> None:
        _check(_lib.mg_set_mass(self.h, float(m)))

    def mg_set_precision(self, precision: int) -> None:
        _check(_lib.mg_set_precision(self.h, int(precision)))

    def level_info(self, level: int):
        L = (ctypes.c_int * 4)()
        dof = ctypes.c_int()
        nv = ctypes.c_int()
        _check(_lib.mg_level_info(self.h, int(level), ctypes.byref(L), ctypes.byref(dof), ctypes.byref(nv)))
        return tuple(L), dof.value, nv.value

    def mg_set_null_vectors(self, level: int, vecs: torch.Tensor) -> None:
        torch.cuda.synchronize()
        _check(_lib.mg_set_null_vectors(self.h, int(level), _ptr(vecs)))

    def mg_get_null_vectors(self, level: int, out: torch.Tensor) -> None:
        torch.cuda.synchronize()
        _check(_lib.mg_get_null_vectors(self.h, int(level), _ptr(out)))

    def mg_get_prolongator(self, level: int, out: torch.Tensor) -> None:
        torch.cuda.synchronize()
        _check(_lib.mg_get_prolongator(self.h, int(level), _ptr(out)))

    def mg_get_coarse_links(self, level: int, out: torch.Tensor) -> None:
        torch.cuda.synchronize()
        _check(_lib.mg_get_coarse_links(self.h, int(level), _ptr(out)))

    def mg_restrict(self, level: int, fine: torch.Tensor, coarse: torch.Tensor, nrhs: int = 1) -> None:
        torch.cuda.synchronize()
        _check(_lib.mg_restrict(self.h, int(level), _ptr(fine), _ptr(coarse), int(nrhs)))

    def mg_prolong(self, level: int, coarse: torch.Tensor, fine: torch.Tensor, nrhs: int = 1) -> None:
        torch.cuda.synchronize()
        _check(_lib.mg_prolong(self.h, int(level), _ptr(coarse), _ptr(fine), int(nrhs)))

    def mg_coarse_apply(self, level: int, inp: torch.Tensor, out: torch.Tensor, dagger: bool = False,
                        nrhs: int = 1) -> None:
        torch.cuda.synchronize()
        _check(_lib.mg_coarse_apply(self.h, int(level), _ptr(inp), _ptr(out), int(bool(dagger)), int(nrhs)))

    def mg_restrict_f32(self, level: int, fine: torch.Tensor, coarse: torch.Tensor, nrhs: int = 1) -> None:
        torch.cuda.synchronize()
        _check(_lib.mg_restrict_f32(self.h, int(level), _ptr(fine), _ptr(coarse), int(nrhs)))

    def mg_prolong_f32(self, level: int, coarse: torch.Tensor, fine: torch.Tensor, nrhs: int = 1) -> None:
        torch.cuda.synchronize()
        _check(_lib.mg_prolong_f32(self.h, int(level), _ptr(coarse), _ptr(fine), int(nrhs)))

    def mg_coarse_apply_f32(self, level: int, inp: torch.Tensor, out: torch.Tensor, dagger: bool = False,
                            nrhs: int = 1) -> None:
        torch.cuda.synchronize()
        _check(_lib.mg_coarse_apply_f32(self.h, int(level), _ptr(inp), _ptr(out), int(bool(dagger)), int(nrhs)))

    def mg_apply_fine(self, prec: int, inp: torch.Tensor, out: torch.Tensor, nrhs: int = 1) -> None:
        torch.cuda.synchronize()
        _check(_lib.mg_apply_fine(self.h, int(prec), _ptr(inp), _ptr(out), int(nrhs)))

    def mg_smoother_residual(self, r: torch.Tensor, e: torch.Tensor, out: torch.Tensor, nrhs: int = 1) -> None:
        torch.cuda.synchronize()
        _check(_lib.mg_smoother_residual(self.h, _ptr(r), _ptr(e), _ptr(out), int(nrhs)))

    def mg_hop_eo(self, prec: int, par: int, a: float, b: float, diag, hop: torch.Tensor, out: torch.Tensor,
                  nrhs: int = 1) -> None:
        torch.cuda.synchronize()
        _check(_lib.mg_hop_eo(self.h, int(prec), int(par), float(a), float(b), _ptr(diag) if diag is not None else None,
                              _ptr(hop), _ptr(out), int(nrhs)))

    def mg_link_reals(self) -> int:
        rc = _lib.mg_link_reals(self.h)
        if rc < 0:
            _check(rc)
        return rc

    def mg_cycle(self, r: torch.Tensor, z: torch.Tensor) -> None:
        torch.cuda.synchronize()
        _check(_lib.mg_cycle(self.h, _ptr(r), _ptr(z)))

    def mg_last_iters(self, nrhs: int):
        arr = (ctypes.c_int * nrhs)()
        _check(_lib.mg_last_iters(self.h, arr, int(nrhs)))
        return list(arr)

    def mg_profile(self, enable: bool) -> None:
        _check(_lib.mg_profile(self.h, int(bool(enable))))

    def mg_profile_get(self, kind: int):
        n = ctypes.c_int()
        ms = ctypes.c_double()
        by = ctypes.c_double()
        _check(_lib.mg_profile_get(self.h, int(kind), ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by)))
        return n.value, ms.value, by.value

    def mg_time_dslash(self, prec: int, nrhs: int = 1, reps: int = 20) -> float:
        ms = ctypes.c_double()
        _check(_lib.mg_time_dslash(self.h, int(prec), int(nrhs), int(reps), ctypes.byref(ms)))
        return ms.value


class MGBatch:
    """Uneven batch of independent lattice instances (``mg_setup_batch``)."""

    def __init__(self, Ls, Us, ms, Nv: int, block=(4, 4, 4, 4), params: Params | None = None):
        torch.cuda.synchronize()
        n = len(Ls)
        self.n = n
        self.params = params if params is not None else default_params()
        geoms = (Geom * n)(*[_geom(L) for L in Ls])
        uptr = (_vp * n)(*[_ptr(U) for U in Us])
        mass = (_d * n)(*[float(m) for m in ms])
        blk = (ctypes.c_int * 4)(*[int(b) for b in block])
        self.h = _vp()
        _check(_lib.mg_setup_batch(n, geoms, uptr, mass, int(Nv), ctypes.byref(blk), ctypes.byref(self.params),
                                   ctypes.byref(self.h)))

    def mg_solve_batch(self, bs, xs, tol: float):
        torch.cuda.synchronize()
        bp = (_vp * self.n)(*[_ptr(b) for b in bs])
        xp = (_vp * self.n)(*[_ptr(x) for x in xs])
        st = (Stats * self.n)()
        rc = _lib.mg_solve_batch(self.h, bp, xp, float(tol), st)
        _check(rc, allow_notconv=True)
        return [s.as_dict() for s in st]

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            _lib.mg_destroy(self.h)
            self.h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
