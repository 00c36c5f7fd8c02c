"""FP64 CPU oracle for adaptive-multigrid GCR on the Wilson-Dirac operator.

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the HIP library in ``paper_0912_2186_amd``; it is a second,
deliberately plain statement of the method (arXiv:0912.2186, Sec. 2-3) in
double precision, written as loops in ``oracle.c`` and wrapped here with
ctypes.  Every array is numpy complex128 in the canonical layouts:

* gauge field ``U[s, mu, a, b]``  (shape ``(V, 4, 3, 3)``)
* fine spinor ``psi[s, spin*3 + colour]``  (shape ``(V, 12)``)
* level vector ``v[s, dof]``; null vectors ``P[alpha, s, dof]``
* coarse links ``Y[xh, d, row, col]`` with ``d = 0`` local, ``1+mu`` forward,
  ``5+mu`` backward.

Site index ``s = x + Lx*(y + Ly*(z + Lz*t))``.  Parity of each function is
pinned by the ``-m "not gpu"`` oracle tests; the adaptive setup's vectors are
random and iterative, so they are pinned by a property (they lie in the
near-null space of a dense singular value decomposition), not value by value.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` with gcc (FP64, OpenMP) into ``liboracle.so``."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    return lib


_lib = _load()
_I4 = ctypes.c_int * 4
_dp = ctypes.POINTER(ctypes.c_double)


def _p(a: np.ndarray):
    assert a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _c(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.complex128)


def vol(L) -> int:
    return int(L[0] * L[1] * L[2] * L[3])


class MGParams(ctypes.Structure):
    """Mirror of the oracle's parameter block (defaults follow Sec. 3:
    4^4 blocks, GCR(8) outer, 4 post-smoothing steps, CG on the normal
    equations at the coarsest level, W-cycle for three levels)."""

    _fields_ = [
        ("nlevels", ctypes.c_int),
        ("block", ctypes.c_int * 8),
        ("nv", ctypes.c_int * 2),
        ("setup_iters", ctypes.c_int),
        ("post_smooth", ctypes.c_int),
        ("gcr_restart", ctypes.c_int),
        ("wcycle", ctypes.c_int),
        ("coarse_tol", ctypes.c_double),
        ("coarse_maxiter", ctypes.c_int),
        ("maxiter", ctypes.c_int),
        ("seed", ctypes.c_uint64),
        ("eo_smoother", ctypes.c_int),
        ("spin_parts", ctypes.c_int),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("outer_iters", ctypes.c_long),
        ("fine_matvecs", ctypes.c_long),
        ("coarse_iters", ctypes.c_long),
        ("restarts", ctypes.c_long),
        ("converged", ctypes.c_int),
        ("true_relres", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib.orc_mg_create.restype = ctypes.c_void_p
_lib.orc_mg_create.argtypes = [_I4, _dp, ctypes.c_double, ctypes.POINTER(MGParams)]
_lib.orc_mg_free.argtypes = [ctypes.c_void_p]
_lib.orc_mg_setup.argtypes = [ctypes.c_void_p]
_lib.orc_mg_set_null_vectors.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp]
_lib.orc_mg_set_mass.argtypes = [ctypes.c_void_p, ctypes.c_double]
_lib.orc_mg_solve.restype = ctypes.c_long
_lib.orc_mg_solve.argtypes = [ctypes.c_void_p, _dp, _dp, ctypes.c_double, ctypes.POINTER(Stats)]
_lib.orc_mg_solve_eo.restype = ctypes.c_long
_lib.orc_mg_solve_eo.argtypes = [ctypes.c_void_p, _dp, _dp, ctypes.c_double, ctypes.POINTER(Stats)]
_lib.orc_mg_cycle.argtypes = [ctypes.c_void_p, _dp, _dp]
_lib.orc_mg_level_info.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                   ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
_lib.orc_mg_get_P.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp]
_lib.orc_mg_get_Y.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp]
_lib.orc_mg_get_null_vectors.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp]
_lib.orc_bicgstab.restype = ctypes.c_long
_lib.orc_bicgstab.argtypes = [_I4, _dp, ctypes.c_double, _dp, _dp, ctypes.c_double, ctypes.c_int,
                              ctypes.POINTER(ctypes.c_double)]
_lib.orc_block_orthonormalize.restype = ctypes.c_int
_lib.orc_block_orthonormalize_ns.restype = ctypes.c_int
_lib.orc_num_threads.restype = ctypes.c_int


def num_threads() -> int:
    return int(_lib.orc_num_threads())


def set_num_threads(n: int) -> None:
    """Thread count of the oracle's OpenMP loops from now on (timing only)."""
    _lib.orc_set_num_threads(ctypes.c_int(int(n)))


def gamma(mu: int) -> np.ndarray:
    out = np.zeros((4, 4), np.complex128)
    _lib.orc_gamma(ctypes.c_int(mu), _p(out))
    return out


def wilson(L, U, m: float, psi) -> np.ndarray:
    """Eq. 2.2: D(U) psi, full operator with the (4+m) diagonal."""
    U = _c(U)
    psi = _c(psi)
    V = vol(L)
    assert U.size == V * 36 and psi.size == V * 12
    out = np.empty_like(psi)
    _lib.orc_wilson(_I4(*L), _p(U), ctypes.c_double(m), _p(psi), _p(out))
    return out


def parity(L) -> np.ndarray:
    """Site parity (x+y+z+t) mod 2 of every site, canonical order."""
    s = np.arange(vol(L))
    x = s % L[0]
    y = (s // L[0]) % L[1]
    z = (s // (L[0] * L[1])) % L[2]
    t = s // (L[0] * L[1] * L[2])
    return (x + y + z + t) & 1


def wilson_hop_parity(L, U, m: float, psi, par: int) -> np.ndarray:
    """D_{par,1-par} psi: hopping terms at sites of parity par from psi at
    the other parity; zero elsewhere."""
    U = _c(U)
    psi = _c(psi)
    out = np.empty_like(psi)
    _lib.orc_wilson_hop_parity(_I4(*L), _p(U), ctypes.c_double(m), _p(psi), _p(out), ctypes.c_int(par))
    return out


def schur_apply(L, U, m: float, psi) -> np.ndarray:
    """S psi_e = (4+m) psi_e - D_eo D_oe psi_e / (4+m) on the even sites
    (odd sites of psi ignored, of the result zero)."""
    U = _c(U)
    psi = _c(psi)
    out = np.empty_like(psi)
    _lib.orc_schur_apply(_I4(*L), _p(U), ctypes.c_double(m), _p(psi), _p(out))
    return out


def coarse_apply(Lc, dof: int, Y, v, dagger: bool = False) -> np.ndarray:
    """Coarse 9-point stencil D_hat v (or its adjoint, written out)."""
    Y = _c(Y)
    v = _c(v)
    assert Y.size == vol(Lc) * 9 * dof * dof and v.size == vol(Lc) * dof
    out = np.empty_like(v)
    _lib.orc_coarse_apply(_I4(*Lc), ctypes.c_int(dof), _p(Y), _p(v), _p(out), ctypes.c_int(int(dagger)))
    return out


def block_orthonormalize_ns(L, dof: int, block, vecs, ns: int) -> np.ndarray:
    """Eq. 2.7 with the per-site components split into ns parts (2:
    chirality, 4: Dirac spin)."""
    vecs = _c(vecs)
    P = np.empty_like(vecs)
    rc = _lib.orc_block_orthonormalize_ns(_I4(*L), ctypes.c_int(dof), _I4(*block), ctypes.c_int(vecs.shape[0]),
                                          ctypes.c_int(ns), _p(vecs), _p(P))
    if rc != 0:
        raise RuntimeError("block Gram-Schmidt breakdown")
    return P


def restrict_ns(L, dof: int, block, P, fine, ns: int) -> np.ndarray:
    P = _c(P)
    fine = _c(fine)
    Lc = coarse_dims(L, block)
    out = np.empty((vol(Lc), ns * P.shape[0]), np.complex128)
    _lib.orc_restrict_ns(_I4(*L), ctypes.c_int(dof), _I4(*block), ctypes.c_int(P.shape[0]), ctypes.c_int(ns), _p(P),
                         _p(fine), _p(out))
    return out


def prolong_ns(L, dof: int, block, P, coarse, ns: int) -> np.ndarray:
    P = _c(P)
    coarse = _c(coarse)
    out = np.empty((vol(L), dof), np.complex128)
    _lib.orc_prolong_ns(_I4(*L), ctypes.c_int(dof), _I4(*block), ctypes.c_int(P.shape[0]), ctypes.c_int(ns), _p(P),
                        _p(coarse), _p(out))
    return out


def coarse_build_wilson_ns(L, U, m: float, block, P, ns: int) -> np.ndarray:
    """Galerkin P^dag D P of the Wilson operator with ns parts per site."""
    U = _c(U)
    P = _c(P)
    Lc = coarse_dims(L, block)
    n = ns * P.shape[0]
    Y = np.empty((vol(Lc), 9, n, n), np.complex128)
    _lib.orc_coarse_build_ns(_I4(*L), ctypes.c_int(0), ctypes.c_int(12), _p(U), ctypes.c_double(m), ctypes.cast(None, _dp),
                             _I4(*block), ctypes.c_int(P.shape[0]), ctypes.c_int(ns), _p(P), _p(Y))
    return Y


def block_orthonormalize(L, dof: int, block, vecs) -> np.ndarray:
    """Eq. 2.7 with the chirality split of Sec. 3: per (block, chirality),
    orthonormal basis of the restricted vectors (MGS twice, diag(R) > 0)."""
    vecs = _c(vecs)
    out = np.empty_like(vecs)
    nv = vecs.shape[0]
    rc = _lib.orc_block_orthonormalize(_I4(*L), ctypes.c_int(dof), _I4(*block), ctypes.c_int(nv),
                                       _p(vecs), _p(out))
    if rc != 0:
        raise np.linalg.LinAlgError("block Gram-Schmidt rank breakdown")
    return out


def coarse_dims(L, block):
    return tuple(int(L[i] // block[i]) for i in range(4))


def restrict(L, dof: int, block, P, fine) -> np.ndarray:
    """r_hat = P^dag r (coarse dof ordered (chi, alpha))."""
    P = _c(P)
    fine = _c(fine)
    nv = P.shape[0]
    out = np.empty((vol(coarse_dims(L, block)), 2 * nv), np.complex128)
    _lib.orc_restrict(_I4(*L), ctypes.c_int(dof), _I4(*block), ctypes.c_int(nv), _p(P), _p(fine), _p(out))
    return out


def prolong(L, dof: int, block, P, coarse) -> np.ndarray:
    """e = P e_hat (Eq. 2.3)."""
    P = _c(P)
    coarse = _c(coarse)
    nv = P.shape[0]
    out = np.empty((vol(L), dof), np.complex128)
    _lib.orc_prolong(_I4(*L), ctypes.c_int(dof), _I4(*block), ctypes.c_int(nv), _p(P), _p(coarse), _p(out))
    return out


def coarse_build_wilson(L, U, m: float, block, P) -> np.ndarray:
    """Galerkin D_hat = P^dag D(U) P as a 9-point stencil (Sec. 2)."""
    U = _c(U)
    P = _c(P)
    nv = P.shape[0]
    Vc = vol(coarse_dims(L, block))
    Y = np.zeros((Vc, 9, 2 * nv, 2 * nv), np.complex128)
    _lib.orc_coarse_build(_I4(*L), ctypes.c_int(0), ctypes.c_int(12), _p(U), ctypes.c_double(m),
                          ctypes.cast(None, _dp), _I4(*block), ctypes.c_int(nv), _p(P), _p(Y))
    return Y


def coarse_build_coarse(L, dof: int, Yf, block, P) -> np.ndarray:
    """Galerkin coarsening of a coarse stencil (third level)."""
    Yf = _c(Yf)
    P = _c(P)
    nv = P.shape[0]
    Vc = vol(coarse_dims(L, block))
    Y = np.zeros((Vc, 9, 2 * nv, 2 * nv), np.complex128)
    _lib.orc_coarse_build(_I4(*L), ctypes.c_int(1), ctypes.c_int(dof), ctypes.cast(None, _dp),
                          ctypes.c_double(0.0), _p(Yf), _I4(*block), ctypes.c_int(nv), _p(P), _p(Y))
    return Y


def philox4x32_10(ctr, key):
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    _lib.orc_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def start_vector(nsite: int, dof: int, seed: int, level: int, alpha: int) -> np.ndarray:
    out = np.empty((nsite, dof), np.complex128)
    _lib.orc_start_vector(ctypes.c_long(nsite), ctypes.c_int(dof), ctypes.c_uint64(seed), ctypes.c_int(level),
                          ctypes.c_int(alpha), _p(out))
    return out


def bicgstab(L, U, m: float, b, tol: float, maxiter: int = 100000):
    """Plain BiCGStab on D x = b from x0 = 0; returns (x, iters, relres)."""
    U = _c(U)
    b = _c(b)
    x = np.zeros_like(b)
    rr = ctypes.c_double()
    it = _lib.orc_bicgstab(_I4(*L), _p(U), ctypes.c_double(m), _p(b), _p(x), ctypes.c_double(tol),
                           ctypes.c_int(maxiter), ctypes.byref(rr))
    return x, int(it), float(rr.value)


def default_params(**kw) -> MGParams:
    p = MGParams()
    p.nlevels = 2
    for i in range(8):
        p.block[i] = 4
    p.nv[0] = 24
    p.nv[1] = 32
    p.setup_iters = 5
    p.post_smooth = 4
    p.gcr_restart = 8
    p.wcycle = 1
    p.coarse_tol = 1e-8
    p.coarse_maxiter = 500
    p.maxiter = 1000
    p.seed = 12345
    p.eo_smoother = 0
    p.spin_parts = 2
    for k, v in kw.items():
        if k == "block":
            flat = list(v[0]) + list(v[1] if len(v) > 1 else v[0])
            for i in range(8):
                p.block[i] = int(flat[i])
        elif k == "nv":
            p.nv[0] = int(v[0])
            p.nv[1] = int(v[1] if len(v) > 1 else v[0])
        else:
            setattr(p, k, v)
    return p


class MG:
    """Oracle multigrid hierarchy: adaptive setup + MG-preconditioned GCR."""

    def __init__(self, L, U, m: float, params: MGParams):
        self.L = tuple(int(v) for v in L)
        self.U = _c(U)
        self.params = params
        self.h = _lib.orc_mg_create(_I4(*self.L), _p(self.U), ctypes.c_double(m), ctypes.byref(params))
        if not self.h:
            raise MemoryError("oracle MG create failed")

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            _lib.orc_mg_free(ctypes.c_void_p(h))
            self.h = None

    def setup(self):
        rc = _lib.orc_mg_setup(ctypes.c_void_p(self.h))
        if rc != 0:
            raise RuntimeError("oracle setup failed: %d" % rc)

    def set_null_vectors(self, level: int, vecs):
        vecs = _c(vecs)
        rc = _lib.orc_mg_set_null_vectors(ctypes.c_void_p(self.h), ctypes.c_int(level), _p(vecs))
        if rc != 0:
            raise RuntimeError("oracle set_null_vectors failed: %d" % rc)

    def set_mass(self, m: float):
        _lib.orc_mg_set_mass(ctypes.c_void_p(self.h), ctypes.c_double(m))

    def level_info(self, level: int):
        L = (ctypes.c_int * 4)()
        dof = ctypes.c_int()
        nv = ctypes.c_int()
        rc = _lib.orc_mg_level_info(ctypes.c_void_p(self.h), ctypes.c_int(level), L, ctypes.byref(dof),
                                    ctypes.byref(nv))
        if rc != 0:
            raise IndexError(level)
        return tuple(L), dof.value, nv.value

    def P(self, level: int) -> np.ndarray:
        L, dof, nv = self.level_info(level)
        out = np.empty((nv, vol(L), dof), np.complex128)
        _lib.orc_mg_get_P(ctypes.c_void_p(self.h), ctypes.c_int(level), _p(out))
        return out

    def null_vectors(self, level: int) -> np.ndarray:
        """Adapted null vectors of a level before block orthonormalisation."""
        L, dof, nv = self.level_info(level)
        out = np.empty((nv, vol(L), dof), np.complex128)
        _lib.orc_mg_get_null_vectors(ctypes.c_void_p(self.h), ctypes.c_int(level), _p(out))
        return out

    def Y(self, level: int) -> np.ndarray:
        L, dof, _ = self.level_info(level)
        out = np.empty((vol(L), 9, dof, dof), np.complex128)
        _lib.orc_mg_get_Y(ctypes.c_void_p(self.h), ctypes.c_int(level), _p(out))
        return out

    def cycle(self, r) -> np.ndarray:
        r = _c(r)
        z = np.zeros_like(r)
        _lib.orc_mg_cycle(ctypes.c_void_p(self.h), _p(r), _p(z))
        return z

    def solve(self, b, tol: float):
        b = _c(b)
        x = np.zeros_like(b)
        st = Stats()
        _lib.orc_mg_solve(ctypes.c_void_p(self.h), _p(b), _p(x), ctypes.c_double(tol), ctypes.byref(st))
        return x, st.as_dict()

    def solve_eo(self, b, tol: float):
        """Red/black solve: GCR on the even-site Schur complement,
        preconditioned with the multigrid cycle of the full operator."""
        b = _c(b)
        x = np.zeros_like(b)
        st = Stats()
        _lib.orc_mg_solve_eo(ctypes.c_void_p(self.h), _p(b), _p(x), ctypes.c_double(tol), ctypes.byref(st))
        return x, st.as_dict()


for _name, _args in [
    ("orc_wilson", [_I4, _dp, ctypes.c_double, _dp, _dp]),
    ("orc_coarse_apply", [_I4, ctypes.c_int, _dp, _dp, _dp, ctypes.c_int]),
    ("orc_block_orthonormalize", [_I4, ctypes.c_int, _I4, ctypes.c_int, _dp, _dp]),
    ("orc_restrict", [_I4, ctypes.c_int, _I4, ctypes.c_int, _dp, _dp, _dp]),
    ("orc_prolong", [_I4, ctypes.c_int, _I4, ctypes.c_int, _dp, _dp, _dp]),
    ("orc_coarse_build", [_I4, ctypes.c_int, ctypes.c_int, _dp, ctypes.c_double, _dp, _I4, ctypes.c_int, _dp, _dp]),
    ("orc_gamma", [ctypes.c_int, _dp]),
    ("orc_wilson_hop_parity", [_I4, _dp, ctypes.c_double, _dp, _dp, ctypes.c_int]),
    ("orc_block_orthonormalize_ns", [_I4, ctypes.c_int, _I4, ctypes.c_int, ctypes.c_int, _dp, _dp]),
    ("orc_restrict_ns", [_I4, ctypes.c_int, _I4, ctypes.c_int, ctypes.c_int, _dp, _dp, _dp]),
    ("orc_prolong_ns", [_I4, ctypes.c_int, _I4, ctypes.c_int, ctypes.c_int, _dp, _dp, _dp]),
    ("orc_coarse_build_ns", [_I4, ctypes.c_int, ctypes.c_int, _dp, ctypes.c_double, _dp, _I4, ctypes.c_int,
                             ctypes.c_int, _dp, _dp]),
    ("orc_schur_apply", [_I4, _dp, ctypes.c_double, _dp, _dp]),
    ("orc_start_vector", [ctypes.c_long, ctypes.c_int, ctypes.c_uint64, ctypes.c_int, ctypes.c_int, _dp]),
]:
    getattr(_lib, _name).argtypes = _args

_lib.orc_cgnr_coarse.restype = ctypes.c_long
_lib.orc_cgnr_coarse.argtypes = [_I4, ctypes.c_int, _dp, _dp, _dp, ctypes.c_double, ctypes.c_int]
_lib.orc_mr_wilson.argtypes = [_I4, _dp, ctypes.c_double, _dp, _dp, ctypes.c_int, _dp]


def cgnr_coarse(Lc, dof: int, Y, b, tol: float, maxiter: int = 10000):
    """CG on the normal equations of a coarse stencil; returns (x, iters)."""
    Y = _c(Y)
    b = _c(b)
    x = np.zeros_like(b)
    it = _lib.orc_cgnr_coarse(_I4(*Lc), ctypes.c_int(dof), _p(Y), _p(b), _p(x), ctypes.c_double(tol),
                              ctypes.c_int(maxiter))
    return x, int(it)


def mr_wilson(L, U, m: float, r, e0, nsteps: int):
    """MR smoothing steps on D e = r from e0; returns (e, residual norms)."""
    U = _c(U)
    r = _c(r)
    e = _c(e0).copy()
    res = np.zeros(nsteps + 1)
    _lib.orc_mr_wilson(_I4(*L), _p(U), ctypes.c_double(m), _p(r), _p(e), ctypes.c_int(nsteps), _p(res))
    return e, res
