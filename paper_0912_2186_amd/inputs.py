"""Seeded synthetic inputs: gauge fields and right-hand sides.

These generators stand in for the paper's beta = 5.5 Wilson ensembles
(arXiv:0912.2186, Fig. 2 and Table 1), which are not available.  They hold
none of the method's arithmetic and serve both the HIP path and the oracle.

* gauge field: U = exp(i eps H) per link, H = sum_a h_a lambda_a / 2 with
  Gell-Mann lambda_a and h_a ~ N(0, 1) i.i.d., drawn from numpy's PCG64 in
  canonical order (t, z, y, x, mu, a).  Shape (V, 4, 3, 3) complex128.
* right-hand sides: Gaussian (re, im ~ N(0,1)), spin-colour point sources,
  Z4 noise (each component uniform in {1, i, -1, -i}).  Shape (V, 12).

Canonical site index s = x + Lx*(y + Ly*(z + Lz*t)).
"""
from __future__ import annotations

import numpy as np

_GELL_MANN = np.zeros((8, 3, 3), np.complex128)
_GELL_MANN[0][0, 1] = _GELL_MANN[0][1, 0] = 1
_GELL_MANN[1][0, 1] = -1j
_GELL_MANN[1][1, 0] = 1j
_GELL_MANN[2][0, 0] = 1
_GELL_MANN[2][1, 1] = -1
_GELL_MANN[3][0, 2] = _GELL_MANN[3][2, 0] = 1
_GELL_MANN[4][0, 2] = -1j
_GELL_MANN[4][2, 0] = 1j
_GELL_MANN[5][1, 2] = _GELL_MANN[5][2, 1] = 1
_GELL_MANN[6][1, 2] = -1j
_GELL_MANN[6][2, 1] = 1j
_GELL_MANN[7][0, 0] = _GELL_MANN[7][1, 1] = 1 / np.sqrt(3)
_GELL_MANN[7][2, 2] = -2 / np.sqrt(3)


def gell_mann() -> np.ndarray:
    return _GELL_MANN.copy()


def volume(L) -> int:
    return int(L[0] * L[1] * L[2] * L[3])


def gauge_field(L, eps: float, seed: int, chunk_sites: int = 1 << 18) -> np.ndarray:
    """SU(3) links U = exp(i eps H), H Gaussian traceless Hermitian."""
    import torch

    V = volume(L)
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.empty((V, 4, 3, 3), np.complex128)
    lam = torch.from_numpy(_GELL_MANN / 2)
    for s0 in range(0, V, chunk_sites):
        n = min(chunk_sites, V - s0)
        h = rng.standard_normal((n, 4, 8))
        H = torch.einsum("sma,aij->smij", torch.from_numpy(h).to(torch.complex128), lam)
        out[s0:s0 + n] = torch.linalg.matrix_exp(1j * eps * H).numpy()
    return out


def unit_gauge(L) -> np.ndarray:
    V = volume(L)
    U = np.zeros((V, 4, 3, 3), np.complex128)
    U[:, :, 0, 0] = U[:, :, 1, 1] = U[:, :, 2, 2] = 1
    return U


def gaussian_rhs(L, seed: int, nrhs: int = 1) -> np.ndarray:
    """nrhs Gaussian complex spinors, shape (nrhs, V, 12)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    V = volume(L)
    re = rng.standard_normal((nrhs, V, 12))
    im = rng.standard_normal((nrhs, V, 12))
    return re + 1j * im


def point_sources(L, site: int = 0) -> np.ndarray:
    """The 12 spin-colour point sources at one site, shape (12, V, 12)."""
    V = volume(L)
    b = np.zeros((12, V, 12), np.complex128)
    for k in range(12):
        b[k, site, k] = 1.0
    return b


def z4_noise(L, seed: int, nrhs: int) -> np.ndarray:
    """Z4 noise vectors, every component uniform in {1, i, -1, -i}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    V = volume(L)
    k = rng.integers(0, 4, size=(nrhs, V, 12))
    return (1j ** k).astype(np.complex128)


def random_su3(n: int, seed: int) -> np.ndarray:
    """n Haar-ish SU(3) matrices (for gauge transformations in tests)."""
    import torch

    rng = np.random.Generator(np.random.PCG64(seed))
    h = rng.standard_normal((n, 8))
    H = torch.einsum("sa,aij->sij", torch.from_numpy(h).to(torch.complex128), torch.from_numpy(_GELL_MANN / 2))
    return torch.linalg.matrix_exp(1j * 2.0 * H).numpy()
