"""Small test helpers (dense assembly of operators from matrix-free applies)."""
import numpy as np


def vol(L):
    return int(L[0] * L[1] * L[2] * L[3])


def dense_from_apply(n, apply):
    """Dense matrix of a linear map given as apply(vector) -> vector."""
    M = np.zeros((n, n), np.complex128)
    e = np.zeros(n, np.complex128)
    for j in range(n):
        e[:] = 0
        e[j] = 1
        M[:, j] = apply(e).reshape(-1)
    return M


def dense_P(L, dof, block, P):
    """Dense prolongator (fine n x coarse n) built column by column from the
    chirality-split block structure: column (xh, chi, alpha) is P[alpha]
    restricted to block xh and to the chi half of the per-site components."""
    V = vol(L)
    nv = P.shape[0]
    Lc = tuple(L[i] // block[i] for i in range(4))
    Vc = vol(Lc)
    h = dof // 2
    M = np.zeros((V * dof, Vc * 2 * nv), np.complex128)
    for s in range(V):
        x = [0] * 4
        t = s
        for mu in range(4):
            x[mu] = t % L[mu]
            t //= L[mu]
        xc = [x[mu] // block[mu] for mu in range(4)]
        xh = xc[0] + Lc[0] * (xc[1] + Lc[1] * (xc[2] + Lc[2] * xc[3]))
        for c in range(dof):
            chi = c // h
            for a in range(nv):
                M[s * dof + c, xh * 2 * nv + chi * nv + a] = P[a, s, c]
    return M


def dense_stencil(Lc, dof, Y):
    """Dense matrix of a 9-point coarse stencil (periodic; forward and
    backward links that land on the same site are summed)."""
    Vc = vol(Lc)
    M = np.zeros((Vc * dof, Vc * dof), np.complex128)
    for s in range(Vc):
        x = [0] * 4
        t = s
        for mu in range(4):
            x[mu] = t % Lc[mu]
            t //= Lc[mu]

        def idx(y):
            return y[0] + Lc[0] * (y[1] + Lc[1] * (y[2] + Lc[2] * y[3]))

        M[s * dof:(s + 1) * dof, s * dof:(s + 1) * dof] += Y[s, 0]
        for mu in range(4):
            for sg, d in ((1, 1 + mu), (-1, 5 + mu)):
                y = list(x)
                y[mu] = (y[mu] + sg) % Lc[mu]
                t = idx(y)
                M[s * dof:(s + 1) * dof, t * dof:(t + 1) * dof] += Y[s, d]
    return M


def relerr(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def site_max(v, L):
    """Largest |re|, |im| over the 12 components of each site: shape (Lt, Lz, Ly, Lx)."""
    v = np.asarray(v).reshape(vol(L), -1)
    m = np.maximum(np.abs(v.real), np.abs(v.imag)).max(axis=1)
    return m.reshape(L[3], L[2], L[1], L[0])


def neighbourhood_scale(inp, L):
    """For every site, the largest component of inp over the site and its 8
    nearest neighbours (the inputs a Wilson operator reads there)."""
    m = site_max(inp, L)
    sc = m.copy()
    for ax in range(4):
        for sh in (1, -1):
            sc = np.maximum(sc, np.roll(m, sh, axis=ax))
    return sc.reshape(-1)


def local_err(out, ref, inp, L, floor=0.0):
    """max over sites of (largest component error at the site) divided by
    max(neighbourhood scale of the operator's input there, floor): a
    per-site bound that a few wrong sites cannot hide, unlike a global norm."""
    d = site_max(np.asarray(out) - np.asarray(ref), L).reshape(-1)
    sc = np.maximum(neighbourhood_scale(inp, L), floor)
    return float(np.max(d / np.maximum(sc, 1e-300)))
