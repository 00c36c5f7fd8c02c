"""Pins of the oracle's full-spin-structure coarsening (Sec. 3: the variant
that exposes the full Dirac spin structure on the coarse blocks, not just
the chiral one): each null vector's restriction to a block is split into
its four spin parts instead of its two chiralities, giving 4 N_nu coarse
degrees of freedom per block, ordered (spin, vector).

* block Gram-Schmidt per (block, spin) equals numpy's QR;
* every column lives in one spin, so gamma_5 P = P gamma_5_hat with
  gamma_5_hat = +1 on spins 0, 1 and -1 on spins 2, 3 (the first and second
  half of the coarse dof, as for the chirality split);
* the Galerkin stencil equals the dense P^dag D P and stays
  gamma_5_hat-hermitian;
* free field with the three colour vectors constant over sites and spins:
  D_hat = (1/b) D_W(m b) on the coarse lattice, the closed form derived
  from Eq. 2.2 + Eq. 2.4;
* the spin split of a set of vectors contains the chirality split of the
  same vectors (projector identity), and the MG solve built on it converges
  in no more outer iterations.
"""
import numpy as np
import pytest

import oracle
from paper_0912_2186_amd import inputs
from helpers import dense_from_apply, dense_stencil, relerr, vol


def rand_vecs(nv, V, dof, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((nv, V, dof)) + 1j * rng.standard_normal((nv, V, dof))


def dense_P_ns(L, dof, block, P, ns):
    """Dense prolongator with column (xh, part, alpha) = P[alpha] on block
    xh and on the components of that part (dof/ns consecutive ones)."""
    V = vol(L)
    nv = P.shape[0]
    Lc = oracle.coarse_dims(L, block)
    h = dof // ns
    M = np.zeros((V * dof, vol(Lc) * ns * nv), np.complex128)
    for s in range(V):
        x = [0] * 4
        t = s
        for mu in range(4):
            x[mu] = t % L[mu]
            t //= L[mu]
        xc = [x[mu] // block[mu] for mu in range(4)]
        xh = xc[0] + Lc[0] * (xc[1] + Lc[1] * (xc[2] + Lc[2] * xc[3]))
        for c in range(dof):
            for a in range(nv):
                M[s * dof + c, xh * ns * nv + (c // h) * nv + a] = P[a, s, c]
    return M


def test_spin_block_gram_schmidt_matches_qr():
    L, block, nv = (4, 4, 4, 4), (2, 2, 2, 2), 4
    vecs = rand_vecs(nv, vol(L), 12, 71)
    P = oracle.block_orthonormalize_ns(L, 12, block, vecs, 4)
    Pd = dense_P_ns(L, 12, block, P, 4)
    Vd = dense_P_ns(L, 12, block, vecs, 4)
    assert np.abs(Pd.conj().T @ Pd - np.eye(Pd.shape[1])).max() < 1e-13
    for q in range(Pd.shape[1] // nv):
        cols = slice(q * nv, (q + 1) * nv)
        rows = np.nonzero(np.abs(Vd[:, cols]).sum(1))[0]
        Q, R = np.linalg.qr(Vd[rows, cols])
        Q = Q * (np.diag(R) / np.abs(np.diag(R)))[None, :]
        assert np.abs(Q - Pd[rows, cols]).max() < 1e-13
    # every column in one spin: gamma_5 P = P gamma_5_hat
    g5 = np.tile(np.array([1.0] * 6 + [-1.0] * 6), vol(L))
    g5h = np.tile(np.array([1.0] * (2 * nv) + [-1.0] * (2 * nv)), Pd.shape[1] // (4 * nv))
    assert np.abs(g5[:, None] * Pd - Pd * g5h[None, :]).max() == 0
    spin = np.tile(np.repeat(np.arange(4), 3), vol(L))
    part = np.tile(np.repeat(np.arange(4), nv), Pd.shape[1] // (4 * nv))
    nz = np.nonzero(Pd)
    assert np.array_equal(spin[nz[0]], part[nz[1]])


@pytest.mark.parametrize("L,block,nv", [((4, 4, 4, 4), (2, 2, 2, 2), 2), ((4, 4, 2, 4), (4, 2, 2, 4), 2)])
def test_spin_galerkin_dense(L, block, nv):
    V = vol(L)
    U = inputs.gauge_field(L, 0.5, 72)
    m = -0.2
    P = oracle.block_orthonormalize_ns(L, 12, block, rand_vecs(nv, V, 12, 73), 4)
    Y = oracle.coarse_build_wilson_ns(L, U, m, block, P, 4)
    D = dense_from_apply(12 * V, lambda e: oracle.wilson(L, U, m, e.reshape(V, 12)))
    Pd = dense_P_ns(L, 12, block, P, 4)
    Lc = oracle.coarse_dims(L, block)
    n = 4 * nv
    Dh = dense_stencil(Lc, n, Y)
    assert np.abs(Dh - Pd.conj().T @ D @ Pd).max() < 1e-12
    s3 = np.tile(np.array([1.0] * (n // 2) + [-1.0] * (n // 2)), vol(Lc))
    assert np.abs(s3[:, None] * Dh * s3[None, :] - Dh.conj().T).max() < 1e-12
    # restriction and prolongation are P^dag and P
    rng = np.random.default_rng(74)
    f = rng.standard_normal((V, 12)) + 1j * rng.standard_normal((V, 12))
    c = oracle.restrict_ns(L, 12, block, P, f, 4)
    assert relerr(c.ravel(), Pd.conj().T @ f.ravel()) < 1e-14
    assert relerr(oracle.prolong_ns(L, 12, block, P, c, 4).ravel(), Pd @ c.ravel()) < 1e-14


@pytest.mark.parametrize("L,b", [((8, 8, 8, 8), 4), ((4, 4, 4, 8), 2)])
def test_spin_free_field_closed_form(L, b):
    """U = 1, three vectors constant over sites and spins (one per colour):
    split by spin on b^4 blocks they are the piecewise-constant prolongator
    of Eq. 2.4 on all 12 components, ordered (spin, colour) like the fine
    components, and P^dag D(m) P = (1/b) D_W(m b)."""
    V = vol(L)
    U = inputs.unit_gauge(L)
    vecs = np.zeros((3, V, 12), np.complex128)
    for c in range(3):
        for s in range(4):
            vecs[c, :, 3 * s + c] = 1
    block = (b, b, b, b)
    P = oracle.block_orthonormalize_ns(L, 12, block, vecs, 4)
    assert np.allclose(np.abs(P[P != 0]), 1 / b ** 2)
    m = -0.3
    Y = oracle.coarse_build_wilson_ns(L, U, m, block, P, 4)
    g = [oracle.gamma(mu) for mu in range(4)]
    I3 = np.eye(3)
    assert np.abs(Y[:, 0] - (m + 4 / b) * np.eye(12)).max() < 1e-13
    for mu in range(4):
        assert np.abs(Y[:, 1 + mu] - (-(1 / (2 * b)) * np.kron(np.eye(4) - g[mu], I3))).max() < 1e-13
        assert np.abs(Y[:, 5 + mu] - (-(1 / (2 * b)) * np.kron(np.eye(4) + g[mu], I3))).max() < 1e-13


def test_spin_split_contains_chirality_split():
    L, block, nv = (4, 4, 4, 4), (2, 2, 2, 2), 3
    vecs = rand_vecs(nv, vol(L), 12, 75)
    Pc = dense_P_ns(L, 12, block, oracle.block_orthonormalize(L, 12, block, vecs), 2)
    Ps = dense_P_ns(L, 12, block, oracle.block_orthonormalize_ns(L, 12, block, vecs, 4), 4)
    assert np.abs(Ps @ (Ps.conj().T @ Pc) - Pc).max() < 1e-12


def test_spin_split_mg_solve():
    """8^4, eps 0.3, m = -0.1: the same 6 adapted vectors split by spin (24
    coarse dof) and by chirality (12): both solves reach 1e-10, the spin
    split in no more outer iterations."""
    L = (8, 8, 8, 8)
    U = inputs.gauge_field(L, 0.3, 101)
    b = inputs.gaussian_rhs(L, 110)[0]
    p = oracle.default_params(nlevels=2, nv=(6,), setup_iters=10, seed=150)
    mg = oracle.MG(L, U, -0.1, p)
    mg.setup()
    vecs = mg.null_vectors(0)
    x, st = mg.solve(b, 1e-10)
    ps = oracle.default_params(nlevels=2, nv=(6,), seed=150, spin_parts=4)
    mg4 = oracle.MG(L, U, -0.1, ps)
    mg4.set_null_vectors(0, vecs)
    assert mg4.level_info(1)[1] == 24
    x4, st4 = mg4.solve(b, 1e-10)
    print("outer iterations: chirality split", st["outer_iters"], "spin split", st4["outer_iters"])
    for xx, ss in ((x, st), (x4, st4)):
        assert ss["converged"]
        assert np.linalg.norm(b - oracle.wilson(L, U, -0.1, xx)) / np.linalg.norm(b) <= 1e-10 * 1.0001
    assert st4["outer_iters"] <= st["outer_iters"]
