"""Pins of the oracle's multigrid pieces (Sec. 2-3): block orthonormalisation
(Eq. 2.7) against numpy's QR, the chirality split (sigma_3 P = P gamma_5),
the Galerkin coarse operator P^dag D P against brute-force dense algebra and
against the free-field closed form derived from Eq. 2.2 + Eq. 2.4, the
coarse-correction projector of Eq. 2.5, and the solvers against dense
solves and their defining monotonicity properties."""
import numpy as np
import pytest

import oracle
from paper_0912_2186_amd import inputs
from helpers import dense_from_apply, dense_P, dense_stencil, relerr, vol


def rand_vecs(nv, V, dof, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((nv, V, dof)) + 1j * rng.standard_normal((nv, V, dof))


@pytest.mark.parametrize("L,block,nv", [((4, 4, 4, 4), (2, 2, 2, 2), 5), ((4, 2, 2, 4), (4, 2, 2, 2), 3)])
def test_block_gram_schmidt_matches_qr(L, block, nv):
    V = vol(L)
    vecs = rand_vecs(nv, V, 12, 1)
    P = oracle.block_orthonormalize(L, 12, block, vecs)
    Pd = dense_P(L, 12, block, P)
    Vd = dense_P(L, 12, block, vecs)
    # P^dag P = 1
    assert np.abs(Pd.conj().T @ Pd - np.eye(Pd.shape[1])).max() < 1e-13
    # per (block, chirality): columns equal numpy's Q with positive diag(R)
    nc = Pd.shape[1] // (2 * nv)
    for q in range(nc * 2):
        cols = slice(q * nv, (q + 1) * nv)
        rows = np.nonzero(np.abs(Vd[:, cols]).sum(1))[0]
        Q, R = np.linalg.qr(Vd[rows, cols])
        ph = np.diag(R) / np.abs(np.diag(R))
        Q = Q * ph[None, :]
        assert np.abs(Q - Pd[rows, cols]).max() < 1e-13
        assert np.abs(Pd[np.setdiff1d(np.arange(Pd.shape[0]), rows), cols]).max() == 0


def test_chirality_split():
    """sigma_3 P = P gamma_5: every column lives in one chirality half."""
    L = (4, 4, 4, 4)
    block = (4, 4, 2, 2)
    nv = 4
    P = oracle.block_orthonormalize(L, 12, block, rand_vecs(nv, vol(L), 12, 2))
    Pd = dense_P(L, 12, block, P)
    g5 = np.tile(np.array([1.0] * 6 + [-1.0] * 6), vol(L))
    Vc = Pd.shape[1] // (2 * nv)
    s3 = np.tile(np.array([1.0] * nv + [-1.0] * nv), Vc)
    assert np.abs(s3[None, :] * Pd - g5[:, None] * Pd).max() == 0


def test_restrict_prolong_are_P_dagger_and_P():
    L = (4, 4, 2, 4)
    block = (2, 2, 2, 2)
    nv = 3
    V = vol(L)
    P = oracle.block_orthonormalize(L, 12, block, rand_vecs(nv, V, 12, 3))
    Pd = dense_P(L, 12, block, P)
    rng = np.random.default_rng(4)
    f = rng.standard_normal((V, 12)) + 1j * rng.standard_normal((V, 12))
    c = oracle.restrict(L, 12, block, P, f)
    assert relerr(c.ravel(), Pd.conj().T @ f.ravel()) < 1e-14
    e = oracle.prolong(L, 12, block, P, c)
    assert relerr(e.ravel(), Pd @ c.ravel()) < 1e-14
    # R P = 1
    assert relerr(oracle.restrict(L, 12, block, P, e), c) < 1e-14


GALERKIN_CASES = [
    # (fine dims, block, nv): coarse extents 2 (aliasing), 1 (self-neighbour), mixed
    ((4, 4, 4, 4), (2, 2, 2, 2), 3),
    ((4, 4, 4, 4), (4, 4, 4, 4), 3),
    ((4, 4, 2, 8), (2, 4, 2, 4), 2),
]


@pytest.mark.parametrize("L,block,nv", GALERKIN_CASES)
def test_galerkin_dense(L, block, nv):
    """Stencil D_hat equals the dense product P^dag D P (Sec. 2)."""
    V = vol(L)
    U = inputs.gauge_field(L, 0.5, 21)
    m = -0.2
    P = oracle.block_orthonormalize(L, 12, block, rand_vecs(nv, V, 12, 5))
    Y = oracle.coarse_build_wilson(L, U, m, block, P)
    D = dense_from_apply(12 * V, lambda e: oracle.wilson(L, U, m, e.reshape(V, 12)))
    Pd = dense_P(L, 12, block, P)
    Lc = oracle.coarse_dims(L, block)
    Dh = dense_stencil(Lc, 2 * nv, Y)
    assert np.abs(Dh - Pd.conj().T @ D @ Pd).max() < 1e-12
    # coarse apply = dense stencil, and its adjoint
    rng = np.random.default_rng(6)
    v = rng.standard_normal((vol(Lc), 2 * nv)) + 1j * rng.standard_normal((vol(Lc), 2 * nv))
    assert relerr(oracle.coarse_apply(Lc, 2 * nv, Y, v).ravel(), Dh @ v.ravel()) < 1e-13
    assert relerr(oracle.coarse_apply(Lc, 2 * nv, Y, v, dagger=True).ravel(), Dh.conj().T @ v.ravel()) < 1e-13
    # gamma5-hermiticity survives coarsening: sigma_3 D_hat sigma_3 = D_hat^dag (Sec. 3)
    s3 = np.tile(np.array([1.0] * nv + [-1.0] * nv), vol(Lc))
    assert np.abs(s3[:, None] * Dh * s3[None, :] - Dh.conj().T).max() < 1e-12


def test_galerkin_third_level_dense():
    """Coarsening a coarse stencil again (three-level hierarchy)."""
    L = (4, 4, 4, 4)
    b1 = (2, 2, 2, 2)
    nv1 = 2
    V = vol(L)
    U = inputs.gauge_field(L, 0.5, 22)
    P1 = oracle.block_orthonormalize(L, 12, b1, rand_vecs(nv1, V, 12, 7))
    Y1 = oracle.coarse_build_wilson(L, U, 0.1, b1, P1)
    L1 = oracle.coarse_dims(L, b1)
    d1 = 2 * nv1
    b2 = (1, 2, 2, 1)
    nv2 = 2
    P2 = oracle.block_orthonormalize(L1, d1, b2, rand_vecs(nv2, vol(L1), d1, 8))
    Y2 = oracle.coarse_build_coarse(L1, d1, Y1, b2, P2)
    L2 = oracle.coarse_dims(L1, b2)
    D1 = dense_stencil(L1, d1, Y1)
    P2d = dense_P(L1, d1, b2, P2)
    assert np.abs(dense_stencil(L2, 2 * nv2, Y2) - P2d.conj().T @ D1 @ P2d).max() < 1e-12


@pytest.mark.parametrize("L,b", [((8, 8, 8, 8), 4), ((4, 4, 4, 8), 2), ((4, 4, 4, 4), 4)])
def test_free_field_coarse_closed_form(L, b):
    """U = 1 and the 6 constant vectors e_{s,c} + e_{s+2,c}: the chirality
    split block basis is the piecewise-constant prolongator of Eq. 2.4 on all
    12 spin-colour components, and P^dag D(m) P = (1/b) D_W(m b) on the coarse
    lattice: local term (m + 4/b), hops -(1/2b)(1 -+ gamma_mu)."""
    V = vol(L)
    U = inputs.unit_gauge(L)
    vecs = np.zeros((6, V, 12), np.complex128)
    for s in range(2):
        for c in range(3):
            vecs[3 * s + c, :, 3 * s + c] = 1
            vecs[3 * s + c, :, 3 * (s + 2) + c] = 1
    block = (b, b, b, b)
    P = oracle.block_orthonormalize(L, 12, block, vecs)
    assert np.allclose(np.abs(P[P != 0]), 1 / b ** 2)
    m = -0.3
    Y = oracle.coarse_build_wilson(L, U, m, block, P)
    g = [oracle.gamma(mu) for mu in range(4)]
    I3 = np.eye(3)
    assert np.abs(Y[:, 0] - (m + 4 / b) * np.eye(12)).max() < 1e-13
    for mu in range(4):
        assert np.abs(Y[:, 1 + mu] - (-(1 / (2 * b)) * np.kron(np.eye(4) - g[mu], I3))).max() < 1e-13
        assert np.abs(Y[:, 5 + mu] - (-(1 / (2 * b)) * np.kron(np.eye(4) + g[mu], I3))).max() < 1e-13


def test_coarse_mass_shift():
    L = (4, 4, 4, 4)
    block = (2, 2, 2, 2)
    U = inputs.gauge_field(L, 0.5, 23)
    P = oracle.block_orthonormalize(L, 12, block, rand_vecs(3, vol(L), 12, 9))
    Y1 = oracle.coarse_build_wilson(L, U, 0.2, block, P)
    Y2 = oracle.coarse_build_wilson(L, U, -0.3, block, P)
    d = Y1 - Y2
    assert np.abs(d[:, 0] - 0.5 * np.eye(6)).max() < 1e-13
    assert np.abs(d[:, 1:]).max() < 1e-13


def test_coarse_correction_projector():
    """Eq. 2.5: calP = 1 - D P (P^dag D P)^-1 P^dag is a projector, and the
    restriction of its output vanishes (the printed 'P calP = 0' read as
    P^dag calP = 0)."""
    L = (2, 2, 2, 4)
    V = vol(L)
    block = (2, 2, 2, 2)
    U = inputs.gauge_field(L, 0.5, 24)
    P = oracle.block_orthonormalize(L, 12, block, rand_vecs(4, V, 12, 10))
    D = dense_from_apply(12 * V, lambda e: oracle.wilson(L, U, -0.1, e.reshape(V, 12)))
    Pd = dense_P(L, 12, block, P)
    Y = oracle.coarse_build_wilson(L, U, -0.1, block, P)
    Dh = dense_stencil(oracle.coarse_dims(L, block), 8, Y)
    C = np.eye(12 * V) - D @ Pd @ np.linalg.solve(Dh, Pd.conj().T)
    assert np.abs(C @ C - C).max() < 1e-11
    assert np.abs(Pd.conj().T @ C).max() < 1e-11


def test_cgnr_matches_dense_solve():
    L = (4, 4, 4, 4)
    block = (2, 2, 2, 2)
    U = inputs.gauge_field(L, 0.5, 25)
    P = oracle.block_orthonormalize(L, 12, block, rand_vecs(3, vol(L), 12, 11))
    Y = oracle.coarse_build_wilson(L, U, 0.05, block, P)
    Lc = oracle.coarse_dims(L, block)
    rng = np.random.default_rng(12)
    b = rng.standard_normal((vol(Lc), 6)) + 1j * rng.standard_normal((vol(Lc), 6))
    x, it = oracle.cgnr_coarse(Lc, 6, Y, b, 1e-12, 5000)
    xd = np.linalg.solve(dense_stencil(Lc, 6, Y), b.ravel())
    assert relerr(x.ravel(), xd) < 1e-9
    r = b - oracle.coarse_apply(Lc, 6, Y, x)
    assert np.linalg.norm(r) <= 1e-12 * np.linalg.norm(b) * 1.0001


def test_mr_never_increases_residual():
    L = (4, 4, 4, 4)
    U = inputs.gauge_field(L, 0.5, 26)
    rng = np.random.default_rng(13)
    r = rng.standard_normal((vol(L), 12)) + 1j * rng.standard_normal((vol(L), 12))
    e, res = oracle.mr_wilson(L, U, -0.2, r, np.zeros_like(r), 8)
    assert np.all(np.diff(res) <= 1e-12 * res[0])
    assert res[-1] < res[0]


def small_params(**kw):
    base = dict(nlevels=2, block=((2, 2, 2, 2),), nv=(4,), setup_iters=5, coarse_tol=1e-10, seed=5)
    base.update(kw)
    return oracle.default_params(**base)


def test_mg_solve_matches_dense_solve():
    L = (4, 4, 4, 4)
    V = vol(L)
    U = inputs.gauge_field(L, 0.4, 27)
    m = -0.1
    mg = oracle.MG(L, U, m, small_params())
    mg.setup()
    b = inputs.gaussian_rhs(L, 28)[0]
    x, st = mg.solve(b, 1e-10)
    D = dense_from_apply(12 * V, lambda e: oracle.wilson(L, U, m, e.reshape(V, 12)))
    xd = np.linalg.solve(D, b.ravel())
    cond = np.linalg.cond(D)
    assert st["converged"] and st["true_relres"] <= 1e-10
    assert relerr(x.ravel(), xd) <= 2 * cond * 1e-10
    r = b - oracle.wilson(L, U, m, x)
    assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(b)


def test_setup_invariants():
    """Null vectors are normalised; the final prolongator is block
    orthonormal; D_hat is the Galerkin product of the fine operator."""
    L = (4, 4, 4, 4)
    V = vol(L)
    U = inputs.gauge_field(L, 0.4, 29)
    mg = oracle.MG(L, U, -0.1, small_params(nv=(3,)))
    mg.setup()
    P = mg.P(0)
    Pd = dense_P(L, 12, (2, 2, 2, 2), P)
    assert np.abs(Pd.conj().T @ Pd - np.eye(Pd.shape[1])).max() < 1e-13
    Y = mg.Y(1)
    Yr = oracle.coarse_build_wilson(L, U, -0.1, (2, 2, 2, 2), P)
    assert np.abs(Y - Yr).max() < 1e-13


def test_set_mass_equals_rebuild():
    L = (4, 4, 4, 4)
    U = inputs.gauge_field(L, 0.4, 30)
    mg = oracle.MG(L, U, -0.1, small_params(nv=(3,)))
    mg.setup()
    P = mg.P(0)
    mg.set_mass(0.25)
    Yr = oracle.coarse_build_wilson(L, U, 0.25, (2, 2, 2, 2), P)
    assert np.abs(mg.Y(1) - Yr).max() < 1e-13


def test_config1_two_level_solve():
    """8^4, eps = 0.3, m = -0.1, 4^4 blocks, Nv = 8, 5 setup iterations,
    one Gaussian RHS, tol 1e-10: the final residual is the oracle's own."""
    L = (8, 8, 8, 8)
    U = inputs.gauge_field(L, 0.3, 101)
    mg = oracle.MG(L, U, -0.1, oracle.default_params(nlevels=2, nv=(8,), setup_iters=5, seed=150))
    mg.setup()
    b = inputs.gaussian_rhs(L, 110)[0]
    x, st = mg.solve(b, 1e-10)
    r = b - oracle.wilson(L, U, -0.1, x)
    assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(b)
    assert st["converged"]
    # fewer outer iterations than the unpreconditioned Krylov baseline
    _, it_bicg, rr = oracle.bicgstab(L, U, -0.1, b, 1e-10)
    assert rr <= 1e-10 and st["outer_iters"] < it_bicg


def test_three_level_w_cycle_solve():
    L = (8, 8, 8, 8)
    U = inputs.gauge_field(L, 0.4, 31)
    p = oracle.default_params(nlevels=3, block=((2, 2, 2, 2), (2, 2, 2, 2)), nv=(4, 4), setup_iters=4,
                              seed=32, coarse_tol=1e-8)
    mg = oracle.MG(L, U, -0.2, p)
    mg.setup()
    assert mg.level_info(2) == ((2, 2, 2, 2), 8, 0)
    Y2 = mg.Y(2)
    L1, d1, _ = mg.level_info(1)
    Yr = oracle.coarse_build_coarse(L1, d1, mg.Y(1), (2, 2, 2, 2), mg.P(1))
    assert np.abs(Y2 - Yr).max() < 1e-13
    b = inputs.gaussian_rhs(L, 33)[0]
    x, st = mg.solve(b, 1e-10)
    r = b - oracle.wilson(L, U, -0.2, x)
    assert st["converged"] and np.linalg.norm(r) <= 1e-10 * np.linalg.norm(b)
