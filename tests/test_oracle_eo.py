"""Pins of the oracle's red/black (even-odd) functions (Sec. 3: multigrid
combined with red/black preconditioning), each against dense linear algebra
built from the pinned Wilson operator:

* the parity blocks of D: D_ee = D_oo = (4+m) 1, and the oracle's hopping
  between sublattices equals the dense off-diagonal blocks;
* the Schur complement S = D_ee - D_eo D_oo^-1 D_oe, applied matrix-free,
  equals its dense formula; it is gamma_5-hermitian and
  det D = (4+m)^(n/2) det S;
* the red/black post-smoother equals MR on the dense S from d_e = 0 with
  d_o = D_oo^-1 (s_o - D_oe d_e), restated in numpy from the prolonged
  correction; with many steps the cycle approaches D^-1 r;
* the red/black outer solve (GCR on S, preconditioned with the full
  cycle on (r_e, 0)) reproduces the dense solution within cond * tol;
* on 8^4 the red/black smoother takes fewer outer iterations than MR on D.
"""
import numpy as np
import pytest

import oracle
from paper_0912_2186_amd import inputs
from helpers import dense_from_apply, dense_P, relerr, vol


def dense_wilson(L, U, m):
    V = vol(L)
    return dense_from_apply(12 * V, lambda e: oracle.wilson(L, U, m, e.reshape(V, 12)))


def blocks(L, D):
    par = np.repeat(oracle.parity(L), 12)
    ev, od = par == 0, par == 1
    return ev, od, D[np.ix_(ev, ev)], D[np.ix_(ev, od)], D[np.ix_(od, ev)], D[np.ix_(od, od)]


@pytest.fixture(scope="module")
def eo44():
    L = (4, 4, 4, 4)
    U = inputs.gauge_field(L, 0.5, 61)
    m = -0.2
    D = dense_wilson(L, U, m)
    rng = np.random.default_rng(62)
    v = rng.standard_normal((vol(L), 12)) + 1j * rng.standard_normal((vol(L), 12))
    return dict(L=L, U=U, m=m, D=D, v=v)


def test_parity_blocks_and_hopping(eo44):
    g = eo44
    L, m = g["L"], g["m"]
    ev, od, Dee, Deo, Doe, Doo = blocks(L, g["D"])
    n2 = Dee.shape[0]
    assert np.abs(Dee - (4 + m) * np.eye(n2)).max() == 0
    assert np.abs(Doo - (4 + m) * np.eye(n2)).max() == 0
    v = g["v"].ravel()
    for par, blk, src in ((0, Deo, od), (1, Doe, ev)):
        h = oracle.wilson_hop_parity(L, g["U"], m, g["v"], par).ravel()
        tgt = ev if par == 0 else od
        assert relerr(h[tgt], blk @ v[src]) < 1e-14
        assert np.abs(h[~tgt]).max() == 0
        # only the other sublattice is read
        w = g["v"].copy().ravel()
        w[tgt] = 1e6
        assert relerr(oracle.wilson_hop_parity(L, g["U"], m, w.reshape(-1, 12), par).ravel()[tgt], blk @ v[src]) < 1e-14


def test_schur_complement(eo44):
    g = eo44
    L, m = g["L"], g["m"]
    ev, od, Dee, Deo, Doe, Doo = blocks(L, g["D"])
    S = Dee - Deo @ np.linalg.solve(Doo, Doe)
    out = oracle.schur_apply(L, g["U"], m, g["v"]).ravel()
    assert relerr(out[ev], S @ g["v"].ravel()[ev]) < 1e-14
    assert np.abs(out[od]).max() == 0
    # gamma_5-hermiticity (gamma_5 = diag(1,1,-1,-1) per site, site-local)
    g5 = np.tile(np.repeat([1.0, 1.0, -1.0, -1.0], 3), vol(L) // 2)
    assert np.abs(np.diag(g5) @ S @ np.diag(g5) - S.conj().T).max() < 1e-13


def test_schur_determinant_identity():
    L = (2, 2, 2, 2)
    U = inputs.gauge_field(L, 0.6, 63)
    m = 0.1
    D = dense_wilson(L, U, m)
    ev, od, Dee, Deo, Doe, Doo = blocks(L, D)
    S = dense_from_apply(Dee.shape[0], lambda e: _schur_dense_apply(L, U, m, e, ev))
    s1, l1 = np.linalg.slogdet(D)
    s2, l2 = np.linalg.slogdet(S)
    n2 = Dee.shape[0]
    assert abs((l2 + n2 * np.log(4 + m)) - l1) < 1e-10
    assert abs(s1 - s2) < 1e-10


def _schur_dense_apply(L, U, m, e, ev):
    v = np.zeros(12 * vol(L), np.complex128)
    v[ev] = e
    return oracle.schur_apply(L, U, m, v.reshape(-1, 12)).ravel()[ev]


def schur_mr_numpy(D, ev, od, m, r, e0, nsteps):
    """s = r - D e0; d_e = nsteps MR steps on S d_e = s_e - D_eo s_o/(4+m)
    from 0; d_o = (s_o - D_oe d_e)/(4+m); e = e0 + d."""
    Dee, Deo, Doe, Doo = D[np.ix_(ev, ev)], D[np.ix_(ev, od)], D[np.ix_(od, ev)], D[np.ix_(od, od)]
    S = Dee - Deo @ np.linalg.solve(Doo, Doe)
    s = r - D @ e0
    be = s[ev] - Deo @ s[od] / (4 + m)
    de = np.zeros_like(be)
    res = be.copy()
    for _ in range(nsteps):
        q = S @ res
        a = np.vdot(q, res) / np.vdot(q, q).real
        de = de + a * res
        res = res - a * q
    d = np.zeros_like(r)
    d[ev] = de
    d[od] = (s[od] - Doe @ de) / (4 + m)
    return e0 + d


def test_red_black_smoother_in_cycle(eo44):
    g = eo44
    L, U, m, D = g["L"], g["U"], g["m"], g["D"]
    blk = (2, 2, 2, 2)
    vecs = np.random.default_rng(64).standard_normal((3, vol(L), 12)) + 0j
    p = oracle.default_params(nlevels=2, block=(blk, blk), nv=(3, 3), post_smooth=4, coarse_tol=1e-14,
                              coarse_maxiter=2000, eo_smoother=1)
    mg = oracle.MG(L, U, m, p)
    mg.set_null_vectors(0, vecs)
    r = g["v"].ravel()
    e = mg.cycle(g["v"]).ravel()
    Pd = dense_P(L, 12, blk, mg.P(0))
    e0 = Pd @ np.linalg.solve(Pd.conj().T @ D @ Pd, Pd.conj().T @ r)
    ev, od = blocks(L, D)[:2]
    ref = schur_mr_numpy(D, ev, od, m, r, e0, 4)
    assert relerr(e, ref) < 1e-11
    # discriminating: 3 steps, or MR on D instead of S, are far off
    assert relerr(schur_mr_numpy(D, ev, od, m, r, e0, 3), ref) > 1e-4
    # many steps: the smoother solves D d = s, so the cycle approaches D^-1 r
    p.post_smooth = 400
    mg2 = oracle.MG(L, U, m, p)
    mg2.set_null_vectors(0, vecs)
    assert relerr(mg2.cycle(g["v"]).ravel(), np.linalg.solve(D, r)) < 1e-8


def test_red_black_outer_solve_matches_dense(eo44):
    g = eo44
    L, U, m, D = g["L"], g["U"], g["m"], g["D"]
    p = oracle.default_params(nlevels=2, block=((2, 2, 2, 2), (2, 2, 2, 2)), nv=(4, 4), setup_iters=4, seed=65)
    mg = oracle.MG(L, U, m, p)
    mg.setup()
    b = g["v"]
    x, st = mg.solve_eo(b, 1e-10)
    assert st["converged"] and st["true_relres"] <= 1e-10
    xd = np.linalg.solve(D, b.ravel())
    cond = np.linalg.cond(D)
    assert relerr(x.ravel(), xd) <= 2 * cond * 1e-10


def test_red_black_smoother_fewer_iterations_8to4():
    """8^4, eps 0.3, m = -0.1, N_nu = 8, 10 setup iterations: MR on the
    Schur complement takes fewer outer iterations than MR on D (the paper
    reports about 30 % from red/black preconditioning)."""
    L = (8, 8, 8, 8)
    U = inputs.gauge_field(L, 0.3, 101)
    b = inputs.gaussian_rhs(L, 110)[0]
    its = {}
    for eo in (0, 1):
        p = oracle.default_params(nlevels=2, nv=(8,), setup_iters=10, seed=150, eo_smoother=eo)
        mg = oracle.MG(L, U, -0.1, p)
        mg.setup()
        x, st = mg.solve(b, 1e-10)
        assert st["converged"]
        r = b[0] - oracle.wilson(L, U, -0.1, x) if b.ndim == 3 else b - oracle.wilson(L, U, -0.1, x)
        assert np.linalg.norm(r) / np.linalg.norm(b) <= 1e-10 * 1.0001
        its[eo] = st["outer_iters"]
    print("outer iterations: MR on D", its[0], "MR on S", its[1])
    assert its[1] < 0.85 * its[0]
