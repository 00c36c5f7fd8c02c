"""Pins of the oracle's multigrid cycle, adaptive setup and iteration-count
behaviour (Sec. 2-3), each against something other than the oracle itself:

* the two-grid cycle without smoothing equals the dense coarse-grid
  correction P (P^dag D P)^-1 P^dag r built from the pinned Wilson operator
  (Eq. 2.5 with the coarse operator formed densely, not from the oracle's
  stencil);
* the three-level V and W cycles equal their dense formulas,
  e_hat = C r_hat (V) and e_hat = C r_hat + C (r_hat - D_hat C r_hat) (W),
  C = P_2 (P_2^dag D_hat P_2)^-1 P_2^dag;
* the post-smoothed cycle equals four minimal-residual steps on D e = r,
  restated here in numpy from the prolonged correction (not from zero);
* the adaptive setup's vectors have a much smaller |D psi| / |psi| than the
  random vectors they start from, and the prolongator is their block
  orthonormalisation;
* Table 1's criterion: as m - m_crit shrinks 10x the MG outer iteration
  count grows by at most 1.5x while unpreconditioned BiCGStab grows by 3x
  or more.
"""
import numpy as np
import pytest

import oracle
from paper_0912_2186_amd import inputs
from helpers import dense_from_apply, dense_P, relerr, vol


def rand_vecs(nv, V, dof, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((nv, V, dof)) + 1j * rng.standard_normal((nv, V, dof))


def dense_wilson(L, U, m):
    V = vol(L)
    return dense_from_apply(12 * V, lambda e: oracle.wilson(L, U, m, e.reshape(V, 12)))


def mr_numpy(D, r, e, nsteps):
    """Minimal-residual steps on D e = r from e: s = r - D e; q = D s;
    a = <q, s> / <q, q>; e += a s; s -= a q."""
    e = e.copy()
    s = r - D @ e
    for _ in range(nsteps):
        q = D @ s
        a = np.vdot(q, s) / np.vdot(q, q).real
        e = e + a * s
        s = s - a * q
    return e


L2G = (4, 4, 4, 4)
B2G = (2, 2, 2, 2)


@pytest.fixture(scope="module")
def two_grid():
    """4^4 lattice, 2^4 aggregates, 3 random null vectors, dense D, P, D_hat."""
    L = L2G
    V = vol(L)
    U = inputs.gauge_field(L, 0.4, 41)
    m = -0.1
    vecs = rand_vecs(3, V, 12, 42)
    D = dense_wilson(L, U, m)
    rng = np.random.default_rng(43)
    r = rng.standard_normal((V, 12)) + 1j * rng.standard_normal((V, 12))
    return dict(L=L, U=U, m=m, vecs=vecs, D=D, r=r)


def make_mg(L, U, m, vecs1, post_smooth, wcycle=1, nlevels=2, block2=(1, 1, 2, 2), vecs2=None):
    nv1 = vecs1.shape[0]
    nv2 = vecs2.shape[0] if vecs2 is not None else nv1
    p = oracle.default_params(nlevels=nlevels, block=(B2G, block2), nv=(nv1, nv2), post_smooth=post_smooth,
                              wcycle=wcycle, coarse_tol=1e-14, coarse_maxiter=2000)
    mg = oracle.MG(L, U, m, p)
    mg.set_null_vectors(0, vecs1)
    if nlevels == 3:
        mg.set_null_vectors(1, vecs2)
    return mg


def test_two_grid_cycle_is_dense_coarse_correction(two_grid):
    """No smoothing, coarse solve to 1e-14: cycle(r) = P (P^dag D P)^-1 P^dag r."""
    g = two_grid
    mg = make_mg(g["L"], g["U"], g["m"], g["vecs"], post_smooth=0)
    e = mg.cycle(g["r"])
    Pd = dense_P(g["L"], 12, B2G, mg.P(0))
    Dh = Pd.conj().T @ g["D"] @ Pd
    ref = Pd @ np.linalg.solve(Dh, Pd.conj().T @ g["r"].ravel())
    assert relerr(e.ravel(), ref) < 1e-11
    # the coarse-grid correction leaves no restricted residual (Eq. 2.5)
    assert np.linalg.norm(Pd.conj().T @ (g["r"].ravel() - g["D"] @ e.ravel())) < 1e-10 * np.linalg.norm(g["r"])


def test_post_smoothed_cycle_is_mr_from_prolonged_correction(two_grid):
    """Four MR post-smoothing steps start from the prolonged coarse
    correction (not from zero)."""
    g = two_grid
    mg = make_mg(g["L"], g["U"], g["m"], g["vecs"], post_smooth=4)
    e = mg.cycle(g["r"]).ravel()
    Pd = dense_P(g["L"], 12, B2G, mg.P(0))
    D = g["D"]
    r = g["r"].ravel()
    e0 = Pd @ np.linalg.solve(Pd.conj().T @ D @ Pd, Pd.conj().T @ r)
    ref = mr_numpy(D, r, e0, 4)
    assert relerr(e, ref) < 1e-11
    # discriminating: smoothing from zero, or with 3 or 5 steps, is far off
    assert relerr(mr_numpy(D, r, np.zeros_like(r), 4), ref) > 1e-3
    assert relerr(mr_numpy(D, r, e0, 3), ref) > 1e-4
    assert relerr(mr_numpy(D, r, e0, 5), ref) > 1e-4


@pytest.mark.parametrize("wcycle", [0, 1])
@pytest.mark.parametrize("post_smooth", [0, 2])
def test_three_level_cycle_dense(two_grid, wcycle, post_smooth):
    """Three levels, written out densely: C(v) = P_2 (P_2^dag D_hat P_2)^-1
    P_2^dag v is the coarsest correction, S_l(r, e) is post_smooth MR steps
    with the level-l operator; level 1: cyc(r_hat) = S_1(r_hat, C r_hat);
    V: e_hat = cyc(r_hat); W: e_hat = cyc(r_hat) + cyc(r_hat - D_hat
    cyc(r_hat)); fine: e = S_0(r, P_1 e_hat).  Without smoothing the W
    cycle's second pass vanishes exactly (P_2^dag (r_hat - D_hat C r_hat) =
    0), so V and W coincide there; with smoothing they differ."""
    g = two_grid
    L = g["L"]
    L1 = oracle.coarse_dims(L, B2G)
    d1 = 2 * g["vecs"].shape[0]
    b2 = (1, 1, 2, 2)
    vecs2 = rand_vecs(2, vol(L1), d1, 44)
    mg = make_mg(L, g["U"], g["m"], g["vecs"], post_smooth=post_smooth, wcycle=wcycle, nlevels=3, block2=b2,
                 vecs2=vecs2)
    e = mg.cycle(g["r"]).ravel()
    P1 = dense_P(L, 12, B2G, mg.P(0))
    P2 = dense_P(L1, d1, b2, mg.P(1))
    D = g["D"]
    D1 = P1.conj().T @ D @ P1
    D2 = P2.conj().T @ D1 @ P2

    def cyc(v):
        return mr_numpy(D1, v, P2 @ np.linalg.solve(D2, P2.conj().T @ v), post_smooth)

    r = g["r"].ravel()
    r1 = P1.conj().T @ r
    e1v = cyc(r1)
    e1w = e1v + cyc(r1 - D1 @ e1v)
    ref = mr_numpy(D, r, P1 @ (e1w if wcycle else e1v), post_smooth)
    other = mr_numpy(D, r, P1 @ (e1v if wcycle else e1w), post_smooth)
    assert relerr(e, ref) < 1e-10
    if post_smooth:
        assert relerr(other, ref) > 1e-4  # the V and W formulas differ here
    else:
        assert relerr(other, ref) < 1e-12


def test_setup_vectors_lie_in_near_null_space():
    """The adaptive setup (Sec. 2) relaxes each random start vector towards
    the near-null space of D.  Pinned by the dense singular value
    decomposition of D on 4^4: this field has 12 small singular values
    (0.28-0.31, the next is 1.24); every adapted vector is normalised,
    |D psi| falls below a fifth of its Philox start's and below 1.5x the
    12th smallest singular value, and 90 % or more of psi lies in the span
    of the 12 lowest right singular vectors.  |D psi| averaged over the
    vectors falls with every setup iteration over the first three; the
    prolongator is the block orthonormalisation of exactly these vectors."""
    L = (4, 4, 4, 4)
    V = vol(L)
    U = inputs.gauge_field(L, 0.4, 29)
    m = -0.1
    D = dense_wilson(L, U, m)
    ev, W = np.linalg.eigh(D.conj().T @ D)  # right singular vectors, sigma^2 ascending
    sig = np.sqrt(np.maximum(ev, 0))
    assert sig[11] < 0.35 and sig[12] > 1.0
    low = W[:, :12]

    def setup(iters):
        p = oracle.default_params(nlevels=2, block=((2, 2, 2, 2),), nv=(4,), setup_iters=iters, coarse_tol=1e-10,
                                  seed=5)
        mg = oracle.MG(L, U, m, p)
        mg.setup()
        return mg

    mg = setup(5)
    vecs = mg.null_vectors(0)
    for k in range(vecs.shape[0]):
        psi = vecs[k].ravel()
        assert abs(np.linalg.norm(psi) - 1) < 1e-12
        start = oracle.start_vector(V, 12, 5, 0, k).ravel()
        r0 = np.linalg.norm(D @ start) / np.linalg.norm(start)
        r1 = np.linalg.norm(D @ psi)
        assert r1 < 0.2 * r0, (k, r0, r1)
        assert r1 < 1.5 * sig[11], (k, r1, sig[11])
        assert np.linalg.norm(low.conj().T @ psi) ** 2 >= 0.9
    Pb = oracle.block_orthonormalize(L, 12, (2, 2, 2, 2), vecs)
    assert np.abs(Pb - mg.P(0)).max() < 1e-13
    means = []
    for it in range(4):
        v = setup(it).null_vectors(0)
        means.append(np.mean([np.linalg.norm(D @ v[k].ravel()) for k in range(v.shape[0])]))
    assert all(np.diff(means) < 0), means


def critical_mass(L, U):
    """m_crit = - min Re lambda(D(m = 0)): the eigenvalues of c - D(0) of
    largest real part (ARPACK), c = 8 above the spectrum's real parts."""
    from scipy.sparse.linalg import LinearOperator, eigs

    V = vol(L)
    c = 8.0
    A = LinearOperator((12 * V, 12 * V), dtype=np.complex128,
                       matvec=lambda v: c * v - oracle.wilson(L, U, 0.0, v.reshape(V, 12)).ravel())
    w = eigs(A, k=6, which="LR", return_eigenvectors=False, tol=1e-6, ncv=60, maxiter=5000)
    return -(c - float(np.max(w.real)))


@pytest.mark.slow
def test_mass_independent_iteration_count():
    """Table 1's criterion on the 8^4 workload's field: one setup at the
    lightest mass, exact coarse shifts to the others; m - m_crit shrinks
    from 0.2 to 0.02 (10x).  MG outer iterations grow <= 1.5x, BiCGStab
    iterations grow >= 3x; every solve reaches 1e-10."""
    L = (8, 8, 8, 8)
    U = inputs.gauge_field(L, 0.3, 101)
    b = inputs.gaussian_rhs(L, 110)[0]
    mcrit = critical_mass(L, U)
    assert -0.24 < mcrit < -0.22  # the value quoted for this field
    dms = [0.2, 0.1, 0.05, 0.02]
    p = oracle.default_params(nlevels=2, nv=(8,), setup_iters=10, seed=150)
    mg = oracle.MG(L, U, mcrit + dms[-1], p)
    mg.setup()
    its_mg, its_bi = [], []
    for dm in dms:
        m = mcrit + dm
        mg.set_mass(m)
        x, st = mg.solve(b, 1e-10)
        assert st["converged"]
        assert np.linalg.norm(b - oracle.wilson(L, U, m, x)) <= 1e-10 * np.linalg.norm(b) * 1.0001
        _, itb, rr = oracle.bicgstab(L, U, m, b, 1e-10)
        assert rr <= 1e-10
        its_mg.append(st["outer_iters"])
        its_bi.append(itb)
    g_mg = its_mg[-1] / its_mg[0]
    g_bi = its_bi[-1] / its_bi[0]
    print("MG", its_mg, "BiCGStab", its_bi)
    assert g_mg <= 1.5, its_mg
    assert g_bi >= 3.0, its_bi
    assert all(np.diff(its_bi) > 0)
