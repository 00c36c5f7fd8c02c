"""Full-spin-structure coarsening (WMG_SPIN_SPLIT: the fine level's null
vectors split by Dirac spin, 4 N_nu coarse dof per block) on the GPU
against the oracle: prolongator, Galerkin links, FP64 and FP16/MFMA
transfers from identical null vectors, the FP64 solve's iteration count,
and a mixed multi-RHS solve to the oracle's 1e-10 (three levels too)."""
import sys

import numpy as np
import pytest

import oracle
from paper_0912_2186_amd import inputs
from helpers import relerr, vol

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).cuda()


def host(t):
    return t.cpu().numpy()


def empty(shape):
    import torch

    return torch.zeros(shape, dtype=torch.complex128, device="cuda")


def rand_vecs(nv, V, dof, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((nv, V, dof)) + 1j * rng.standard_normal((nv, V, dof))


@pytest.mark.parametrize("L,block,nv", [((8, 8, 8, 8), (4, 4, 4, 4), 4), ((4, 4, 4, 8), (2, 2, 2, 4), 3),
                                        ((8, 4, 4, 8), (4, 4, 2, 2), 6)])
def test_spin_split_galerkin_and_transfers(wmg, L, block, nv):
    say("spin split galerkin", L, block, nv)
    V = vol(L)
    m = -0.15
    U = inputs.gauge_field(L, 0.5, 311)
    p = wmg.default_params(setup_iters=1, seed=3, nrhs_max=2, flags=wmg.WMG_SPIN_SPLIT)
    mg = wmg.MG(L, dev(U), m, nv, block, p)
    assert mg.level_info(1)[1] == 4 * nv
    vecs = rand_vecs(nv, V, 12, 312)
    mg.mg_set_null_vectors(0, dev(vecs))
    P_ref = oracle.block_orthonormalize_ns(L, 12, block, vecs, 4)
    P_gpu = empty((nv, V, 12))
    mg.mg_get_prolongator(0, P_gpu)
    assert relerr(host(P_gpu), P_ref) < 1e-13
    Lc = oracle.coarse_dims(L, block)
    Vc, n = vol(Lc), 4 * nv
    Y_ref = oracle.coarse_build_wilson_ns(L, U, m, block, P_ref, 4)
    Y_gpu = empty((Vc, 9, n, n))
    mg.mg_get_coarse_links(1, Y_gpu)
    e = relerr(host(Y_gpu), Y_ref)
    say("  coarse links relerr", e)
    assert e < 1e-12
    f = inputs.gaussian_rhs(L, 313, 2)
    c = empty((2, Vc, n))
    mg.mg_restrict(0, dev(f), c, 2)
    ref = np.stack([oracle.restrict_ns(L, 12, block, P_ref, f[r], 4) for r in range(2)])
    assert relerr(host(c), ref) < 1e-13
    fo = empty((2, V, 12))
    mg.mg_prolong(0, dev(ref), fo, 2)
    assert relerr(host(fo), np.stack([oracle.prolong_ns(L, 12, block, P_ref, ref[r], 4) for r in range(2)])) < 1e-13
    for dag in (False, True):
        o = empty((Vc, n))
        mg.mg_coarse_apply(1, dev(ref[0]), o, dagger=dag)
        assert relerr(host(o), oracle.coarse_apply(Lc, n, Y_ref, ref[0], dagger=dag)) < 1e-13


@pytest.mark.parametrize("nv,nrhs", [(8, 3), (12, 28)])
def test_spin_split_low_precision_transfers(wmg, nv, nrhs):
    """FP16-stored P, FP32 vectors (matrix-core restriction and
    prolongation on 4^4 aggregates) with the spin split."""
    L, block = (8, 8, 8, 8), (4, 4, 4, 4)
    say("spin split lowprec transfers", nv, nrhs)
    V = vol(L)
    U = inputs.gauge_field(L, 0.5, 314)
    p = wmg.default_params(setup_iters=0, seed=2, nrhs_max=nrhs, precision=wmg.WMG_MIXED, flags=wmg.WMG_SPIN_SPLIT)
    mg = wmg.MG(L, dev(U), -0.1, nv, block, p)
    vecs = rand_vecs(nv, V, 12, 315)
    mg.mg_set_null_vectors(0, dev(vecs))
    P = oracle.block_orthonormalize_ns(L, 12, block, vecs, 4)
    Vc = vol(oracle.coarse_dims(L, block))
    f = inputs.gaussian_rhs(L, 316, nrhs)
    c = empty((nrhs, Vc, 4 * nv))
    mg.mg_restrict_f32(0, dev(f), c, nrhs)
    ref = np.stack([oracle.restrict_ns(L, 12, block, P, f[r], 4) for r in range(nrhs)])
    e1 = relerr(host(c), ref)
    cr = rand_vecs(nrhs, Vc, 4 * nv, 317)
    fo = empty((nrhs, V, 12))
    mg.mg_prolong_f32(0, dev(cr), fo, nrhs)
    e2 = relerr(host(fo), np.stack([oracle.prolong_ns(L, 12, block, P, cr[r], 4) for r in range(nrhs)]))
    say("  restrict relerr", e1, "prolong relerr", e2)
    assert e1 < 2e-3 and e2 < 2e-3


def test_spin_split_fp64_iteration_parity(wmg):
    L = (8, 8, 8, 12)
    V = vol(L)
    say("spin split fp64 parity", L)
    U = inputs.gauge_field(L, 0.4, 304)
    m = -0.05
    p = wmg.default_params(setup_iters=1, seed=1, flags=wmg.WMG_SPIN_SPLIT)
    mg = wmg.MG(L, dev(U), m, 4, (4, 4, 4, 4), p)
    og = oracle.MG(L, U, m, oracle.default_params(nlevels=2, nv=(4,), seed=1, setup_iters=6, spin_parts=4))
    og.setup()
    vecs = og.null_vectors(0)
    mg.mg_set_null_vectors(0, dev(vecs))
    b = inputs.gaussian_rhs(L, 41)[0]
    x = empty((1, V, 12))
    st = mg.mg_solve(dev(b[None]), x, 1e-10)
    xo, sto = og.solve(b, 1e-10)
    say("  gpu", st, "oracle", sto)
    assert st["converged"] and abs(st["outer_iters"] - sto["outer_iters"]) <= 1
    xg = host(x)[0]
    assert np.linalg.norm(b - oracle.wilson(L, U, m, xg)) <= 1e-10 * np.linalg.norm(b) * 1.0001
    assert relerr(xg, xo) < 1e-7


@pytest.mark.parametrize("levels", [2, 3])
def test_spin_split_mixed_multi_rhs(wmg, levels):
    """16^3x32, eps 0.6, m = -0.32: N_nu = 12 split by spin (48 coarse dof,
    the matrix-core stencil), red/black smoother, mixed precision, 2 point +
    2 Z4 right-hand sides; three levels with a chirality split of 2^4
    aggregates below.  Every rhs reaches the oracle's 1e-10."""
    L = (16, 16, 16, 32)
    V = vol(L)
    say("spin split mixed", L, "levels", levels)
    U = inputs.gauge_field(L, 0.6, 3301)
    m = -0.32
    b = np.concatenate([inputs.point_sources(L)[:2], inputs.z4_noise(L, 3310, 2)])
    kw = dict(levels=3, block=((4, 4, 4, 4), (2, 2, 2, 2)), nvec=(12, 24)) if levels == 3 else {}
    p = wmg.default_params(setup_iters=10, seed=3350, nrhs_max=4, precision=wmg.WMG_MIXED, coarse_tol=1e-5,
                           flags=wmg.WMG_SPIN_SPLIT | wmg.WMG_EO_SMOOTHER, **kw)
    mg = wmg.MG(L, dev(U), m, 12, (4, 4, 4, 4), p)
    assert mg.level_info(1)[1] == 48
    x = empty((4, V, 12))
    st = mg.mg_solve(dev(b), x, 1e-10)
    mg.close()
    say("  ", st)
    assert st["converged"]
    xh = host(x)
    for k in range(4):
        rr = np.linalg.norm(b[k] - oracle.wilson(L, U, m, xh[k])) / np.linalg.norm(b[k])
        say("  rhs", k, "oracle relres", rr)
        assert rr <= 1e-10 * 1.0001
