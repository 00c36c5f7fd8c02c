"""Red/black (even-odd) preconditioned smoother (Sec. 3: MG combined with
red/black preconditioning) on the GPU against the oracle: one FP64 cycle
from identical null vectors, FP64 solve iteration parity, and the
mixed-precision multi-RHS solve (FP16 sublattice residuals) reaching the
oracle's 1e-10 in fewer outer iterations than the MR-on-D smoother; and
the red/black hopping kernel itself, site by site, in its three precision
forms."""
import sys

import numpy as np
import pytest

import oracle
from paper_0912_2186_amd import inputs
from helpers import local_err, relerr, vol

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


def _round(a, dt):
    return a.real.astype(dt).astype(np.float64) + 1j * a.imag.astype(dt).astype(np.float64)


def _decaying(L, site, kappa, seed):
    rng = np.random.default_rng(seed)
    V = vol(L)
    x0 = np.unravel_index(site, (L[3], L[2], L[1], L[0]))
    grid = np.indices((L[3], L[2], L[1], L[0]))
    d = np.zeros((L[3], L[2], L[1], L[0]))
    for ax, n in enumerate((L[3], L[2], L[1], L[0])):
        a = np.abs(grid[ax] - x0[ax])
        d = d + np.minimum(a, n - a)
    return np.exp(-kappa * d).reshape(V, 1) * (rng.standard_normal((V, 12)) + 1j * rng.standard_normal((V, 12)))


# (lattice, aggregate): several tiles with a ragged last chunk per slab, and
# a lattice whose z extent admits only slabs of 1, 2 or 6 z-slices
@pytest.mark.parametrize("L,block", [((20, 14, 4, 6), (4, 2, 4, 2)), ((8, 8, 6, 12), (4, 4, 2, 4))])
@pytest.mark.parametrize("prec", [0, 3, 4, 5, 6])
def test_hop_kernel_per_site(wmg, L, block, prec):
    """out = a diag + b H_par(hop) from the GPU kernel against the oracle's
    D_{par,1-par} (H = -2 D_{par,1-par}), both parities, both link formats,
    three right-hand sides (Gaussian, point source, decaying point source),
    inputs pre-rounded to the kernel's storage formats so both sides see the
    same values.  Per-site bound in units of the neighbourhood's largest
    input component (floor 2^-9 of the largest component for the FP16
    forms): FP64 256 u64 (|a| + 16 |b|); FP16 forms 64 * 2^-11 (|a| + 16 |b|),
    the links being FP16 on the GPU and exact in the oracle."""
    V = vol(L)
    m = -0.25
    m4 = 4 + m
    U = inputs.gauge_field(L, 0.5, 401)
    par_of = oracle.parity(L)
    src = np.stack([inputs.gaussian_rhs(L, 402)[0], inputs.point_sources(L)[5], _decaying(L, 17, 1.5, 403)])
    dg = np.stack([inputs.gaussian_rhs(L, 404)[0], inputs.z4_noise(L, 405, 1)[0], _decaying(L, 3, 1.0, 406)])
    if prec == 0:
        hop_in, diag_in = src, dg
    elif prec in (3, 5, 6):
        hop_in, diag_in = _round(src, np.float16), _round(dg, np.float16)
    else:
        hop_in, diag_in = _round(src, np.float32), _round(dg, np.float16)
    # prec 5 is the fused last step of the smoother (FP16 input, FP32
    # output; 6 the same with FP16 output): parity 1 only, and the even
    # sites return hop's own values
    cases = ((1, 0.0, 1.0), (0, m4, -0.25 / m4), (1, 1.0 / m4, 0.5 / m4))
    if prec >= 5:
        cases = ((1, 1.0 / m4, 0.5 / m4), (1, 0.0, 1.0))
    for flags in (0, wmg.WMG_LINKS18):
        p = wmg.default_params(setup_iters=1, seed=7, nrhs_max=3, flags=flags)
        mg = wmg.MG(L, dev(U), m, 4, block, p)
        for par, a, b in cases:
            out = empty((3, V, 12))
            mg.mg_hop_eo(prec, par, a, b, dev(diag_in) if a != 0.0 else None, dev(hop_in), out, 3)
            oh = host(out)
            for r in range(3):
                mask = (par_of == par)[:, None]
                ref = (a * diag_in[r] + b * (-2.0) * oracle.wilson_hop_parity(L, U, m, hop_in[r], par)) * mask
                if prec >= 5:
                    ref = ref + hop_in[r] * ~mask
                sc_in = np.concatenate([hop_in[r], diag_in[r]], axis=1) if a != 0.0 else hop_in[r]
                k = abs(a) + 16 * abs(b)
                if prec == 0:
                    le = local_err(oh[r], ref, sc_in, L)
                    bound = 256 * 2.0 ** -52 * k
                else:
                    le = local_err(oh[r], ref, sc_in, L, floor=2.0 ** -9 * np.abs(sc_in).max())
                    bound = 64 * 2.0 ** -11 * k
                say("  L", L, "prec", prec, "links", mg.mg_link_reals(), "par", par, "rhs", r,
                    "relerr %.2e site %.2e" % (relerr(oh[r], ref), le))
                assert le < bound
                if prec >= 5:
                    assert np.array_equal(oh[r][~mask[:, 0]], hop_in[r][~mask[:, 0]])
                else:
                    assert np.all(oh[r][~mask[:, 0]] == 0)
                if prec == 6:
                    assert np.array_equal(oh[r], _round(oh[r], np.float16))
        mg.close()


@pytest.mark.parametrize("flags", [0, "links18"])
def test_red_black_cycle_parity(wmg, flags):
    L = (8, 8, 8, 8)
    V = vol(L)
    fl = wmg.WMG_EO_SMOOTHER | (wmg.WMG_LINKS18 if flags == "links18" else 0)
    say("red/black cycle parity", L, "flags", fl)
    U = inputs.gauge_field(L, 0.4, 303)
    m = -0.1
    p = wmg.default_params(setup_iters=1, seed=1, coarse_tol=1e-12, flags=fl)
    mg = wmg.MG(L, dev(U), m, 6, (4, 4, 4, 4), p)
    vecs = rand_vecs(6, V, 12, 31)
    mg.mg_set_null_vectors(0, dev(vecs))
    og = oracle.MG(L, U, m, oracle.default_params(nlevels=2, nv=(6,), coarse_tol=1e-12, eo_smoother=1))
    og.set_null_vectors(0, vecs)
    r = inputs.gaussian_rhs(L, 32)[0]
    z = empty((V, 12))
    mg.mg_cycle(dev(r), z)
    ref = og.cycle(r)
    e = relerr(host(z), ref)
    # discriminating: the cycle with MR on D differs
    og0 = oracle.MG(L, U, m, oracle.default_params(nlevels=2, nv=(6,), coarse_tol=1e-12))
    og0.set_null_vectors(0, vecs)
    say("  cycle relerr", e, "vs MR-on-D cycle", relerr(og0.cycle(r), ref))
    assert e < 1e-9
    assert relerr(og0.cycle(r), ref) > 1e-3


def test_red_black_fp64_solve_iteration_parity(wmg):
    L = (8, 8, 8, 12)
    V = vol(L)
    say("red/black fp64 solve parity", L)
    U = inputs.gauge_field(L, 0.4, 304)
    m = -0.05
    p = wmg.default_params(setup_iters=1, seed=1, flags=wmg.WMG_EO_SMOOTHER)
    mg = wmg.MG(L, dev(U), m, 6, (4, 4, 4, 4), p)
    og = oracle.MG(L, U, m, oracle.default_params(nlevels=2, nv=(6,), seed=1, setup_iters=6, eo_smoother=1))
    og.setup()
    vecs = og.P(0)
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


def test_red_black_mixed_multi_rhs(wmg):
    """16^3x32, eps 0.6, m = -0.32, N_nu = 24, mixed precision, 2 point + 2
    Z4 right-hand sides: with the red/black smoother every rhs reaches the
    oracle's 1e-10 and the outer count drops; the cycle's output stored in
    FP16 (the default with the red/black smoother) needs at most one outer
    iteration more than stored in FP32 (WMG_Z32)."""
    L = (16, 16, 16, 32)
    V = vol(L)
    say("red/black mixed multi-rhs", L)
    U = inputs.gauge_field(L, 0.6, 3301)
    m = -0.32
    b = np.concatenate([inputs.point_sources(L)[:2], inputs.z4_noise(L, 3310, 2)])
    its = {}
    for fl in (0, wmg.WMG_EO_SMOOTHER, wmg.WMG_EO_SMOOTHER | wmg.WMG_Z32):
        p = wmg.default_params(setup_iters=10, seed=3350, nrhs_max=4, precision=wmg.WMG_MIXED, coarse_tol=1e-5,
                               flags=fl)
        mg = wmg.MG(L, dev(U), m, 24, (4, 4, 4, 4), p)
        x = empty((4, V, 12))
        st = mg.mg_solve(dev(b), x, 1e-10)
        st2 = mg.mg_solve(dev(b), x, 1e-10)
        mg.close()
        say("  flags", fl, st2)
        assert st["converged"] and st2["converged"]
        its[fl] = st2["outer_iters"]
        xh = host(x)
        for k in (0, 2):
            rr = np.linalg.norm(b[k] - oracle.wilson(L, U, m, xh[k])) / np.linalg.norm(b[k])
            say("    rhs", k, "oracle relres", rr)
            assert rr <= 1e-10 * 1.0001
    assert its[wmg.WMG_EO_SMOOTHER] < its[0]
    assert its[wmg.WMG_EO_SMOOTHER] <= its[wmg.WMG_EO_SMOOTHER | wmg.WMG_Z32] + 1


@pytest.mark.parametrize("prec", [0, 3, 4])
def test_hop_kernel_tilings_identical(wmg, prec):
    """Every work order the autotuner may pick for the red/black hop (slab
    depth, rhs tiles swept in groups, the last group short) computes each
    site with the same operations, so the outputs are bit-identical to the
    default's; the default is checked against the oracle per site on three
    of the 16 right-hand sides (bounds as in test_hop_kernel_per_site).
    16^1 x 12 x 8 x 6 gives ragged chunks per slab; 16 rhs give 6, 8 or 16
    rhs tiles (three, two or one rhs per thread), so groups of 2-5 leave a
    short last group."""
    L = (16, 12, 8, 6)
    V = vol(L)
    m = -0.25
    m4 = 4 + m
    nr = 16
    U = inputs.gauge_field(L, 0.5, 411)
    par_of = oracle.parity(L)
    src = inputs.gaussian_rhs(L, 412, nr)
    dg = inputs.gaussian_rhs(L, 413, nr)
    if prec == 3:
        src, dg = _round(src, np.float16), _round(dg, np.float16)
    elif prec == 4:
        src, dg = _round(src, np.float32), _round(dg, np.float16)
    p = wmg.default_params(setup_iters=1, seed=7, nrhs_max=nr)
    mg = wmg.MG(L, dev(U), m, 4, (4, 4, 4, 2), p)
    try:
        for par, a, b in ((1, 0.0, 1.0), (0, m4, -0.25 / m4)):
            outs = []
            for cand in range(16):
                wmg.tune_force(cand)
                out = empty((nr, V, 12))
                mg.mg_hop_eo(prec, par, a, b, dev(dg) if a != 0.0 else None, dev(src), out, nr)
                outs.append(host(out))
            wmg.tune_force(-1)
            for r in (0, 7, 15):
                mask = (par_of == par)[:, None]
                ref = (a * dg[r] + b * (-2.0) * oracle.wilson_hop_parity(L, U, m, src[r], par)) * mask
                sc_in = np.concatenate([src[r], dg[r]], axis=1) if a != 0.0 else src[r]
                k = abs(a) + 16 * abs(b)
                if prec == 0:
                    le, bound = local_err(outs[0][r], ref, sc_in, L), 256 * 2.0 ** -52 * k
                else:
                    le = local_err(outs[0][r], ref, sc_in, L, floor=2.0 ** -9 * np.abs(sc_in).max())
                    bound = 64 * 2.0 ** -11 * k
                assert le < bound
            diff = [c for c in range(1, 16) if not np.array_equal(outs[c], outs[0])]
            say("  prec", prec, "par", par, "tilings differing from the default:", diff)
            assert not diff
    finally:
        wmg.tune_force(-1)
        mg.close()


def test_red_black_mixed_max_rhs_then_fewer(wmg):
    """One mixed red/black context solving the maximum of 64 right-hand
    sides, then 3, then 64 again in the same buffers (the cycle's FP16
    output z, the FP16 smoother fields, the coarse stencil's FP16 products
    with their per-rhs scales at 64 rhs, two rhs tiles of 32): every solve
    converges and the oracle's FP64 residual of a sample of each is below
    1e-10."""
    L = (8, 8, 8, 8)
    V = vol(L)
    say("red/black mixed, 64 rhs then 3 then 64", L)
    U = inputs.gauge_field(L, 0.5, 3401)
    m = -0.2
    p = wmg.default_params(setup_iters=6, seed=3402, nrhs_max=64, precision=wmg.WMG_MIXED, coarse_tol=1e-5,
                           flags=wmg.WMG_EO_SMOOTHER)
    mg = wmg.MG(L, dev(U), m, 24, (4, 4, 4, 4), p)
    b64 = np.concatenate([inputs.point_sources(L), inputs.gaussian_rhs(L, 3403, 52)])
    b3 = np.concatenate([inputs.point_sources(L)[3:4], inputs.z4_noise(L, 3404, 2)])
    try:
        for b, sample in ((b64, (0, 11, 40, 63)), (b3, (0, 1, 2)), (b64, (5, 63))):
            n = b.shape[0]
            x = empty((n, V, 12))
            st = mg.mg_solve(dev(b), x, 1e-10)
            say("  nrhs", n, st)
            assert st["converged"] and st["true_relres"] <= 1e-10
            xh = host(x)
            for r in sample:
                res = np.linalg.norm(b[r] - oracle.wilson(L, U, m, xh[r])) / np.linalg.norm(b[r])
                assert res <= 1e-10 * 1.0001, (n, r, res)
    finally:
        mg.close()
