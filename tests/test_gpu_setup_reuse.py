"""Setup reuse (the paper's Sec. 4: the setup is a fixed cost to amortise,
and as the gauge field evolves it is refreshed rather than redone): a
saved setup reloads into an identical hierarchy whose Galerkin operator is
the oracle's P^dag D P from the same vectors; for links that moved
(U' = exp(i delta H') U, one step of a Monte Carlo chain) a refresh from
the old vectors restores the solver at a fraction of a new setup's cost."""
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


def solve(mg, L, U, m, b):
    x = empty((1, vol(L), 12))
    st = mg.mg_solve(dev(b), x, 1e-10)
    rr = np.linalg.norm(b[0] - oracle.wilson(L, U, m, host(x)[0])) / np.linalg.norm(b[0])
    assert st["converged"] and rr <= 1e-10 * 1.0001
    return st["outer_iters"]


def test_save_load_refresh(wmg, tmp_path):
    L = (8, 8, 8, 16)
    blk = (4, 4, 4, 4)
    nv = 12
    m = -0.3
    U = inputs.gauge_field(L, 0.5, 501)
    b = inputs.gaussian_rhs(L, 510)
    p = wmg.default_params(setup_iters=10, seed=550)
    mg = wmg.MG(L, dev(U), m, nv, blk, p)
    it0 = solve(mg, L, U, m, b)
    path = str(tmp_path / "setup.wmg")
    mg.mg_save(path)
    say("saved", path, "iterations", it0)

    # reload for the same links: the same hierarchy, bit for bit
    mg2 = wmg.MG.load(path, L, dev(U), m)
    Vc = vol(oracle.coarse_dims(L, blk))
    Y1, Y2 = empty((Vc, 9, 2 * nv, 2 * nv)), empty((Vc, 9, 2 * nv, 2 * nv))
    mg.mg_get_coarse_links(1, Y1)
    mg2.mg_get_coarse_links(1, Y2)
    assert np.array_equal(host(Y1), host(Y2))
    assert solve(mg2, L, U, m, b) == it0
    # and its Galerkin operator is the oracle's from the saved vectors
    vecs = empty((nv, vol(L), 12))
    mg2.mg_get_null_vectors(0, vecs)
    P = oracle.block_orthonormalize(L, 12, blk, host(vecs))
    assert relerr(host(Y2), oracle.coarse_build_wilson(L, U, m, blk, P)) < 1e-12
    mg2.close()

    # one step of a chain, U' = exp(i 0.25 H') U: every variant converges;
    # the counts are reported (at this size they move by a few either way)
    G = inputs.gauge_field(L, 0.25, 502)
    Up = np.einsum("smab,smbc->smac", G, U)
    stale = wmg.MG.load(path, L, dev(Up), m)  # old vectors, Galerkin operator rebuilt for U'
    it_stale = solve(stale, L, Up, m, b)
    stale.close()
    fresh = wmg.MG(L, dev(Up), m, nv, blk, p)
    it_fresh = solve(fresh, L, Up, m, b)
    setup_fresh = fresh.mg_solve(dev(b), empty((1, vol(L), 12)), 1e-10)["setup_s"]
    fresh.close()
    step = wmg.MG.load(path, L, dev(U), m)
    step.mg_refresh(dev(Up), 3)
    it_ref = solve(step, L, Up, m, b)
    setup_ref = step.mg_solve(dev(b), empty((1, vol(L), 12)), 1e-10)["setup_s"]
    step.close()
    say("chain step: before", it0, "stale", it_stale, "refreshed", it_ref, "new setup", it_fresh,
        "| setup s: refresh %.3f new %.3f" % (setup_ref, setup_fresh))
    assert it_ref <= 1.25 * it_fresh + 1
    assert setup_ref < setup_fresh

    # an unrelated field: the saved vectors are no longer near-null, the
    # stale hierarchy is poor, and a refresh restores a new setup's count
    Uz = inputs.gauge_field(L, 0.5, 599)
    stale = wmg.MG.load(path, L, dev(Uz), m)
    it_stale = solve(stale, L, Uz, m, b)
    stale.close()
    fresh = wmg.MG(L, dev(Uz), m, nv, blk, p)
    it_fresh = solve(fresh, L, Uz, m, b)
    fresh.close()
    mg.mg_refresh(dev(Uz), 5)
    it_ref = solve(mg, L, Uz, m, b)
    say("new field: stale", it_stale, "refreshed", it_ref, "new setup", it_fresh)
    assert it_ref < it_stale
    assert it_ref <= 1.3 * it_fresh + 2
    mg.close()


def test_load_rejects_bad_files(wmg, tmp_path):
    L = (8, 8, 8, 8)
    U = dev(inputs.gauge_field(L, 0.3, 503))
    bad = tmp_path / "garbage.wmg"
    bad.write_bytes(b"not a setup" * 100)
    for path in (str(tmp_path / "missing.wmg"), str(bad)):
        with pytest.raises(wmg.WmgError) as e:
            wmg.MG.load(path, L, U, -0.1)
        assert e.value.code == wmg.WMG_EINVAL
    # a good file, cut short, and one for another lattice
    p = wmg.default_params(setup_iters=2, seed=5)
    mg = wmg.MG(L, U, -0.1, 4, (4, 4, 4, 4), p)
    good = tmp_path / "good.wmg"
    mg.mg_save(str(good))
    mg.close()
    data = good.read_bytes()
    cut = tmp_path / "cut.wmg"
    cut.write_bytes(data[: len(data) // 2])
    flip = tmp_path / "flip.wmg"
    flip.write_bytes(data[:-100] + bytes([data[-100] ^ 1]) + data[-99:])
    for path in (cut, flip):
        with pytest.raises(wmg.WmgError) as e:
            wmg.MG.load(str(path), L, U, -0.1)
        say(path.name, e.value)
    L2 = (8, 8, 8, 16)
    with pytest.raises(wmg.WmgError):
        wmg.MG.load(str(good), L2, dev(inputs.gauge_field(L2, 0.3, 504)), -0.1)
