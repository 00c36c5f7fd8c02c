"""The coarsest CGNR run as captured HIP graphs (WMG_GRAPHS) gives the same
solve, bit for bit, as the launch-by-launch loop: the graphs hold the same
launches in the same order.  Three solves in a row on the graph context
(the first fills buffers and tuner choices, the second captures, the third
replays) each match the reference solve, with the program's own eager work
and synchronisations between the replays."""
import sys

import numpy as np
import pytest

import oracle
from paper_0912_2186_amd import inputs
from helpers import vol

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).cuda()


def test_graph_cgnr_matches_eager(wmg):
    import torch

    L = (8, 8, 8, 16)
    V = vol(L)
    m = -0.2
    U = inputs.gauge_field(L, 0.5, 305)
    b = np.concatenate([inputs.point_sources(L)[:1], inputs.z4_noise(L, 51, 2)])
    nrhs = b.shape[0]
    base = dict(setup_iters=4, seed=9, precision=wmg.WMG_MIXED, nrhs_max=nrhs, coarse_tol=1e-5)
    ref = wmg.MG(L, dev(U), m, 24, (4, 4, 4, 4), wmg.default_params(flags=wmg.WMG_EO_SMOOTHER, **base))
    gr = wmg.MG(L, dev(U), m, 24, (4, 4, 4, 4),
                wmg.default_params(flags=wmg.WMG_EO_SMOOTHER | wmg.WMG_GRAPHS, **base))
    xr = torch.zeros((nrhs, V, 12), dtype=torch.complex128, device="cuda")
    st_ref = ref.mg_solve(dev(b), xr, 1e-10)
    xr_h = xr.cpu().numpy()
    for k in range(3):
        xg = torch.zeros_like(xr)
        st = gr.mg_solve(dev(b), xg, 1e-10)
        torch.cuda.synchronize()
        d = np.abs(xg.cpu().numpy() - xr_h).max()
        say("solve", k, st["outer_iters"], st["coarse_iters"], "max |x_graph - x_eager| =", d)
        assert st["outer_iters"] == st_ref["outer_iters"] and st["coarse_iters"] == st_ref["coarse_iters"]
        assert d == 0.0
        # eager work between replays
        torch.cuda.synchronize()
        _ = (xg * 2).sum().item()
    rr = np.linalg.norm(b[1] - oracle.wilson(L, U, m, xr_h[1])) / np.linalg.norm(b[1])
    assert rr <= 1e-10 * 1.0001
    ref.close()
    gr.close()
