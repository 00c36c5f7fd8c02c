"""The allocation-free BiCGStab entry point (work buffers in the library's
fixed device array) against bicgstab_solve, the same solve with buffers the
library allocates, both through the C ABI; the oracle's FP64 operator checks
the residual of every result."""
import numpy as np
import pytest
import torch

import oracle
from paper_0912_2186_amd import inputs, wmg

pytestmark = pytest.mark.gpu


def test_noalloc_matches_bicgstab_two_calls():
    # the larger lattice first, then a smaller one: the second call finds the
    # first call's data in the array and must clear what it needs
    cases = [((8, 8, 8, 16), 0.3, -0.05, 901, False), ((8, 8, 8, 8), 0.3, -0.1, 902, True)]
    for L, eps, m, seed, own_stream in cases:
        print("no-alloc case L=%s m=%g own_stream=%s" % (L, m, own_stream), flush=True)
        Uh = inputs.gauge_field(L, eps, seed)
        bh = inputs.gaussian_rhs(L, seed + 9)[0]
        U = torch.from_numpy(Uh).cuda()
        b = torch.from_numpy(bh).cuda()
        x_ref = torch.zeros_like(b)
        x_na = torch.full_like(b, 7.0)  # x is output only
        st_ref = wmg.bicgstab_solve(L, U, m, b, x_ref, 1e-10)
        stream = torch.cuda.Stream() if own_stream else None
        torch.cuda.synchronize()
        st_na = wmg.bicgstab_solve_noalloc(L, U, m, b, x_na, 1e-10, stream=stream)
        torch.cuda.synchronize()
        assert st_ref["converged"] and st_na["converged"]
        assert st_na["outer_iters"] == st_ref["outer_iters"]
        d = (x_na - x_ref).abs().max().item() / x_ref.abs().max().item()
        assert d <= 1e-12, d
        xh = x_na.cpu().numpy()
        r = bh - oracle.wilson(L, Uh, m, xh)
        rel = np.linalg.norm(r) / np.linalg.norm(bh)
        print("  iterations %d, max |x_na - x_ref| / max |x_ref| = %.2e, oracle relres %.2e"
              % (st_na["outer_iters"], d, rel), flush=True)
        assert rel <= 1e-10 * 1.001


def test_noalloc_rejects_lattice_beyond_the_array():
    L = (16, 16, 16, 8)  # 32768 sites need ~70 MB of scratch, more than the array holds
    U = torch.from_numpy(inputs.gauge_field(L, 0.3, 903)).cuda()
    b = torch.from_numpy(inputs.gaussian_rhs(L, 904)[0]).cuda()
    x = torch.zeros_like(b)
    with pytest.raises(wmg.WmgError) as e:
        wmg.bicgstab_solve_noalloc(L, U, -0.1, b, x, 1e-10)
    assert e.value.code == wmg.WMG_EINVAL
    assert "fixed maximum" in str(e.value)
    assert torch.count_nonzero(x).item() == 0
