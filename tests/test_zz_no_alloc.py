"""md_newton_step_noalloc (the library's fixed per-GPU scratch instead of a
caller workspace) gives the bits of md_newton_step, on two calls in a row,
the second with a smaller input, then the first input again."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2012_06607_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2012_06607_amd import binding
    binding.lib()
    return binding


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def one_step(B, sysm, x, noalloc):
    m = sysm.m
    sd = B.DeviceSystem(sysm)
    xg = torch.as_tensor(np.ascontiguousarray(x), device="cuda")
    nrm = torch.zeros((m, 2), dtype=torch.float64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    if noalloc:
        B.md_newton_step_noalloc(sd, xg, nrm, st)
    else:
        B.md_newton_step(sd, xg, dx_norm=nrm, status=st)
    return host(xg), host(nrm), int(host(st)[0])


def test_noalloc_matches_workspace_entry_point(B):
    # a quad-double step of 32 unknowns at degree 16 (about 4 MB of scratch),
    # then a double-double step of 8 unknowns at degree 8 (0.2 MB), then the
    # first again: each result equals md_newton_step's on the same input
    big = I.newton_system((1202, 0), 32, 4, terms=8)
    small = I.newton_system((0, 0), 8, 2)
    cases = [(big, 16), (small, 8), (big, 16)]
    for (sysm, x0), d in cases:
        x = I.series_start(x0, d)
        print(f"noalloc step m={sysm.m} n={sysm.n} d={d}", flush=True)
        # from the second step's input, so that every coefficient changes
        x, _, st0 = one_step(B, sysm, x, False)
        assert st0 == 0
        want = one_step(B, sysm, x, False)
        got = one_step(B, sysm, x, True)
        assert got[2] == want[2] == 0
        assert np.array_equal(got[0], want[0])
        assert np.array_equal(got[1], want[1])
        assert got[1][0, 0] > 0
