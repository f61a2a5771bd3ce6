"""The allocation-free entry point (hs_build_static) against hs_build_ex.

hs_build_static runs the same kernels on a workspace that is a device array
inside the library, so its H, S and info must be bitwise those of
hs_build_ex with a caller workspace, in every reduction mode and with either
per-atom stage. Two calls in a row (a larger problem, then a smaller one)
show that what the first call leaves in the array does not leak into the
second.
"""

import numpy as np
import pytest

from hs_inputs import make_problem
from _parity import MODE_NAME

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _static(r, **kw):
    """hs_build_static on a DeviceBuild's inputs into fresh outputs."""
    from paper_1611_00606_amd import hs_build_static
    torch = _torch()
    H = torch.full_like(r.H, complex(np.nan, np.nan))
    S = torch.full_like(r.S, complex(np.nan, np.nan))
    info = torch.full_like(r.info, -7)
    hs_build_static(r.A, r.B, r.T_AA, r.T_AB, r.T_BB, r.U, r.N_A, r.N_L, r.N_G, H, S,
                    info=info, mode=r.mode, nl_per_atom=r.nl_per_atom, batch=r.batch, **kw)
    torch.cuda.synchronize()
    return H.cpu().numpy(), S.cpu().numpy(), info.cpu().numpy()


@pytest.mark.parametrize("batch", [0, 1])
@pytest.mark.parametrize("mode", [0, 1, 2, 3, 4, 5], ids=lambda m: MODE_NAME[m])
def test_static_equals_workspace_build(mode, batch):
    from paper_1611_00606_amd import DeviceBuild
    torch = _torch()
    big = make_problem(6, [16, 49, 81, 121, 7, 64], 700, seed=61, fail_atoms=[2], planted={3: 40})
    small = make_problem(3, 25, 333, seed=62, fail_atoms=[0])
    for p in (big, small):
        print(f"case static N_A={p.N_A} N_G={p.N_G} mode={MODE_NAME[mode]} batch={batch}",
              flush=True)
        r = DeviceBuild.from_problem(p, mode=mode, batch=batch)
        r.run()
        torch.cuda.synchronize()
        H0, S0, i0 = r.results()
        H1, S1, i1 = _static(r)
        assert np.array_equal(H1, H0) and np.array_equal(S1, S0) and np.array_equal(i1, i0)


def test_static_on_a_side_stream():
    from paper_1611_00606_amd import DeviceBuild
    torch = _torch()
    p = make_problem(4, 33, 410, seed=63, fail_atoms=[1])
    r = DeviceBuild.from_problem(p)
    r.run()
    torch.cuda.synchronize()
    H0, S0, i0 = r.results()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        H1, S1, i1 = _static(r, stream=s)
    assert np.array_equal(H1, H0) and np.array_equal(S1, S0) and np.array_equal(i1, i0)
