"""The benchmark's timed launch configuration against the oracle, in every
reduction mode; complex U; the paper's two system shapes.

* bench.py times builds whose per-atom stage is the batched persistent launch
  (batch = 1) with tile shapes the autotuner picks for the workload; here that
  exact configuration is built at N_A = 100, N_L = 81, N_G = 8000 in each of
  the five reduction modes (FP64, split FP16, split INT8, FP64 3M, split
  BF16) and its
  sampled columns and bilinear probes are compared with the oracle.
* U enters S only through |u|^2 (Sec. 2, the U_a^H U_a factor of the equation
  for S); with complex U a kernel that squared Re(u) or u itself would
  differ from the oracle far beyond the bounds, which each complex-U case
  checks it would.
* NaCl (N_A = 512, N_L = 49, N_G = 9273) and AuAg (N_A = 108, N_L = 121,
  N_G = 13379) are the paper's systems at K_max = 4.0 (Tab. 1), here with
  synthetic values of those shapes.
"""

import numpy as np
import pytest

from hs_inputs import make_config, make_problem
from _parity import MODE_NAME, MODE_TOL, check_full, check_sampled, sample_columns

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _free():
    torch = _torch()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def _tuned(p):
    from paper_1611_00606_amd.tuning import autotune
    tuning, _ = autotune(sorted(set(p.nl.tolist())), p.N_G, reps=3)
    return tuning


@pytest.fixture(scope="module")
def precision():
    p = make_config("precision", seed=0)
    return p, _tuned(p)


@pytest.mark.parametrize("mode", [0, 1, 2, 3, 4, 5], ids=lambda m: MODE_NAME[m])
def test_bench_configuration_sampled(precision, mode):
    from paper_1611_00606_amd import DeviceBuild
    p, tuning = precision
    print(f"case precision N_G={p.N_G} batch=1 tuned mode={MODE_NAME[mode]}", flush=True)
    r = DeviceBuild.from_problem(p, mode=mode, batch=1, tuning=tuning)
    r.run()
    _torch().cuda.synchronize()
    check_sampled(p, r, sample_columns(p.N_G), MODE_TOL[mode])
    del r
    _free()


CU_CASES = {
    "uniform_failing": lambda: make_problem(4, 33, 300, seed=41, fail_atoms=[2], complex_u=True),
    "mixed_nl_planted": lambda: make_problem(5, [16, 49, 81, 121, 7], 517, seed=42,
                                             planted={1: 20}, complex_u=True),
}


@pytest.mark.parametrize("batch", [0, 1])
@pytest.mark.parametrize("case", list(CU_CASES))
@pytest.mark.parametrize("mode", [0, 1, 2, 3, 4, 5], ids=lambda m: MODE_NAME[m])
def test_complex_u_full(mode, case, batch):
    from paper_1611_00606_amd import DeviceBuild
    p = CU_CASES[case]()
    assert np.all(np.abs(p.U.imag) > 0)
    print(f"case {case} complex U N_G={p.N_G} mode={MODE_NAME[mode]} batch={batch}", flush=True)
    r = DeviceBuild.from_problem(p, mode=mode, batch=batch)
    r.run()
    _torch().cuda.synchronize()
    H, S, info = r.results()
    tol = MODE_TOL[mode]
    check_full(p, H, S, info, tol)
    # the case discriminates: weighting B's rows by Re(u)^2 or by Re(u^2)
    # instead of |u|^2 would move S by far more than the bound
    for w in (p.U.real ** 2, (p.U * p.U).real):
        d = np.abs(p.U) ** 2 - w
        shift = p.B.conj().T @ (d[:, None] * p.B)
        assert np.linalg.norm(shift) > 1e3 * tol * np.linalg.norm(S)


@pytest.mark.parametrize("name", ["nacl_kmax4", "auag_kmax4"])
def test_paper_shape_sampled(name):
    """The paper's system shapes at K_max = 4.0 in the timed configuration."""
    from paper_1611_00606_amd import DeviceBuild
    p = make_config(name, seed=0)
    print(f"case {name} N_A={p.N_A} N_L={int(p.nl[0])} N_G={p.N_G} K={p.K}", flush=True)
    r = DeviceBuild.from_problem(p, batch=1, tuning=_tuned(p))
    r.run()
    _torch().cuda.synchronize()
    check_sampled(p, r, sample_columns(p.N_G), MODE_TOL[0])
    del r
    _free()
