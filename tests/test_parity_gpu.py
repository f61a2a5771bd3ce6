"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Small and medium cases compare every element (relative Frobenius error of H
and S <= 1e-12, the FP64 bound); the large workloads, built here with
separate per-atom launches (batch = 0), compare sampled columns computed one
by one by the oracle and bilinear probes. The launch configuration the
benchmark times (batched per-atom stage, autotuned tile shapes) is checked
the same way in test_bench_config_gpu.py. The Cholesky flags are integer
decisions and must match exactly (inputs are built with a clear margin).
"""

import numpy as np
import pytest

import oracle as O
from hs_inputs import make_config, make_problem, cn

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _torch():
    import torch
    return torch


def _run(p, stream=None):
    from paper_1611_00606_amd import DeviceBuild
    torch = _torch()
    print(f"case N_A={p.N_A} nl={sorted(set(p.nl.tolist()))} N_G={p.N_G} failing={p.failing} "
          f"planted={p.planted}", flush=True)
    r = DeviceBuild.from_problem(p)
    r.run(stream=stream)
    torch.cuda.synchronize()
    return r


def _rel(x, y):
    return np.linalg.norm(x - y) / np.linalg.norm(y)


def _expected_info(p):
    info = np.zeros(p.N_A, np.int32)
    for a in p.failing:
        info[a] = 1
    for a, piv in p.planted.items():
        info[a] = piv
    return info


def _check_full(p, H, S, info):
    Hr = O.hamiltonian(p.A, p.B, p.T_AA, p.T_AB, p.T_BB, p.nl)
    Sr = O.overlap(p.A, p.B, p.U, p.nl)
    eh, es = _rel(H, Hr), _rel(S, Sr)
    print(f"  rel err H {eh:.2e} S {es:.2e}", flush=True)
    assert eh <= TOL and es <= TOL, (eh, es)
    # exactly Hermitian with a real diagonal
    assert np.array_equal(H, H.conj().T)
    assert np.array_equal(S, S.conj().T)
    assert np.all(H.diagonal().imag == 0) and np.all(S.diagonal().imag == 0)
    assert np.array_equal(info, _expected_info(p))


CASES = {
    "plain_tiny": lambda: make_config("plain_tiny", seed=0),
    "plain_gpu": lambda: make_config("plain_gpu", seed=0),
    "one_element": lambda: make_problem(1, 1, 1, seed=2),
    "ng_tile_plus_one": lambda: make_problem(2, 3, 129, seed=3),
    "ng_below_block": lambda: make_problem(3, 5, 7, seed=4, fail_atoms=[2]),
    "nl_max_128": lambda: make_problem(2, 128, 200, seed=5, planted={1: 100}),
    "nl_64_planted": lambda: make_problem(3, 64, 385, seed=6, planted={0: 64, 2: 2}),
    "all_failing": lambda: make_problem(3, 9, 300, seed=7, fail_atoms=[0, 1, 2]),
    "mixed_nl": lambda: make_problem(6, [16, 49, 81, 121, 1, 128], 700, seed=8,
                                     fail_atoms=[2], planted={3: 50}),
    "long_contraction": lambda: make_problem(260, 128, 97, seed=10, fail_atoms=[5, 200]),
}


@pytest.mark.parametrize("name", list(CASES))
def test_full_parity(name):
    p = CASES[name]()
    r = _run(p)
    _check_full(p, *r.results())


def test_sync_entry_point_matches_async():
    from paper_1611_00606_amd import hs_build
    torch = _torch()
    p = make_config("plain_gpu", seed=1)
    r = _run(p)
    H1, S1, _ = r.results()
    H = torch.zeros_like(r.H)
    S = torch.zeros_like(r.S)
    hs_build(r.A, r.B, r.T_AA, r.T_AB, r.T_BB, r.U, p.N_A, 49, p.N_G, H, S)
    assert np.array_equal(H.cpu().numpy(), H1) and np.array_equal(S.cpu().numpy(), S1)


def test_deterministic_and_inputs_untouched():
    torch = _torch()
    p = make_problem(5, 33, 650, seed=9, fail_atoms=[4])
    r = _run(p)
    H1, S1, i1 = r.results()
    before = [t.clone() for t in (r.A, r.B, r.T_AA, r.T_AB, r.T_BB, r.U)]
    r.H.fill_(0)
    r.S.fill_(0)
    r.run()
    torch.cuda.synchronize()
    H2, S2, i2 = r.results()
    assert np.array_equal(H1, H2) and np.array_equal(S1, S2) and np.array_equal(i1, i2)
    for b, t in zip(before, (r.A, r.B, r.T_AA, r.T_AB, r.T_BB, r.U)):
        assert torch.equal(b, t)


def test_upper_triangles_of_hermitian_inputs_are_not_read():
    """Only the lower triangles of T_AA and T_BB (imaginary part of their
    diagonals excluded) define the operators."""
    torch = _torch()
    p = make_problem(3, 20, 260, seed=10, fail_atoms=[1])
    r = _run(p)
    H1, S1, i1 = r.results()
    q = p.copy()
    for name in ("T_AA", "T_BB"):
        for a in range(q.N_A):
            t = q.t_block(name, a).copy()
            t[np.triu_indices(20, 1)] = 1e30 + 7j
            t[np.diag_indices(20)] += 3j
            q.set_t_block(name, a, t)
    r2 = _run(q)
    H2, S2, i2 = r2.results()
    assert np.array_equal(H1, H2) and np.array_equal(S1, S2) and np.array_equal(i1, i2)


def test_nan_pivot_selects_failure_branch():
    p = make_problem(2, 12, 50, seed=11)
    t = p.t_block("T_AA", 1).copy()
    t[6, 6] = np.nan
    p.set_t_block("T_AA", 1, t)
    r = _run(p)
    assert r.info.cpu().numpy().tolist() == [0, 7]


def test_side_stream_and_no_info():
    from paper_1611_00606_amd import hs_build_ex
    torch = _torch()
    p = make_problem(4, 25, 333, seed=12, fail_atoms=[0])
    r = _run(p)
    H1, S1, _ = r.results()
    s = torch.cuda.Stream()
    H = torch.zeros_like(r.H)
    S = torch.zeros_like(r.S)
    with torch.cuda.stream(s):
        hs_build_ex(r.A, r.B, r.T_AA, r.T_AB, r.T_BB, r.U, p.N_A, 25, p.N_G, H, S,
                    workspace=r.workspace, info=None, stream=s)
    s.synchronize()
    assert np.array_equal(H.cpu().numpy(), H1) and np.array_equal(S.cpu().numpy(), S1)


def test_workspace_too_small_is_reported():
    from paper_1611_00606_amd import HSError, hs_build_ex
    torch = _torch()
    p = make_problem(2, 8, 40, seed=13)
    r = _run(p)
    small = torch.empty(r.workspace.numel() - 1, dtype=torch.uint8, device=r.workspace.device)
    with pytest.raises(HSError) as e:
        hs_build_ex(r.A, r.B, r.T_AA, r.T_AB, r.T_BB, r.U, p.N_A, 8, p.N_G, r.H, r.S,
                    workspace=small)
    assert e.value.status == 2


def _check_sampled(p, r, cols, n_probe=3):
    H, S = r.H, r.S
    torch = _torch()
    idx = torch.as_tensor(np.asarray(cols), device=H.device)
    Hc = H.index_select(1, idx).cpu().numpy()
    Sc = S.index_select(1, idx).cpu().numpy()
    Hr = O.hamiltonian_columns(p.A, p.B, p.T_AA, p.T_AB, p.T_BB, p.nl, cols)
    Sr = O.overlap_columns(p.A, p.B, p.U, p.nl, cols)
    for j, g in enumerate(cols):
        eh = np.linalg.norm(Hc[:, j] - Hr[:, j]) / np.linalg.norm(Hr[:, j])
        es = np.linalg.norm(Sc[:, j] - Sr[:, j]) / np.linalg.norm(Sr[:, j])
        assert eh <= TOL and es <= TOL, (g, eh, es)
    rng = np.random.default_rng(0)
    Hd = H.cpu().numpy()
    Sd = S.cpu().numpy()
    assert np.array_equal(Hd, Hd.conj().T) and np.array_equal(Sd, Sd.conj().T)
    fro_h, fro_s = np.linalg.norm(Hd), np.linalg.norm(Sd)
    for _ in range(n_probe):
        x, y = cn(rng, (p.N_G,)), cn(rng, (p.N_G,))
        h, s = O.bilinear(p.A, p.B, p.T_AA, p.T_AB, p.T_BB, p.U, p.nl, x, y)
        nx, ny = np.linalg.norm(x), np.linalg.norm(y)
        assert abs(y.conj() @ (Hd @ x) - h) <= TOL * fro_h * nx * ny
        assert abs(y.conj() @ (Sd @ x) - s) <= TOL * fro_s * nx * ny
    assert np.array_equal(r.info.cpu().numpy(), _expected_info(p))


@pytest.mark.parametrize("name", ["precision", "batching"])
def test_full_size_sampled(name):
    p = make_config(name, seed=0)
    r = _run(p)
    rng = np.random.default_rng(1)
    cols = sorted(set([0, 1, 127, 128, p.N_G // 2, p.N_G - 1] + rng.integers(0, p.N_G, 6).tolist()))
    _check_sampled(p, r, cols)
