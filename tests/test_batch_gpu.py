"""Batched per-atom stage (hs_options.batch = 1) through the C ABI.

The persistent launch prepares every atom and computes every Z_a, W_a tile
with the tile shape of its N_L. Each tile runs the same contraction order as
the separate launches (stages of 16 rows, MFMA K steps of 4), so H, S and
info are compared BITWISE with the unbatched build, for every tile shape,
and the batched build is also checked against the CPU oracle (relative
Frobenius error <= 1e-12, exact info).
"""

import numpy as np
import pytest

import oracle as O
from hs_inputs import make_config, make_problem

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _run(p, **kw):
    import torch
    from paper_1611_00606_amd import DeviceBuild
    print(f"case N_A={p.N_A} nl={sorted(set(p.nl.tolist()))} N_G={p.N_G} {kw}", flush=True)
    r = DeviceBuild.from_problem(p, **kw)
    r.run()
    torch.cuda.synchronize()
    return r


def _expected_info(p):
    info = np.zeros(p.N_A, np.int32)
    for a in p.failing:
        info[a] = 1
    for a, piv in p.planted.items():
        info[a] = piv
    return info


def _rel(x, y):
    return np.linalg.norm(x - y) / np.linalg.norm(y)


def _uniform(c):
    from paper_1611_00606_amd.tuning import tuning_from_table
    return tuning_from_table({v: c for v in range(1, 129)})


CASES = {
    "mixed_failing": lambda: make_problem(6, [16, 49, 81, 121, 1, 128], 700, seed=8,
                                          fail_atoms=[2], planted={3: 50}),
    "ragged_small": lambda: make_problem(5, [3, 17, 33, 65, 2], 131, seed=11, fail_atoms=[4]),
    "one_element": lambda: make_problem(1, 1, 1, seed=2),
    "nl_max_128": lambda: make_problem(2, 128, 200, seed=5, planted={1: 100}),
}


@pytest.mark.parametrize("name", list(CASES))
def test_batch_parity(name):
    p = CASES[name]()
    rb = _run(p, batch=1)
    H, S, info = rb.results()
    Hr = O.hamiltonian(p.A, p.B, p.T_AA, p.T_AB, p.T_BB, p.nl)
    Sr = O.overlap(p.A, p.B, p.U, p.nl)
    eh, es = _rel(H, Hr), _rel(S, Sr)
    print(f"  batched rel err H {eh:.2e} S {es:.2e}", flush=True)
    assert eh <= TOL and es <= TOL
    assert np.array_equal(info, _expected_info(p))
    r0 = _run(p, batch=0)
    H0, S0, info0 = r0.results()
    assert np.array_equal(H, H0) and np.array_equal(S, S0) and np.array_equal(info, info0)


@pytest.mark.parametrize("shape", range(8))
def test_every_tile_shape_matches_unbatched(shape):
    from paper_1611_00606_amd import HS_NUM_TILE_CONFIGS
    assert HS_NUM_TILE_CONFIGS == 8
    p = make_problem(7, [16, 49, 81, 121, 5, 128, 33], 523, seed=12, fail_atoms=[1],
                     planted={2: 30})
    r0 = _run(p, batch=0)
    H0, S0, info0 = r0.results()
    rb = _run(p, batch=1, tuning=_uniform(shape))
    H, S, info = rb.results()
    assert np.array_equal(H, H0) and np.array_equal(S, S0)
    assert np.array_equal(info, info0) and np.array_equal(info, _expected_info(p))


def test_many_atoms_queue():
    """600 atoms (three table chunks), N_L 1..24, many queue items per block."""
    rng = np.random.default_rng(3)
    nl = rng.integers(1, 25, size=600).tolist()
    p = make_problem(600, nl, 257, seed=13, n_fail=30)
    rb = _run(p, batch=1)
    H, S, info = rb.results()
    r0 = _run(p, batch=0)
    H0, S0, info0 = r0.results()
    assert np.array_equal(H, H0) and np.array_equal(S, S0) and np.array_equal(info, info0)
    assert np.array_equal(info, _expected_info(p))


def test_batch_deterministic_and_split():
    import torch
    p = make_problem(4, [16, 81, 121, 49], 400, seed=14, fail_atoms=[0])
    rb = _run(p, batch=1)
    H1, S1, _ = rb.results()
    rb.H.zero_()
    rb.S.zero_()
    rb.run()
    torch.cuda.synchronize()
    H2, S2, _ = rb.results()
    assert np.array_equal(H1, H2) and np.array_equal(S1, S2)
    rs = _run(p, batch=1, mode=1)
    Hs, Ss, info = rs.results()
    assert _rel(Hs, H1) <= 1e-9 and _rel(Ss, S1) <= 1e-9
    assert np.array_equal(info, _expected_info(p))


def test_batch_in_context():
    """Context builds with batch = 1 reuse the cached preparation."""
    import torch
    from paper_1611_00606_amd.serving import Context
    p = make_problem(5, [16, 49, 81, 121, 7], 450, seed=15, fail_atoms=[3])
    ctx = Context(p.T_AA, p.T_AB, p.T_BB, p.U, p.nl)
    dev = torch.device("cuda:0")
    A = torch.from_numpy(p.A).to(dev)
    Bm = torch.from_numpy(p.B).to(dev)
    out = []
    for batch in (0, 1):
        H = torch.empty((p.N_G, p.N_G), dtype=torch.complex128, device=dev)
        S = torch.empty_like(H)
        ws = torch.empty(ctx.workspace_bytes(p.N_G), dtype=torch.uint8, device=dev)
        ctx.build(A, Bm, p.N_G, H, S, ws, batch=batch, tuning=_uniform(0) if batch else None)
        torch.cuda.synchronize()
        out.append((H.cpu().numpy(), S.cpu().numpy()))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    assert np.array_equal(ctx.info(), _expected_info(p))
    ctx.close()


def test_autotuner():
    from paper_1611_00606_amd import HS_NUM_TILE_CONFIGS, hs_autotune_atoms, hs_tile_config
    vals = [16, 121, 16]
    t, ms = hs_autotune_atoms(vals, 1000, reps=2)
    print("  autotune ms", ms.tolist(), flush=True)
    assert ms.shape == (3, HS_NUM_TILE_CONFIGS) and np.all(ms > 0) and np.all(np.isfinite(ms))
    assert np.array_equal(ms[0], ms[2])
    for i, v in enumerate(vals):
        assert t.cfg[v] == int(np.argmin(ms[i]))
        assert hs_tile_config(t.cfg[v]) is not None


def test_batching_workload_sampled():
    """The 128-atom mixed-N_L workload at N_G = 6000, tuned shapes: bitwise
    equal to the unbatched build (and the oracle on sampled columns)."""
    import torch
    from paper_1611_00606_amd.tuning import autotune
    p = make_config("batching", seed=0)
    tuning, report = autotune(sorted(set(p.nl.tolist())), p.N_G, reps=2)
    print("  tuned", {v: r["bm_bn"] for v, r in report.items()}, flush=True)
    rb = _run(p, batch=1, tuning=tuning)
    cols = [0, 1, 2999, p.N_G - 1]
    idx = torch.as_tensor(cols, device=rb.H.device)
    Hb = rb.H.index_select(1, idx).cpu().numpy()
    Sb = rb.S.index_select(1, idx).cpu().numpy()
    info = rb.info.cpu().numpy()
    del rb
    torch.cuda.empty_cache()
    r0 = _run(p, batch=0)
    assert np.array_equal(Hb, r0.H.index_select(1, idx).cpu().numpy())
    assert np.array_equal(Sb, r0.S.index_select(1, idx).cpu().numpy())
    assert np.array_equal(info, _expected_info(p))
    Hr = O.hamiltonian_columns(p.A, p.B, p.T_AA, p.T_AB, p.T_BB, p.nl, cols)
    assert _rel(Hb, Hr) <= TOL


def test_autotune_cache_round_trip(tmp_path):
    """The tuner's JSON cache: a first call measures and stores, a second
    reads the same choices back without measuring, a new N_L is measured
    alone and added, and a build with the cached table is bitwise the one
    with the measured table."""
    import json
    from paper_1611_00606_amd.tuning import autotune
    cache = str(tmp_path / "tune.json")
    n_g = 600
    t1, r1 = autotune([16, 81], n_g, reps=1, cache=cache)
    assert all(r1[v]["ms"] is not None for v in (16, 81))
    stored = json.load(open(cache))
    assert sorted(k.split("/")[-1] for k in stored) == ["N_L=16", "N_L=81"]
    assert all(f"N_G={n_g}" in k for k in stored)
    t2, r2 = autotune([81, 16], n_g, reps=1, cache=cache)
    assert all(r2[v]["ms"] is None for v in (16, 81))   # read back, not measured
    assert bytes(t1.cfg) == bytes(t2.cfg)
    t3, r3 = autotune([16, 49, 81], n_g, reps=1, cache=cache)
    assert r3[49]["ms"] is not None and r3[16]["ms"] is None and r3[81]["ms"] is None
    assert len(json.load(open(cache))) == 3
    assert t3.cfg[16] == t1.cfg[16] and t3.cfg[81] == t1.cfg[81]
    p = make_problem(3, [16, 81, 49], n_g, seed=31, fail_atoms=[1])
    ra = _run(p, batch=1, tuning=t3)
    Ha, Sa, ia = ra.results()
    from paper_1611_00606_amd.tuning import tuning_from_table
    rb = _run(p, batch=1, tuning=tuning_from_table({v: int(t3.cfg[v]) for v in (16, 49, 81)}))
    Hb, Sb, ib = rb.results()
    assert np.array_equal(Ha, Hb) and np.array_equal(Sa, Sb) and np.array_equal(ia, ib)
    assert _rel(Ha, O.hamiltonian(p.A, p.B, p.T_AA, p.T_AB, p.T_BB, p.nl)) <= TOL
