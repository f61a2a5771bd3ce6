"""Serving form on the GPU: resident context, continuous batching.

* a context build equals the one-shot build bitwise (same kernels, cached
  atom-side data);
* every request's H and S are the same alone and in a mix of concurrently
  admitted requests (bitwise: the kernels are deterministic);
* the arena never holds more than its budget while requests are admitted;
* served results match the CPU oracle;
* on the serving workload's own atom set (64 atoms, N_L = 64) and request
  sizes (N_G 1500..9000, fresh A, B per request), in every reduction
  mode: every request alone against the oracle (sampled columns, bilinear
  probe), and bitwise the same result in a contended mix.
"""

import ctypes

import numpy as np
import pytest

import oracle as O
from hs_inputs import make_problem
from _parity import MODE_NAME, MODE_TOL, check_columns_and_probes, rel, sample_columns

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _torch():
    import torch
    return torch


def _pinned(x):
    torch = _torch()
    t = torch.empty(x.shape, dtype=torch.complex128, pin_memory=True)
    t.numpy()[...] = x
    return t


@pytest.fixture(scope="module")
def atoms():
    # 5 atoms of mixed N_L, one taking the failure branch, one planted pivot
    return make_problem(5, [16, 49, 25, 64, 9], 1, seed=21, fail_atoms=[2], planted={3: 30})


@pytest.fixture(scope="module")
def ctx(atoms):
    from paper_1611_00606_amd.serving import Context
    c = Context(atoms.T_AA, atoms.T_AB, atoms.T_BB, atoms.U, atoms.nl)
    yield c
    c.close()


def _requests(atoms, sizes, seed):
    """Request r: A, B of N_G = sizes[r] drawn for the context's atoms."""
    out = []
    for r, n_g in enumerate(sizes):
        p = make_problem(atoms.N_A, atoms.nl, int(n_g), seed=seed + r)
        out.append((int(n_g), p.A, p.B))
    return out


def test_context_build_equals_one_shot(atoms, ctx):
    from paper_1611_00606_amd import DeviceBuild
    torch = _torch()
    assert np.array_equal(ctx.info(), np.array([0, 0, 1, 30, 0], np.int32))
    n_g = 700
    q = make_problem(atoms.N_A, atoms.nl, n_g, seed=3)
    q.T_AA, q.T_AB, q.T_BB, q.U = atoms.T_AA, atoms.T_AB, atoms.T_BB, atoms.U
    r = DeviceBuild.from_problem(q)
    r.run()
    torch.cuda.synchronize()
    H1, S1, _ = r.results()
    dev = torch.device("cuda:0")
    A = torch.from_numpy(q.A).to(dev)
    Bm = torch.from_numpy(q.B).to(dev)
    H = torch.empty((n_g, n_g), dtype=torch.complex128, device=dev)
    S = torch.empty_like(H)
    ws = torch.empty(ctx.workspace_bytes(n_g), dtype=torch.uint8, device=dev)
    ctx.build(A, Bm, n_g, H, S, ws)
    torch.cuda.synchronize()
    assert np.array_equal(H.cpu().numpy(), H1) and np.array_equal(S.cpu().numpy(), S1)


def _serve(ctx, reqs, arrivals, n_slots, arena, keep):
    from paper_1611_00606_amd.serving import ServingLoop, device_matrix_to_host
    pins = [(_pinned(A), _pinned(Bm)) for _, A, Bm in reqs]
    rq = [{"id": i, "N_G": n_g, "A_ptr": pins[i][0].data_ptr(), "B_ptr": pins[i][1].data_ptr(),
           "ld": n_g} for i, (n_g, _, _) in enumerate(reqs)]
    got = {}

    def on_result(res):
        if res["id"] in keep:
            got[res["id"]] = (device_matrix_to_host(res["H"], res["N_G"]),
                              device_matrix_to_host(res["S"], res["N_G"]))

    loop = ServingLoop(ctx, n_slots, arena)
    recs = loop.run(rq, arrivals, on_result=on_result)
    peak = loop.peak_bytes
    loop.close()
    return recs, got, peak


def test_alone_equals_mix_and_budget(atoms, ctx):
    sizes = [300, 1100, 257, 900, 640, 1500, 128, 1024]
    reqs = _requests(atoms, sizes, seed=100)
    keep = set(range(len(sizes)))
    # alone: one slot, arrivals far apart, one request at a time
    alone = {}
    for i in range(len(reqs)):
        _, got, _ = _serve(ctx, [reqs[i]], [0.0], 1, ctx.footprint_bytes(reqs[i][0]), {0})
        alone[i] = got[0]
    # mix: burst of arrivals, 3 slots, an arena that holds about 3 requests
    arena = int(3.2 * max(ctx.footprint_bytes(n) for n in sizes))
    recs, got, peak = _serve(ctx, reqs, [0.0] * len(reqs), 3, arena, keep)
    assert peak <= arena
    assert len(recs) == len(reqs)
    # several requests were in flight together
    overl = sum(1 for a in recs for b in recs if a["id"] < b["id"]
                and a["admit"] < b["done"] and b["admit"] < a["done"])
    assert overl >= 1
    for i in range(len(reqs)):
        assert np.array_equal(alone[i][0], got[i][0]), i
        assert np.array_equal(alone[i][1], got[i][1]), i


def test_served_results_match_oracle(atoms, ctx):
    sizes = [450, 777]
    reqs = _requests(atoms, sizes, seed=200)
    recs, got, _ = _serve(ctx, reqs, [0.0, 0.001], 2, 10 * ctx.footprint_bytes(777), {0, 1})
    for i, (n_g, A, Bm) in enumerate(reqs):
        Hr = O.hamiltonian(A, Bm, atoms.T_AA, atoms.T_AB, atoms.T_BB, atoms.nl)
        Sr = O.overlap(A, Bm, atoms.U, atoms.nl)
        H, S = got[i]
        assert np.linalg.norm(H - Hr) / np.linalg.norm(Hr) <= TOL
        assert np.linalg.norm(S - Sr) / np.linalg.norm(Sr) <= TOL
        assert np.array_equal(H, H.conj().T)


def test_oversized_request_is_rejected(atoms, ctx):
    from paper_1611_00606_amd import HSError, hs_server_create, hs_server_destroy, hs_server_submit
    srv = hs_server_create(ctx.handle, 1, ctx.footprint_bytes(100))
    buf = np.zeros((ctx.K, 200), np.complex128)
    with pytest.raises(HSError) as e:
        hs_server_submit(srv, 1, 200, buf.ctypes.data, buf.ctypes.data, 200)
    assert e.value.status == 3
    hs_server_destroy(srv)


# --------------------------------------------------------------------------
# The serving workload itself: 64 atoms of N_L = 64 resident, requests with
# fresh seeded A, B and N_G from 1500 to 9000, in every reduction mode.
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def c5_atoms():
    from hs_inputs import serving_atoms
    return serving_atoms(0)


@pytest.fixture(scope="module")
def c5_ctx(c5_atoms):
    from paper_1611_00606_amd.serving import Context
    a = c5_atoms
    c = Context(a.T_AA, a.T_AB, a.T_BB, a.U, a.nl)
    yield c
    c.close()


@pytest.fixture(scope="module")
def c5_requests(c5_atoms):
    """Eight requests: the smallest and largest N_G of the range and the first
    six sizes of the seeded stream, each with its own A, B (pinned host)."""
    from concurrent.futures import ThreadPoolExecutor
    from hs_inputs import serving_request_ab, serving_requests
    sizes = [1500, 9000] + [int(x) for x in serving_requests(0)[:6]]
    K = c5_atoms.K

    def one(r):
        A, Bm = serving_request_ab(0, r, sizes[r], K)
        return sizes[r], _pinned(A), _pinned(Bm)

    with ThreadPoolExecutor(4) as ex:
        return list(ex.map(one, range(len(sizes))))


def _serve_mode(ctx, reqs, arrivals, n_slots, arena, mode, on_host):
    """Serve pinned requests [(N_G, A, B)] in `mode`; on_host(i, H, S) gets
    host copies of every result."""
    from paper_1611_00606_amd.serving import ServingLoop, device_matrix_to_host
    rq = [{"id": i, "N_G": n_g, "A_ptr": A.data_ptr(), "B_ptr": Bm.data_ptr(), "ld": n_g}
          for i, (n_g, A, Bm) in enumerate(reqs)]

    def on_result(res):
        n = res["N_G"]
        on_host(res["id"], device_matrix_to_host(res["H"], n), device_matrix_to_host(res["S"], n))

    loop = ServingLoop(ctx, n_slots, arena, mode=mode)
    recs = loop.run(rq, arrivals, on_result=on_result)
    peak = loop.peak_bytes
    loop.close()
    return recs, peak


@pytest.mark.parametrize("mode", [0, 1, 2, 3, 4, 5], ids=lambda m: MODE_NAME[m])
def test_serving_workload_alone_equals_mix_and_oracle(c5_atoms, c5_ctx, c5_requests, mode):
    """Each request alone (one slot, nothing else in flight): sampled columns
    and bilinear probes against the oracle. Then all eight arrive at once on
    three slots with an arena that holds about three of them: the arena
    stays within its budget, requests overlap and queue, and every result is
    bitwise the one served alone."""
    a, ctx, reqs = c5_atoms, c5_ctx, c5_requests
    tol = MODE_TOL[mode]
    alone = {}
    for i, (n_g, A, Bm) in enumerate(reqs):
        print(f"case serving request {i} N_G={n_g} mode={MODE_NAME[mode]} alone", flush=True)

        def keep(_, H, S, i=i):
            alone[i] = (H, S)

        _serve_mode(ctx, [reqs[i]], [0.0], 1, ctx.footprint_bytes(n_g, mode), mode, keep)
        H, S = alone[i]
        cols = sample_columns(n_g, seed=i, n_random=2)
        check_columns_and_probes(A.numpy(), Bm.numpy(), a.T_AA, a.T_AB, a.T_BB, a.U, a.nl,
                                 H, S, cols, tol, n_probe=1, probe_seed=i)
    arena = int(3.2 * max(ctx.footprint_bytes(n, mode) for n, _, _ in reqs))
    same = {}

    def compare(i, H, S):
        same[i] = bool(np.array_equal(H, alone[i][0]) and np.array_equal(S, alone[i][1]))

    print(f"case serving mix of {len(reqs)} mode={MODE_NAME[mode]}", flush=True)
    recs, peak = _serve_mode(ctx, reqs, [0.0] * len(reqs), 3, arena, mode, compare)
    assert peak <= arena
    assert len(recs) == len(reqs)
    overl = sum(1 for x in recs for y in recs if x["id"] < y["id"]
                and x["admit"] < y["done"] and y["admit"] < x["done"])
    assert overl >= 1
    assert max(r["admit"] - r["submit"] for r in recs) > 0.0   # someone queued
    assert all(same[i] for i in range(len(reqs))), same


@pytest.mark.parametrize("mode", [0, 1, 2, 3, 4, 5], ids=lambda m: MODE_NAME[m])
def test_context_complex_u_matches_oracle(mode):
    """The resident context keeps |u|^2 of a complex U (its S matches the oracle)."""
    from paper_1611_00606_amd.serving import Context
    torch = _torch()
    atoms = make_problem(4, [16, 49, 25, 64], 1, seed=51, fail_atoms=[1], complex_u=True)
    q = make_problem(atoms.N_A, atoms.nl, 411, seed=52)
    ctx = Context(atoms.T_AA, atoms.T_AB, atoms.T_BB, atoms.U, atoms.nl)
    try:
        dev = torch.device("cuda:0")
        A = torch.from_numpy(q.A).to(dev)
        Bm = torch.from_numpy(q.B).to(dev)
        H = torch.empty((q.N_G, q.N_G), dtype=torch.complex128, device=dev)
        S = torch.empty_like(H)
        ws = torch.empty(ctx.workspace_bytes(q.N_G, mode), dtype=torch.uint8, device=dev)
        ctx.build(A, Bm, q.N_G, H, S, ws, mode=mode)
        torch.cuda.synchronize()
        Hr = O.hamiltonian(q.A, q.B, atoms.T_AA, atoms.T_AB, atoms.T_BB, atoms.nl)
        Sr = O.overlap(q.A, q.B, atoms.U, atoms.nl)
        eh = rel(H.cpu().numpy(), Hr)
        es = rel(S.cpu().numpy(), Sr)
        print(f"  context complex U mode={MODE_NAME[mode]} rel err H {eh:.2e} S {es:.2e}", flush=True)
        assert eh <= MODE_TOL[mode] and es <= MODE_TOL[mode]
    finally:
        ctx.close()
