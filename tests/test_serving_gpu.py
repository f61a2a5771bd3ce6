"""Serving form on the GPU: resident context, continuous batching.

* a context build equals the one-shot build bitwise (same kernels, cached
  atom-side data);
* every request's H and S are the same alone and in a mix of concurrently
  admitted requests (bitwise: the kernels are deterministic);
* the arena never holds more than its budget while requests are admitted;
* served results match the CPU oracle.
"""

import ctypes

import numpy as np
import pytest

import oracle as O
from hs_inputs import make_problem

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
