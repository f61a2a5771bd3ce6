"""Reduction of the generalized eigenproblem (Sec. 1.1) on the GPU, through
the C ABI, against the CPU oracle (oracle.gep_reduce).

Tolerance: the Cholesky factor and L^-1 H L^-H computed in two different
FP64 summation orders differ by about cond(S) * u * sqrt(N) relative to
their norms. The overlaps here have cond(S) <= ~130 (measured on the built
workloads) and N <= 2000, i.e. ~1e-12 at the very worst; observed
differences are ~1e-15. Both outputs are held to the FP64 bar of the build,
1e-12 relative Frobenius error. The failing-pivot index is an integer
decision and must match exactly (planted with a clear margin).
"""

import numpy as np
import pytest
import scipy.linalg as sl

import oracle as O
from hs_inputs import make_config, make_problem, cn

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _torch():
    import torch
    return torch


def _rel(x, y):
    return np.linalg.norm(x - y) / np.linalg.norm(y)


def _random_pair(N, seed, shift=None):
    """Hermitian H and Hermitian positive definite S = A A^H + shift I."""
    rng = np.random.default_rng(seed)
    B = cn(rng, (N, N))
    H = B + B.conj().T
    A = cn(rng, (N, N))
    S = A @ A.conj().T + (N if shift is None else shift) * np.eye(N)
    S = 0.5 * (S + S.conj().T)
    return H, S


def _gep_gpu(H, S, stream=None, upper_garbage=False, mode=0):
    from paper_1611_00606_amd import hs_gep_reduce
    torch = _torch()
    N = H.shape[0]
    print(f"gep N={N} mode={mode}", flush=True)
    dev = torch.device("cuda:0")
    Sd = S.copy()
    if upper_garbage:
        Sd[np.triu_indices(N, 1)] = 1e300 - 5j
    Hg = torch.from_numpy(np.ascontiguousarray(H)).to(dev)
    Sg = torch.from_numpy(np.ascontiguousarray(Sd)).to(dev)
    L = torch.full((N, N), 7 + 7j, dtype=torch.complex128, device=dev)
    Ht = torch.full((N, N), 7 + 7j, dtype=torch.complex128, device=dev)
    info = torch.full((1,), -5, dtype=torch.int32, device=dev)
    hs_gep_reduce(Hg, Sg, L, Ht, info=info, stream=stream, mode=mode)
    torch.cuda.synchronize()
    assert np.array_equal(Hg.cpu().numpy(), H, equal_nan=True), "H modified"
    assert np.array_equal(Sg.cpu().numpy(), Sd, equal_nan=True), "S modified"
    return L.cpu().numpy(), Ht.cpu().numpy(), int(info.item())


def _check(H, S, L, Ht, info):
    L0, Ht0, inf0 = O.gep_reduce(H, S)
    assert inf0 == 0 and info == 0
    eL, eH = _rel(L, L0), _rel(Ht, Ht0)
    print(f"  rel err L {eL:.2e} Ht {eH:.2e}", flush=True)
    assert eL <= TOL and eH <= TOL, (eL, eH)
    assert np.all(np.triu(L, 1) == 0)
    assert np.all(L.diagonal().imag == 0) and np.all(L.diagonal().real > 0)
    assert np.array_equal(Ht, Ht.conj().T)
    assert np.all(Ht.diagonal().imag == 0)


@pytest.mark.parametrize("N", [1, 2, 63, 64, 65, 129, 300, 257])
def test_random_pairs(N):
    H, S = _random_pair(N, seed=100 + N)
    _check(H, S, *_gep_gpu(H, S))


def test_two_term_form_against_the_oracle():
    """N >= 4096 takes the form Ht = WH^H MH + MH^H WH (H split into its lower
    triangle and that triangle's conjugate transpose): full comparison at a
    size past the switch, with a ragged last panel."""
    H, S = _random_pair(4200, seed=42)
    _check(H, S, *_gep_gpu(H, S))


@pytest.mark.parametrize("mode", [0, 3])
@pytest.mark.parametrize("cond", [1e4, 1e8])
def test_ill_conditioned_overlap(cond, mode):
    """S with singular values spread over [1/cond, 1] (the paper's overlaps are
    positive definite up to a few very small singular values). Two correct
    FP64 orders of the reduction differ in Ht by about cond(S) u (u = 2^-53)
    and in L by about cond(S)^{1/2} u, so the comparison with the oracle uses
    10 cond(S) u for Ht and 10 N cond(S)^{1/2} u for L; the backward
    residuals do not grow with cond(S) for S = L L^H (1e-13) and grow with
    cond(L) = cond(S)^{1/2} for L Ht L^H = H (100 cond(S)^{1/2} u)."""
    u = 2.0 ** -53
    N = 600
    rng = np.random.default_rng(int(np.log10(cond)))
    Q, _ = np.linalg.qr(cn(rng, (N, N)))
    sv = np.logspace(0.0, -np.log10(cond), N)
    S = (Q * sv) @ Q.conj().T
    S = 0.5 * (S + S.conj().T)
    B = cn(rng, (N, N))
    H = B + B.conj().T
    L, Ht, info = _gep_gpu(H, S, mode=mode)
    L0, Ht0, inf0 = O.gep_reduce(H, S)
    assert info == 0 and inf0 == 0
    eL, eH = _rel(L, L0), _rel(Ht, Ht0)
    rS = np.linalg.norm(L @ L.conj().T - S) / np.linalg.norm(S)
    rH = np.linalg.norm(L @ Ht @ L.conj().T - H) / np.linalg.norm(H)
    print(f"  cond {cond:.0e} mode {mode}: L {eL:.2e} Ht {eH:.2e} res S {rS:.2e} res H {rH:.2e}",
          flush=True)
    assert eL <= 10 * N * np.sqrt(cond) * u
    assert eH <= 10 * cond * u
    assert rS <= 1e-13
    assert rH <= 100 * np.sqrt(cond) * u
    assert np.array_equal(Ht, Ht.conj().T)


def test_eigenvalues_match_generalized_problem():
    """Ht has the generalized eigenvalues of (H, S): the point of the reduction."""
    H, S = _random_pair(200, seed=7, shift=20.0)
    L, Ht, info = _gep_gpu(H, S)
    assert info == 0
    w = np.linalg.eigvalsh(Ht)
    w0 = sl.eigh(H, S, eigvals_only=True)
    err = np.max(np.abs(w - w0)) / np.max(np.abs(w0))
    print(f"  eigenvalue rel err {err:.2e}", flush=True)
    assert err <= TOL


def _built(p, name, mode=0):
    from paper_1611_00606_amd import DeviceBuild, hs_gep_reduce
    torch = _torch()
    r = DeviceBuild.from_problem(p)
    r.run()
    torch.cuda.synchronize()
    H, S, _ = r.results()
    L = torch.empty_like(r.H)
    Ht = torch.empty_like(r.H)
    info = torch.zeros(1, dtype=torch.int32, device=r.H.device)
    print(f"gep of built {name} N={p.N_G} mode={mode}", flush=True)
    hs_gep_reduce(r.H, r.S, L, Ht, info=info, mode=mode)
    torch.cuda.synchronize()
    return H, S, L.cpu().numpy(), Ht.cpu().numpy(), int(info.item())


# S = sum_a A_a^H A_a + B_a^H U_a^H U_a B_a has rank <= 2 K (K = sum_a N_L):
# these have 2 K >= N_G, so S is positive definite
BUILT = {
    "six_atoms": lambda: make_problem(6, 49, 300, seed=12, fail_atoms=[1]),
    "plain_gpu": lambda: make_config("plain_gpu", seed=0),
}


@pytest.mark.parametrize("name", list(BUILT))
def test_built_overlap_and_hamiltonian(name):
    """H and S straight from the GPU build, reduced on the GPU."""
    _check(*_built(BUILT[name](), name))


def test_rank_deficient_overlap_fails():
    """4 atoms x 16 rows: S has rank <= 2 K = 128 < N_G = 256, so a pivot at
    or after 129 is zero up to rounding and the reduction must report one
    (which one rounding decides: the oracle and the GPU may differ)."""
    p = make_config("plain_tiny", seed=0)
    H, S, L, Ht, info = _built(p, "plain_tiny")
    info0 = O.gep_reduce(H, S)[2]
    K = int(np.sum(p.nl))
    print(f"  info gpu {info} oracle {info0} (2K = {2 * K})", flush=True)
    assert 2 * K < info <= p.N_G and 2 * K < info0 <= p.N_G


def test_upper_triangle_of_s_is_not_read():
    H, S = _random_pair(190, seed=3)
    a = _gep_gpu(H, S)
    b = _gep_gpu(H, S, upper_garbage=True)
    assert all(np.array_equal(x, y) for x, y in zip(a[:2], b[:2])) and a[2] == b[2] == 0


def test_deterministic_on_a_side_stream():
    torch = _torch()
    H, S = _random_pair(333, seed=4)
    a = _gep_gpu(H, S)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b = _gep_gpu(H, S, stream=s)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_overlapping_calls_on_two_streams():
    """Two reductions enqueued back to back on two streams (sharing the
    library's streams) give the same bits as each alone; N = 1500 uses the
    lookahead and the background stream."""
    from paper_1611_00606_amd import hs_gep_reduce
    torch = _torch()
    dev = torch.device("cuda:0")
    pairs = [_random_pair(1500, seed=s) for s in (21, 22)]
    alone = [_gep_gpu(H, S) for H, S in pairs]
    ins = [(torch.from_numpy(H).to(dev), torch.from_numpy(S).to(dev)) for H, S in pairs]
    outs = [(torch.empty_like(h), torch.empty_like(h), torch.zeros(1, dtype=torch.int32, device=dev))
            for h, _ in ins]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    torch.cuda.synchronize()
    for (h, sm), (L, Ht, inf), st in zip(ins, outs, streams):
        with torch.cuda.stream(st):
            hs_gep_reduce(h, sm, L, Ht, info=inf, stream=st)
    torch.cuda.synchronize()
    for (L, Ht, inf), (La, Hta, ia) in zip(outs, alone):
        assert int(inf.item()) == ia == 0
        assert np.array_equal(L.cpu().numpy(), La) and np.array_equal(Ht.cpu().numpy(), Hta)


@pytest.mark.parametrize("N,pivot", [(150, 1), (150, 64), (150, 65), (300, 200), (300, 300)])
def test_failing_pivot_index(N, pivot):
    """S = M D M^H with D_pp < 0: the first pivot that is not > 0 is p
    (M unit lower, so the leading p-1 minors are positive definite)."""
    rng = np.random.default_rng(N + pivot)
    M = np.tril(0.3 * cn(rng, (N, N)), -1) + np.eye(N)
    d = rng.uniform(1.0, 2.0, N)
    d[pivot - 1] = -1.0
    S = (M * d) @ M.conj().T
    S = 0.5 * (S + S.conj().T)
    H, _ = _random_pair(N, seed=1)
    _, _, info0 = O.gep_reduce(H, S)
    assert info0 == pivot
    _, _, info = _gep_gpu(H, S)
    assert info == pivot


def test_nan_pivot():
    H, S = _random_pair(100, seed=5)
    S[70, 70] = np.nan
    assert O.gep_reduce(H, S)[2] == 71
    assert _gep_gpu(H, S)[2] == 71


def test_without_info_pointer_and_workspace_checks():
    from paper_1611_00606_amd import hs_gep_reduce, hs_gep_workspace_bytes
    torch = _torch()
    H, S = _random_pair(80, seed=6)
    dev = torch.device("cuda:0")
    Hg = torch.from_numpy(H).to(dev)
    Sg = torch.from_numpy(S).to(dev)
    L = torch.empty_like(Hg)
    Ht = torch.empty_like(Hg)
    small = torch.empty(hs_gep_workspace_bytes(80) - 256, dtype=torch.uint8, device=dev)
    assert hs_gep_reduce(Hg, Sg, L, Ht, workspace=small, check=False) == 2
    hs_gep_reduce(Hg, Sg, L, Ht)
    torch.cuda.synchronize()
    _check(H, S, L.cpu().numpy(), Ht.cpu().numpy(), 0)


def test_full_size_residuals():
    """N = 8000 (the large build workload): the outputs satisfy the defining
    identities S = L L^H and H = L Ht L^H to FP64 backward-error level,
    checked with plain complex128 products."""
    from paper_1611_00606_amd import DeviceBuild, hs_gep_reduce
    torch = _torch()
    p = make_config("precision", seed=0)
    r = DeviceBuild.from_problem(p)
    r.run()
    torch.cuda.synchronize()
    N = p.N_G
    L = torch.empty_like(r.H)
    Ht = torch.empty_like(r.H)
    info = torch.zeros(1, dtype=torch.int32, device=r.H.device)
    print(f"gep of built precision N={N}", flush=True)
    hs_gep_reduce(r.H, r.S, L, Ht, info=info)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    r1 = torch.linalg.matrix_norm(L @ L.conj().T - r.S) / torch.linalg.matrix_norm(r.S)
    r2 = torch.linalg.matrix_norm(L @ Ht @ L.conj().T - r.H) / torch.linalg.matrix_norm(r.H)
    print(f"  residual S {r1.item():.2e} H {r2.item():.2e}", flush=True)
    assert r1.item() <= 1e-13 and r2.item() <= 1e-12
    assert torch.equal(Ht, Ht.conj().T)
    assert torch.count_nonzero(torch.triu(L, 1)).item() == 0
    # sampled columns of Ht against the oracle's definition: Ht e_j = L^-1 H L^-H e_j
    Lc = L.cpu().numpy()
    Hc = r.H.cpu().numpy()
    for j in (0, 4095, N - 1):
        e = np.zeros(N, np.complex128)
        e[j] = 1.0
        col = sl.solve_triangular(Lc, Hc @ sl.solve_triangular(Lc, e, lower=True, trans="C"),
                                  lower=True)
        got = Ht[:, j].cpu().numpy()
        err = np.linalg.norm(got - col) / np.linalg.norm(col)
        print(f"  column {j} rel err {err:.2e}", flush=True)
        assert err <= TOL


def test_largest_size_residuals():
    """N = 16000: the inverse's recursion has 64 nodes at one depth, more than
    one batched launch holds, and the workspace is 20 GB. The outputs satisfy
    S = L L^H and H = L Ht L^H to backward-error level (complex128 products
    on the device) and a few columns of Ht match the definition."""
    from paper_1611_00606_amd import hs_gep_reduce
    torch = _torch()
    N = 16000
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev).manual_seed(16000)
    A = torch.randn(N, N, dtype=torch.complex128, device=dev, generator=g)
    S = A @ A.conj().T / N + torch.eye(N, dtype=torch.complex128, device=dev)
    S = 0.5 * (S + S.conj().T)
    H = torch.randn(N, N, dtype=torch.complex128, device=dev, generator=g)
    H = H + H.conj().T
    del A
    L = torch.empty_like(S)
    Ht = torch.empty_like(S)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    print(f"gep N={N}", flush=True)
    hs_gep_reduce(H, S, L, Ht, info=info)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    r1 = torch.linalg.matrix_norm(L @ L.conj().T - S) / torch.linalg.matrix_norm(S)
    r2 = torch.linalg.matrix_norm(L @ Ht @ L.conj().T - H) / torch.linalg.matrix_norm(H)
    print(f"  residual S {r1.item():.2e} H {r2.item():.2e}", flush=True)
    assert r1.item() <= 1e-13 and r2.item() <= 1e-12
    assert torch.equal(Ht, Ht.conj().T)
    assert torch.count_nonzero(torch.triu(L, 1)).item() == 0
    Lc = L.cpu().numpy()
    for j in (0, 8191, N - 1):
        e = np.zeros(N, np.complex128)
        e[j] = 1.0
        hcol = (H @ torch.from_numpy(sl.solve_triangular(Lc, e, lower=True, trans="C")).to(dev)).cpu().numpy()
        col = sl.solve_triangular(Lc, hcol, lower=True)
        err = np.linalg.norm(Ht[:, j].cpu().numpy() - col) / np.linalg.norm(col)
        print(f"  column {j} rel err {err:.2e}", flush=True)
        assert err <= TOL


# ---------------------------------------------------------------------------
# The products in the 3M form (hs_gep_reduce_ex with HS_FP64_3M). The 128x128
# diagonal blocks are still factored and inverted in the 4-product form; the
# 3M products change only the rounding (the imaginary parts' bound grows by a
# small constant factor), so the same bars hold.

@pytest.mark.parametrize("N", [1, 2, 65, 129, 300, 1100, 4200])
def test_3m_random_pairs(N):
    from paper_1611_00606_amd import HS_FP64_3M
    H, S = _random_pair(N, seed=700 + N)
    _check(H, S, *_gep_gpu(H, S, mode=HS_FP64_3M))


def test_3m_built_overlap_and_hamiltonian():
    from paper_1611_00606_amd import HS_FP64_3M
    _check(*_built(BUILT["plain_gpu"](), "plain_gpu", mode=HS_FP64_3M))


def test_3m_differs_from_fp64_by_rounding_and_is_deterministic():
    from paper_1611_00606_amd import HS_FP64, HS_FP64_3M
    H, S = _random_pair(1100, seed=71)
    L4, Ht4, i4 = _gep_gpu(H, S, mode=HS_FP64)
    L3, Ht3, i3 = _gep_gpu(H, S, mode=HS_FP64_3M)
    L3b, Ht3b, _ = _gep_gpu(H, S, mode=HS_FP64_3M)
    assert i4 == i3 == 0
    assert np.array_equal(L3, L3b) and np.array_equal(Ht3, Ht3b)
    assert not np.array_equal(Ht3, Ht4)   # the mode reached other kernels
    assert _rel(L3, L4) <= TOL and _rel(Ht3, Ht4) <= TOL


def test_3m_failing_pivot_index():
    from paper_1611_00606_amd import HS_FP64_3M
    H, S = _random_pair(300, seed=72)
    S[200, 200] = -1.0   # leading minor 201 not positive definite
    _, _, info = _gep_gpu(H, S, mode=HS_FP64_3M)
    assert info == O.gep_reduce(H, S)[2]


def test_3m_full_size_residuals():
    """N = 8000 in the 3M form: S = L L^H and H = L Ht L^H to the same
    backward-error bars as the 4-product form."""
    from paper_1611_00606_amd import DeviceBuild, HS_FP64_3M, hs_gep_reduce
    torch = _torch()
    p = make_config("precision", seed=0)
    r = DeviceBuild.from_problem(p)
    r.run()
    torch.cuda.synchronize()
    L = torch.empty_like(r.H)
    Ht = torch.empty_like(r.H)
    info = torch.zeros(1, dtype=torch.int32, device=r.H.device)
    print(f"gep 3M of built precision N={p.N_G}", flush=True)
    hs_gep_reduce(r.H, r.S, L, Ht, info=info, mode=HS_FP64_3M)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    r1 = torch.linalg.matrix_norm(L @ L.conj().T - r.S) / torch.linalg.matrix_norm(r.S)
    r2 = torch.linalg.matrix_norm(L @ Ht @ L.conj().T - r.H) / torch.linalg.matrix_norm(r.H)
    print(f"  residual S {r1.item():.2e} H {r2.item():.2e}", flush=True)
    assert r1.item() <= 1e-13 and r2.item() <= 1e-12
    assert torch.equal(Ht, Ht.conj().T)
    assert torch.count_nonzero(torch.triu(L, 1)).item() == 0
