"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: every check has an independent
source (a hand-worked example, a closed form of a special case, an invariant,
a library routine, or a second derivation through Alg. 1's own steps).
"""

import os

import numpy as np
import pytest
import scipy.linalg

import oracle as O
from hs_inputs import make_config, make_problem, cn

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _H(p):
    return O.hamiltonian(p.A, p.B, p.T_AA, p.T_AB, p.T_BB, p.nl)


def _S(p):
    return O.overlap(p.A, p.B, p.U, p.nl)


def _rel(x, y):
    return np.linalg.norm(x - y) / np.linalg.norm(y)


@pytest.fixture(scope="module")
def tiny():
    return make_config("plain_tiny", seed=3)


@pytest.fixture(scope="module")
def mid():
    return make_config("plain_gpu", seed=0)


# P1: the matrix form equals the literal index sums (Sec. 1.1 vs Sec. 2).
@pytest.mark.parametrize("nl,fail", [(4, []), ([1, 3, 4], [2]), ([2, 4], [0])])
def test_entrywise_equals_matrix_form(nl, fail):
    n_a = 3 if np.isscalar(nl) else len(nl)
    p = make_problem(n_a, nl, 8, seed=11, fail_atoms=fail)
    H0 = O.hamiltonian_entrywise(p.A, p.B, p.T_AA, p.T_AB, p.T_BB, p.nl)
    S0 = O.overlap_entrywise(p.A, p.B, p.U, p.nl)
    assert _rel(_H(p), H0) <= 1e-14
    assert _rel(_S(p), S0) <= 1e-14


def test_einsum_triple_sum_on_tiny_config(tiny):
    """The plain_tiny case through an unoptimised triple-sum einsum per atom."""
    p = tiny
    H = np.zeros((p.N_G, p.N_G), complex)
    S = np.zeros((p.N_G, p.N_G), complex)
    r = 0
    for a in range(p.N_A):
        n = int(p.nl[a])
        Aa, Ba, u = p.A[r:r + n], p.B[r:r + n], p.U[r:r + n]
        tab = p.t_block("T_AB", a)
        for X, T, Y in ((Aa, p.t_block("T_AA", a), Aa), (Aa, tab, Ba),
                        (Ba, tab.conj().T, Aa), (Ba, p.t_block("T_BB", a), Ba)):
            H += np.einsum("lp,lm,mq->pq", X.conj(), T, Y, optimize=False)
        S += np.einsum("lp,lq->pq", Aa.conj(), Aa, optimize=False)
        S += np.einsum("l,lp,lq->pq", np.abs(u) ** 2, Ba.conj(), Ba, optimize=False)
        r += n
    assert _rel(_H(p), H) <= 1e-14
    assert _rel(_S(p), S) <= 1e-14


# P2: a hand-worked example with exact Gaussian-integer arithmetic.
def test_hand_worked_scalar_atom():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "scalar_atom.txt"))
            if l.strip() and not l.startswith("#")]
    A = np.array([[1 + 2j, 3 - 1j]])
    B = np.array([[2 + 0j, -1 + 1j]])
    nl = np.array([1], np.int32)
    H = O.hamiltonian(A, B, np.array([2 + 0j]), np.array([1 + 1j]), np.array([-1 + 0j]), nl)
    S = O.overlap(A, B, np.array([2j]), nl)
    for m, gp, g, re, im in rows:
        got = {"H": H, "S": S}[m][int(gp) - 1, int(g) - 1]
        assert got == complex(float(re), float(im)), (m, gp, g, got)


# P3: closed forms of S for U = I and U = 0.
def test_overlap_closed_forms(mid):
    p = mid.copy()
    p.U[:] = 1.0
    stacked = p.A.conj().T @ p.A + p.B.conj().T @ p.B
    assert _rel(_S(p), stacked) <= 1e-13
    p.U[:] = 0.0
    assert _rel(_S(p), p.A.conj().T @ p.A) <= 1e-13


# P4: H_AA closed forms, and the cross-pin H(T_AA = I, rest 0) == S(U = 0).
def test_hamiltonian_closed_forms(mid):
    p = mid.copy()
    p.T_AB[:] = 0
    p.T_BB[:] = 0
    for a in range(p.N_A):
        p.set_t_block("T_AA", a, np.eye(int(p.nl[a])))
    AhA = p.A.conj().T @ p.A
    assert _rel(_H(p), AhA) <= 1e-13
    q = p.copy()
    q.U[:] = 0
    assert _rel(_H(p), _S(q)) <= 1e-13
    for a in range(p.N_A):
        p.set_t_block("T_AA", a, (2.5 - 0.0j) * np.eye(int(p.nl[a])))
    assert _rel(_H(p), 2.5 * AhA) <= 1e-13


# P5, P6: Hermiticity of both; S positive semidefinite (Sec. 1.1).
def test_hermitian_and_psd(mid):
    H, S = _H(mid), _S(mid)
    assert np.linalg.norm(H - H.conj().T) <= 1e-14 * np.linalg.norm(H)
    assert np.linalg.norm(S - S.conj().T) <= 1e-14 * np.linalg.norm(S)
    ev = np.linalg.eigvalsh(S)
    assert ev.min() >= -1e-13 * ev.max()
    evh = np.linalg.eigvalsh(H)
    assert evh.min() < 0 < evh.max()     # H is not definite


# P7: invariance under a unitary change of the per-atom (l,m) basis.
def test_unitary_invariance():
    p = make_problem(3, 6, 40, seed=5, fail_atoms=[1])
    q = p.copy()
    rng = np.random.default_rng(9)
    r = 0
    for a in range(p.N_A):
        n = int(p.nl[a])
        Q, _ = np.linalg.qr(cn(rng, (n, n)))
        q.A[r:r + n] = Q @ p.A[r:r + n]
        q.B[r:r + n] = Q @ p.B[r:r + n]
        for name in ("T_AA", "T_AB", "T_BB"):
            q.set_t_block(name, a, Q @ p.t_block(name, a) @ Q.conj().T)
        r += n
    assert _rel(_H(q), _H(p)) <= 1e-13
    # a permutation of the rows (with U permuted alike) leaves S unchanged too
    q = p.copy()
    r = 0
    for a in range(p.N_A):
        n = int(p.nl[a])
        perm = rng.permutation(n)
        for name in ("A", "B", "U"):
            getattr(q, name)[r:r + n] = getattr(p, name)[r:r + n][perm]
        P = np.eye(n)[perm]
        for name in ("T_AA", "T_AB", "T_BB"):
            q.set_t_block(name, a, P @ p.t_block(name, a) @ P.T)
        r += n
    assert _rel(_S(q), _S(p)) <= 1e-14
    assert _rel(_H(q), _H(p)) <= 1e-13


# P8: H is real-linear in the T matrices jointly (T^BA = T^AB^H makes it
# conjugate-linear in T^AB, so complex coefficients would not pass through);
# S does not see T, H does not see U.
def test_linearity_and_independence():
    p = make_problem(3, 5, 30, seed=6)
    q = make_problem(3, 5, 30, seed=7)
    pq = p.copy()
    for name in ("T_AA", "T_AB", "T_BB"):
        setattr(pq, name, 2.0 * getattr(p, name) - 0.5 * getattr(q, name))
    H = O.hamiltonian(p.A, p.B, pq.T_AA, pq.T_AB, pq.T_BB, p.nl)
    Hp = _H(p)
    Hq = O.hamiltonian(p.A, p.B, q.T_AA, q.T_AB, q.T_BB, p.nl)
    assert _rel(H, 2.0 * Hp - 0.5 * Hq) <= 1e-13
    r = p.copy()
    r.T_AA, r.T_AB, r.T_BB = q.T_AA, q.T_AB, q.T_BB
    assert np.array_equal(_S(r), _S(p))
    r = p.copy()
    r.U = q.U
    assert np.array_equal(_H(r), _H(p))


# P9: additivity over atoms (also pins mixed-N_L packing).
def test_atom_additivity():
    p = make_problem(5, [3, 6, 2, 6, 4], 50, seed=8, fail_atoms=[3])
    m = 2
    k1 = int(p.nl[:m].sum())
    t1 = int((p.nl[:m].astype(int) ** 2).sum())
    H1 = O.hamiltonian(p.A[:k1], p.B[:k1], p.T_AA[:t1], p.T_AB[:t1], p.T_BB[:t1], p.nl[:m])
    H2 = O.hamiltonian(p.A[k1:], p.B[k1:], p.T_AA[t1:], p.T_AB[t1:], p.T_BB[t1:], p.nl[m:])
    S1 = O.overlap(p.A[:k1], p.B[:k1], p.U[:k1], p.nl[:m])
    S2 = O.overlap(p.A[k1:], p.B[k1:], p.U[k1:], p.nl[m:])
    assert _rel(_H(p), H1 + H2) <= 1e-14
    assert _rel(_S(p), S1 + S2) <= 1e-14


# P10: bilinear probes y^H H x, y^H S x through per-atom vectors.
def test_bilinear_probe(mid):
    H, S = _H(mid), _S(mid)
    rng = np.random.default_rng(1)
    for _ in range(3):
        x, y = cn(rng, (mid.N_G,)), cn(rng, (mid.N_G,))
        h, s = O.bilinear(mid.A, mid.B, mid.T_AA, mid.T_AB, mid.T_BB, mid.U, mid.nl, x, y)
        assert abs(h - y.conj() @ H @ x) <= 1e-12 * np.linalg.norm(H) * np.linalg.norm(x) * np.linalg.norm(y)
        assert abs(s - y.conj() @ S @ x) <= 1e-12 * np.linalg.norm(S) * np.linalg.norm(x) * np.linalg.norm(y)


def test_column_forms(mid):
    cols = [0, 7, 999, mid.N_G - 1]
    Hc = O.hamiltonian_columns(mid.A, mid.B, mid.T_AA, mid.T_AB, mid.T_BB, mid.nl, cols)
    Sc = O.overlap_columns(mid.A, mid.B, mid.U, mid.nl, cols)
    rng = np.random.default_rng(2)
    y = cn(rng, (mid.N_G,))
    for j, g in enumerate(cols):
        x = np.zeros(mid.N_G, complex)
        x[g] = 1.0
        h, s = O.bilinear(mid.A, mid.B, mid.T_AA, mid.T_AB, mid.T_BB, mid.U, mid.nl, x, y)
        assert abs(y.conj() @ Hc[:, j] - h) <= 1e-12 * np.linalg.norm(Hc[:, j]) * np.linalg.norm(y)
        assert abs(y.conj() @ Sc[:, j] - s) <= 1e-12 * np.linalg.norm(Sc[:, j]) * np.linalg.norm(y)


# P11: Alg. 1 through SciPy BLAS/LAPACK (a second derivation) equals the oracle.
@pytest.mark.parametrize("case", ["plain_gpu", "mixed"])
def test_algorithm1_equals_definition(case, mid):
    p = mid if case == "plain_gpu" else make_problem(
        8, [4, 9, 16, 25, 4, 9, 16, 25], 300, seed=4, fail_atoms=[1, 6], planted={3: 7})
    H, S, info = O.algorithm1(p.A, p.B, p.T_AA, p.T_AB, p.T_BB, p.U, p.nl)
    assert _rel(H, _H(p)) <= 1e-13
    assert _rel(S, _S(p)) <= 1e-13
    expect = np.zeros(p.N_A, np.int32)
    for a in p.failing:
        expect[a] = 1
    for a, piv in p.planted.items():
        expect[a] = piv
    assert np.array_equal(info, expect)


def test_atom_products_against_algorithm_steps(mid):
    """Z, Y/X from their definitions; their stacked products rebuild H (Alg. 1's zher2k,
    failure-branch zgemm and HPD zherk)."""
    p = mid
    Z, W, info = O.atom_products(p.A, p.B, p.T_AA, p.T_AB, p.T_BB, p.nl)
    assert sorted(np.nonzero(info)[0].tolist()) == p.failing
    rows = np.repeat(info != 0, p.nl)
    P = np.where(rows[:, None], p.A, W)
    H = Z.conj().T @ p.B + p.B.conj().T @ Z + P.conj().T @ W
    assert _rel(H, _H(p)) <= 1e-13


# P12: traces.
def test_traces(mid):
    p = mid
    trS = np.sum(np.abs(p.A) ** 2) + np.sum(np.abs(p.U[:, None] * p.B) ** 2)
    assert abs(np.trace(_S(p)) - trS) <= 1e-13 * trS
    trH = 0j
    r = 0
    for a in range(p.N_A):
        n = int(p.nl[a])
        Aa, Ba = p.A[r:r + n], p.B[r:r + n]
        trH += np.trace(p.t_block("T_AA", a) @ Aa @ Aa.conj().T)
        trH += 2 * np.real(np.trace(p.t_block("T_AB", a) @ Ba @ Aa.conj().T))
        trH += np.trace(p.t_block("T_BB", a) @ Ba @ Ba.conj().T)
        r += n
    assert abs(np.trace(_H(p)) - trH) <= 1e-12 * np.linalg.norm(_H(p))


# P13: the per-atom Cholesky against LAPACK zpotrf, incl. planted failures.
@pytest.mark.parametrize("n,pivot", [(16, 0), (49, 0), (81, 0), (121, 0),
                                     (16, 1), (49, 17), (81, 81), (121, 60)])
def test_cholesky_against_lapack(n, pivot):
    p = make_problem(1, n, 1, seed=n + pivot, planted={0: pivot} if pivot else None)
    T = p.t_block("T_AA", 0)
    C, info = O.cholesky_lower(T)
    c_ref, info_ref = scipy.linalg.lapack.zpotrf(T, lower=1)
    assert info == info_ref == pivot
    if info == 0:
        assert np.allclose(C, np.tril(c_ref), rtol=0, atol=1e-13 * np.abs(c_ref).max())
        assert np.linalg.norm(C @ C.conj().T - T) <= 10 * n * 2.2e-16 * np.linalg.norm(T)
        assert np.all(np.diag(C).real > 0) and np.all(np.diag(C).imag == 0)


def test_cholesky_shift_and_nan():
    p = make_problem(4, 49, 1, seed=2, fail_atoms=[0, 3])
    for a, want in ((0, 1), (1, 0), (2, 0), (3, 1)):
        assert O.cholesky_lower(p.t_block("T_AA", a))[1] == want
    T = p.t_block("T_AA", 1).copy()
    T[5, 5] = np.nan
    assert O.cholesky_lower(T)[1] == 6
    T = p.t_block("T_AA", 1).copy()
    T[9, 2] = np.nan           # a NaN below the diagonal poisons pivot 10
    assert O.cholesky_lower(T)[1] == 10
    # only the lower triangle is read
    T = p.t_block("T_AA", 1).copy()
    T[np.triu_indices(49, 1)] = 1e30
    C, info = O.cholesky_lower(T)
    assert info == 0


# P14: the flop formulas of Alg. 1 reproduce the paper's Tab. 6 rates.
def test_flop_formulas_reproduce_table6():
    from paper_1611_00606_amd.flops import paper_step_flops
    f = paper_step_flops(np.full(512, 49), 9273, np.zeros(512, int))
    want = {"loop1": f["loop1_zgemm_TBA_A"] + f["loop1_zhemm_TBB_B"], "S1": f["S_zherk_A"],
            "S2": f["S_zherk_UB"], "H1": f["H_zher2k_Z_B"]}
    rows = [l.split() for l in open(os.path.join(GOLDEN, "tab6_nacl_kmax4.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 4
    for name, _, sec, gf in rows:
        printed = float(sec) * float(gf) * 1e9
        assert abs(printed / want[name] - 1) < 3e-3, (name, printed, want[name])
