"""Planted mistakes in the oracle must trip at least one independent pin.

Each mutant is a copy of an oracle function with one plausible slip (a lost
conjugate, a dropped term, a transposed operand, an off-by-one). The pins used
are the hand-worked example, the Alg. 1 route through SciPy BLAS/LAPACK and
the closed forms; none of them calls the oracle function under test.
"""

import os

import numpy as np
import pytest

import oracle as O
from hs_inputs import make_problem

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _atoms(nl):
    r = t = 0
    for n in nl:
        n = int(n)
        yield slice(r, r + n), slice(t, t + n * n), n
        r += n
        t += n * n


def _ham_mutant(kind):
    def h(A, B, T_AA, T_AB, T_BB, nl):
        H = np.zeros((A.shape[1],) * 2, complex)
        for rs, ts, n in _atoms(nl):
            Aa, Ba = A[rs], B[rs]
            taa, tab, tbb = (T[ts].reshape(n, n) for T in (T_AA, T_AB, T_BB))
            tba = {"tba_no_herm": tab, "tba_no_conj": tab.T}.get(kind, tab.conj().T)
            if kind == "taa_transposed":
                taa = taa.T
            left = Aa.T if kind == "lost_conj_left" else Aa.conj().T
            H += left @ (taa @ Aa + tab @ Ba)
            H += Ba.conj().T @ (tba @ Aa + (0 if kind == "dropped_tbb" else tbb @ Ba))
            if kind == "ab_swapped":
                H += Ba.conj().T @ tab @ Aa - Aa.conj().T @ tab @ Ba
        return H
    return h


def _ovl_mutant(kind):
    def s(A, B, U, nl):
        S = np.zeros((A.shape[1],) * 2, complex)
        for rs, _, _ in _atoms(nl):
            Aa, Ba, u = A[rs], B[rs], U[rs]
            if kind != "dropped_aha":
                S += Aa.conj().T @ Aa
            w = u if kind == "u_not_squared" else np.abs(u) ** 2
            S += Ba.conj().T @ (w[:, None] * Ba)
        return S
    return s


def _pins_failed(ham, ovl):
    failed = []
    # hand-worked example
    rows = [l.split() for l in open(os.path.join(GOLDEN, "scalar_atom.txt"))
            if l.strip() and not l.startswith("#")]
    A = np.array([[1 + 2j, 3 - 1j]])
    B = np.array([[2 + 0j, -1 + 1j]])
    nl = np.array([1])
    H = ham(A, B, np.array([2 + 0j]), np.array([1 + 1j]), np.array([-1 + 0j]), nl)
    S = ovl(A, B, np.array([2j]), nl)
    for m, gp, g, re, im in rows:
        if {"H": H, "S": S}[m][int(gp) - 1, int(g) - 1] != complex(float(re), float(im)):
            failed.append("hand_worked")
            break
    # second derivation through Alg. 1
    p = make_problem(3, [3, 5, 4], 24, seed=2, fail_atoms=[1])
    H2, S2, _ = O.algorithm1(p.A, p.B, p.T_AA, p.T_AB, p.T_BB, p.U, p.nl)
    if np.linalg.norm(ham(p.A, p.B, p.T_AA, p.T_AB, p.T_BB, p.nl) - H2) > 1e-12 * np.linalg.norm(H2):
        failed.append("algorithm1_H")
    if np.linalg.norm(ovl(p.A, p.B, p.U, p.nl) - S2) > 1e-12 * np.linalg.norm(S2):
        failed.append("algorithm1_S")
    # closed form U = I
    q = p.copy()
    q.U[:] = 1
    ref = q.A.conj().T @ q.A + q.B.conj().T @ q.B
    if np.linalg.norm(ovl(q.A, q.B, q.U, q.nl) - ref) > 1e-12 * np.linalg.norm(ref):
        failed.append("closed_form_S")
    return failed


def test_unmutated_oracle_passes_all_pins():
    assert _pins_failed(O.hamiltonian, O.overlap) == []


@pytest.mark.parametrize("kind", ["tba_no_herm", "tba_no_conj", "taa_transposed",
                                  "lost_conj_left", "dropped_tbb", "ab_swapped"])
def test_hamiltonian_mutant_is_caught(kind):
    assert _pins_failed(_ham_mutant(kind), O.overlap)


@pytest.mark.parametrize("kind", ["dropped_aha", "u_not_squared"])
def test_overlap_mutant_is_caught(kind):
    assert _pins_failed(O.hamiltonian, _ovl_mutant(kind))


def test_cholesky_off_by_one_is_caught():
    """A 0-based failure index disagrees with LAPACK's zpotrf info."""
    import scipy.linalg
    p = make_problem(1, 20, 1, seed=1, planted={0: 9})
    T = p.t_block("T_AA", 0)
    assert O.cholesky_lower(T)[1] == scipy.linalg.lapack.zpotrf(T, lower=1)[1]
    assert O.cholesky_lower(T)[1] - 1 != scipy.linalg.lapack.zpotrf(T, lower=1)[1]
