"""Pins of the generalized-eigenproblem oracle (oracle/gep.py), CPU only.

Each pin fixes the oracle against something other than itself: the
eigenvalues of the generalized problem from LAPACK's zhegv route
(scipy.linalg.eigh(H, S)), NumPy's own Cholesky, closed forms for S = I and
S = c^2 I, and a planted non-positive pivot.
"""

import numpy as np
import scipy.linalg as sl

import oracle as O
from hs_inputs import make_problem


def _hs(n_atoms=6, nl=16, n_g=120, seed=3):
    p = make_problem(n_atoms, nl, n_g, seed=seed)
    H = O.hamiltonian(p.A, p.B, p.T_AA, p.T_AB, p.T_BB, p.nl)
    S = O.overlap(p.A, p.B, p.U, p.nl)
    return H, S


def test_factor_reproduces_S_and_matches_numpy():
    H, S = _hs()
    L, info = O.cholesky_full(S)
    assert info == 0
    assert np.allclose(np.triu(L, 1), 0)
    assert np.all(np.diag(L).real > 0) and np.all(np.diag(L).imag == 0)
    assert np.linalg.norm(L @ L.conj().T - S) <= 1e-14 * np.linalg.norm(S) * 10
    Ln = np.linalg.cholesky(S)
    assert np.linalg.norm(L - Ln) <= 1e-12 * np.linalg.norm(Ln)


def test_reduced_eigenvalues_are_the_generalized_ones():
    H, S = _hs()
    L, Ht, info = O.gep_reduce(H, S)
    assert info == 0
    assert np.linalg.norm(Ht - Ht.conj().T) <= 1e-12 * np.linalg.norm(Ht)
    lam = np.linalg.eigvalsh(0.5 * (Ht + Ht.conj().T))
    ref = sl.eigh(H, S, eigvals_only=True)
    assert np.max(np.abs(lam - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_closed_forms():
    H, _ = _hs(n_g=40)
    n = H.shape[0]
    # Ht = L^{-1} (L^{-1} H)^H = H^H for L = I (H itself is Hermitian only
    # up to the rounding of its own sums)
    L, Ht, info = O.gep_reduce(H, np.eye(n))
    assert info == 0 and np.array_equal(L, np.eye(n)) and np.array_equal(Ht, H.conj().T)
    c = 4.0
    L, Ht, info = O.gep_reduce(H, c * c * np.eye(n))
    assert np.array_equal(L, c * np.eye(n)) and np.array_equal(Ht, H.conj().T / (c * c))


def test_planted_pivot():
    H, S = _hs(n_g=50)
    # make the leading 7x7 minor singular-negative: S_77 below the Schur value
    L, _ = O.cholesky_full(S)
    S2 = S.copy()
    d7 = S[6, 6].real - np.sum(np.abs(L[6, :6]) ** 2)
    S2[6, 6] -= 2 * d7
    _, Ht, info = O.gep_reduce(H, S2)
    assert info == 7 and Ht is None
