"""H and S through the factored identities of Sec. 2, on the host with SciPy's
BLAS/LAPACK.

TEST INFRASTRUCTURE ONLY (same rules as hs_oracle): a second derivation of H
and S that pins the direct oracle, and the host-side analogue of the paper's
CPU-only method (its Alg. 1 reaches H and S through the same identities).

Derivation, one output term at a time (Sec. 2):
  * S is the Gram matrix of the rows of all atoms' A_a and U_a B_a stacked
    into one matrix G: S = G^H G, a single Hermitian rank-k update.
  * The cross and B-B terms of H, A^H T^AB B + B^H T^BA A + B^H T^BB B with
    T^BA = (T^AB)^H, equal Z^H B + B^H Z for Z = T^BA A + 1/2 T^BB B (atom by
    atom), a single Hermitian rank-2k update over the stacked rows.
  * The A-A term A_a^H T^AA_a A_a: where T^AA_a = C_a C_a^H has a Cholesky
    factor (lower C_a), it is (C_a^H A_a)^H (C_a^H A_a), a Hermitian rank-k
    update of the triangular products; where it has none (the failure case
    the paper describes), the general product A_a^H (T^AA_a A_a).
Only lower triangles are accumulated; the result is mirrored at the end.
Inputs are not modified.
"""

from __future__ import annotations

import numpy as np
from scipy.linalg import blas, lapack


def _hermitian_from_lower(C):
    """Full Hermitian matrix from its lower triangle (diagonal imaginary part 0)."""
    L = np.tril(C, -1)
    out = L + L.conj().T
    out[np.diag_indices(C.shape[0])] = C.diagonal().real
    return out


def _hermitian_block(t):
    """The Hermitian matrix a zhemm/zpotrf reader sees in t: its lower
    triangle, mirrored, with the diagonal's imaginary part dropped."""
    full = np.tril(t) + np.tril(t, -1).conj().T
    full[np.diag_indices(t.shape[0])] = t.diagonal().real
    return full


def _atom_slices(nl):
    nl = np.asarray(nl, dtype=np.int64)
    rows = np.concatenate([[0], np.cumsum(nl)])
    toff = np.concatenate([[0], np.cumsum(nl * nl)])
    for a, n in enumerate(nl):
        yield a, slice(rows[a], rows[a + 1]), slice(toff[a], toff[a + 1]), int(n)


def _gram_lower(G, C=None):
    """lower(C + G^H G) by zherk (C None: zero)."""
    G = np.asfortranarray(G)
    if C is None:
        return blas.zherk(1.0, G, trans=2, lower=1)
    return blas.zherk(1.0, G, beta=1.0, c=np.asfortranarray(C), trans=2, lower=1)


def overlap_factored(A, B, U, nl):
    """S = G^H G with G = [A; U B] (rows of every atom stacked)."""
    G = np.concatenate([A, U[:, None] * B])
    return _hermitian_from_lower(_gram_lower(G))


def hamiltonian_factored(A, B, T_AA, T_AB, T_BB, nl):
    """H by its factored terms; returns (H, info) with info[a] the Cholesky
    status of T^AA_a (0, or LAPACK's first failing pivot)."""
    n_g = A.shape[1]
    n_atoms = len(nl)
    # cross and B-B terms: Z^H B + B^H Z, Z = T^BA A + 1/2 T^BB B per atom
    Z = np.empty_like(A)
    for _, rs, ts, n in _atom_slices(nl):
        t_ba = T_AB[ts].reshape(n, n).conj().T
        t_bb = T_BB[ts].reshape(n, n)
        Z[rs] = t_ba @ A[rs] + 0.5 * (_hermitian_block(t_bb) @ B[rs])
    H = blas.zher2k(1.0, np.asfortranarray(Z), np.asfortranarray(B), trans=2, lower=1)
    # A-A term: triangular factors where they exist, general products elsewhere
    info = np.zeros(n_atoms, dtype=np.int32)
    factored, unfactored = [], None
    for a, rs, ts, n in _atom_slices(nl):
        t_aa = np.asfortranarray(T_AA[ts].reshape(n, n))
        c, info[a] = lapack.zpotrf(t_aa, lower=1)
        Aa = np.asfortranarray(A[rs])
        if info[a] == 0:
            factored.append(blas.ztrmm(1.0, c, Aa, side=0, lower=1, trans_a=2))
        else:
            term = Aa.conj().T @ (_hermitian_block(t_aa) @ Aa)
            unfactored = term if unfactored is None else unfactored + term
    if factored:
        H = _gram_lower(np.concatenate(factored), H)
    if unfactored is not None:
        H = H + np.tril(unfactored)
    assert H.shape == (n_g, n_g)
    return _hermitian_from_lower(H), info


def algorithm1(A, B, T_AA, T_AB, T_BB, U, nl):
    """(H, S, info) through the factored identities (see the module docstring)."""
    H, info = hamiltonian_factored(A, B, T_AA, T_AB, T_BB, nl)
    return H, overlap_factored(A, B, U, nl), info
