"""Alg. 1 of the paper on the host, through SciPy's BLAS/LAPACK.

TEST INFRASTRUCTURE ONLY (same rules as hs_oracle): used to pin the direct
oracle with a second, independent derivation of H and S, and as the
"CPU only" reference method the paper's tables compare against.

Follows Alg. 1 step by step, with the library routine the paper names for
each step:
  first loop   Z_a = T^BA_a A_a (zgemm) ; Z_a += 1/2 T^BB_a B_a (zhemm)
               H = Z^H B + B^H Z (zher2k)
  S            S = A^H A (zherk) ; B' = U B (scaling) ; S += B'^H B' (zherk)
  second loop  C_a = Cholesky(T^AA_a) (zpotrf)
               success: Y_a = C_a^H A_a (ztrmm), stacked into Y_HPD
               failure: X_a = T^AA_a A_a (zhemm), stacked into X_notHPD,
                        A_a stacked into A_notHPD
               H += A_notHPD^H X_notHPD (zgemm) ; H += Y_HPD^H Y_HPD (zherk)
The Hermitian routines fill the lower triangle; the result is completed by
conjugate mirroring. Inputs are not modified (the paper's backup/restore of
A and B is therefore unnecessary).
"""

from __future__ import annotations

import numpy as np
from scipy.linalg import blas, lapack


def _mirror_lower(C):
    """Full Hermitian matrix from its lower triangle (diagonal imaginary part 0)."""
    L = np.tril(C, -1)
    out = L + L.conj().T
    out[np.diag_indices(C.shape[0])] = C.diagonal().real
    return out


def algorithm1(A, B, T_AA, T_AB, T_BB, U, nl):
    """Returns (H, S, info) computed by the steps of Alg. 1."""
    nl = np.asarray(nl, dtype=np.int64)
    rows = np.concatenate([[0], np.cumsum(nl)])
    toff = np.concatenate([[0], np.cumsum(nl * nl)])
    n_g = A.shape[1]

    def blk(T, a):
        n = int(nl[a])
        return np.asfortranarray(T[toff[a]:toff[a + 1]].reshape(n, n))

    # First part of H
    Z = np.empty_like(A)
    for a in range(len(nl)):
        rs = slice(rows[a], rows[a + 1])
        Aa, Ba = np.asfortranarray(A[rs]), np.asfortranarray(B[rs])
        tba = np.asfortranarray(blk(T_AB, a).conj().T)
        za = blas.zgemm(1.0, tba, Aa)
        za = blas.zhemm(0.5, blk(T_BB, a), Ba, beta=1.0, c=za, side=0, lower=1)
        Z[rs] = za
    H = blas.zher2k(1.0, np.asfortranarray(Z), np.asfortranarray(B), trans=2, lower=1)

    # S
    S = blas.zherk(1.0, np.asfortranarray(A), trans=2, lower=1)
    Bu = U[:, None] * B
    S = blas.zherk(1.0, np.asfortranarray(Bu), beta=1.0, c=S, trans=2, lower=1)

    # Second part of H
    info = np.zeros(len(nl), dtype=np.int32)
    Y, X, An = [], [], []
    for a in range(len(nl)):
        rs = slice(rows[a], rows[a + 1])
        Aa = np.asfortranarray(A[rs])
        taa = blk(T_AA, a)
        c, inf = lapack.zpotrf(taa, lower=1)
        info[a] = inf
        if inf == 0:
            Y.append(blas.ztrmm(1.0, c, Aa, side=0, lower=1, trans_a=2, diag=0))
        else:
            X.append(blas.zhemm(1.0, taa, Aa, side=0, lower=1))
            An.append(Aa)
    if X:
        Xs = np.asfortranarray(np.concatenate(X))
        As = np.asfortranarray(np.concatenate(An))
        H = H + np.tril(blas.zgemm(1.0, As, Xs, trans_a=2))
    if Y:
        Ys = np.asfortranarray(np.concatenate(Y))
        H = blas.zherk(1.0, Ys, beta=1.0, c=np.asfortranarray(H), trans=2, lower=1)

    assert H.shape == (n_g, n_g)
    return _mirror_lower(H), _mirror_lower(S), info
