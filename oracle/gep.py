"""CPU oracle of the reduction of the generalized eigenproblem to standard form.

TEST INFRASTRUCTURE ONLY (see the package header). Shares no code with the
HIP path.

Sec. 1.1: the Kohn-Sham equations become, per k-point, the generalized
eigenvalue problem  sum_G' [H_{G,G'} - lambda S_{G,G'}] c_G' = 0  with S
Hermitian and generically positive definite (up to a few very small singular
values). The standard reduction, the step that follows the build, is

    S = L L^H          (Cholesky, L lower with a positive real diagonal)
    Ht = L^{-1} H L^{-H}

so that H x = lambda S x  <=>  Ht y = lambda y with y = L^H x.

  * `cholesky_full`: the column (Crout) recurrence of the factor, with the
    LAPACK-style 1-based index of the first pivot that is not positive;
  * `gep_reduce`: L and Ht through plain forward substitutions
    (L^{-1} H, then L^{-1} (L^{-1} H)^H, which equals L^{-1} H L^{-H} for a
    Hermitian H).
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sl

from .hs_oracle import cholesky_lower

__all__ = ["cholesky_full", "gep_reduce"]


def cholesky_full(S):
    """(L, info) with S = L L^H from S's lower triangle; info 0 or the first
    failing pivot (1-based), L then holds the columns before it."""
    return cholesky_lower(np.asarray(S, dtype=np.complex128))


def gep_reduce(H, S):
    """(L, Ht, info): Cholesky factor of S and L^{-1} H L^{-H} (Ht is None
    when S is not positive definite)."""
    L, info = cholesky_full(S)
    if info != 0:
        return L, None, info
    X = sl.solve_triangular(L, np.asarray(H, dtype=np.complex128), lower=True)
    Ht = sl.solve_triangular(L, X.conj().T, lower=True)
    return L, Ht, 0
