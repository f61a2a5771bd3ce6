"""CPU oracle for the FLAPW Hamiltonian/overlap build.

TEST INFRASTRUCTURE ONLY. Nothing on the product path may import, call or
link this module: only the tests, the smoke check and the benchmark's CPU
baseline leg use it. It shares no code with the HIP path.

Everything is plain NumPy complex128 (IEEE binary64), written to be checked by
eye against the paper:

  * `overlap`, `hamiltonian`: the matrix forms of Sec. 2 (the equations for H
    and S), summed atom by atom with plain products. T^[BA] is not an input:
    it is T^[AB]^H, as Sec. 2 notes when it rewrites H_{AB+BA+BB}.
  * `overlap_entrywise`, `hamiltonian_entrywise`: the index forms of Sec. 1.1
    (the equations for (S)_{G',G} and (H)_{G',G}) as literal loops, for tiny
    inputs only.
  * `overlap_columns`, `hamiltonian_columns`: the same matrix forms restricted
    to chosen columns G, for spot checks of large outputs.
  * `bilinear`: y^H H x and y^H S x through per-atom vectors, O(K N_G) per
    probe.
  * `cholesky_lower`: the Cholesky factor T = C C^H (C lower, positive
    diagonal) that Alg. 1 attempts per atom, with LAPACK-style failure info:
    the 1-based index of the first pivot that is not positive (or NaN).
  * `atom_products`: the per-atom operands of Alg. 1 (Z_a of its first loop,
    Y_a / X_a of its second loop), each from its plain definition.

Readings taken where the paper is silent:
  * the Cholesky factor is lower with T = C C^H (the "C_a C_a" of Sec. 2 has
    lost a conjugate-transpose; Alg. 1 then forms Y_a = C_a^H A_a);
  * a factorization fails at the first pivot d_j <= 0 or NaN, no tolerance;
  * U_a is the diagonal of U_a, one complex value per row of A_a; only |u|^2
    enters S;
  * the oracle returns the full dense matrices (no symmetrisation).

Data layout (the ABI layout, see hs_inputs): A, B [K, N_G] with atoms stacked
along rows; T_* packed per-atom N_L x N_L blocks; U [K]; nl [N_A].
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "overlap",
    "hamiltonian",
    "overlap_entrywise",
    "hamiltonian_entrywise",
    "overlap_columns",
    "hamiltonian_columns",
    "bilinear",
    "cholesky_lower",
    "atom_products",
]


def _atoms(nl):
    """Yield (a, row slice, T block slice, N_L) for every atom."""
    r0 = 0
    t0 = 0
    for a, n in enumerate(np.asarray(nl, dtype=np.int64)):
        n = int(n)
        yield a, slice(r0, r0 + n), slice(t0, t0 + n * n), n
        r0 += n
        t0 += n * n


def _blk(T, ts, n):
    return T[ts].reshape(n, n)


# --------------------------------------------------------------------------
# Matrix forms (Sec. 2, equations for H and S)
# --------------------------------------------------------------------------

def overlap(A, B, U, nl):
    """S = sum_a A_a^H A_a + B_a^H U_a^H U_a B_a  (Sec. 2, equation for S)."""
    n_g = A.shape[1]
    S = np.zeros((n_g, n_g), dtype=np.complex128)
    for _, rs, _, _ in _atoms(nl):
        Aa = A[rs]
        UBa = U[rs][:, None] * B[rs]          # U_a B_a with U_a diagonal
        S += Aa.conj().T @ Aa
        S += UBa.conj().T @ UBa
    return S


def hamiltonian(A, B, T_AA, T_AB, T_BB, nl):
    """H = sum_a A_a^H T^AA A_a + A_a^H T^AB B_a + B_a^H T^BA A_a + B_a^H T^BB B_a.

    Sec. 2, equation for H, with T^BA := T^AB^H (Sec. 2). Evaluated per atom
    as A_a^H (T^AA A_a + T^AB B_a) + B_a^H (T^BA A_a + T^BB B_a), which is the
    same four terms grouped by their left factor.
    """
    n_g = A.shape[1]
    H = np.zeros((n_g, n_g), dtype=np.complex128)
    for _, rs, ts, n in _atoms(nl):
        Aa, Ba = A[rs], B[rs]
        taa, tab, tbb = _blk(T_AA, ts, n), _blk(T_AB, ts, n), _blk(T_BB, ts, n)
        tba = tab.conj().T
        H += Aa.conj().T @ (taa @ Aa + tab @ Ba)
        H += Ba.conj().T @ (tba @ Aa + tbb @ Ba)
    return H


def overlap_columns(A, B, U, nl, cols):
    """Columns `cols` of S: S[:, g] for g in cols, from the equation for S."""
    cols = np.asarray(cols)
    out = np.zeros((A.shape[1], cols.size), dtype=np.complex128)
    for _, rs, _, _ in _atoms(nl):
        Aa, Ba, u = A[rs], B[rs], U[rs]
        out += Aa.conj().T @ Aa[:, cols]
        out += (u[:, None] * Ba).conj().T @ (u[:, None] * Ba[:, cols])
    return out


def hamiltonian_columns(A, B, T_AA, T_AB, T_BB, nl, cols):
    """Columns `cols` of H: H[:, g] for g in cols, from the equation for H."""
    cols = np.asarray(cols)
    out = np.zeros((A.shape[1], cols.size), dtype=np.complex128)
    for _, rs, ts, n in _atoms(nl):
        Aa, Ba = A[rs], B[rs]
        taa, tab, tbb = _blk(T_AA, ts, n), _blk(T_AB, ts, n), _blk(T_BB, ts, n)
        tba = tab.conj().T
        ac, bc = Aa[:, cols], Ba[:, cols]
        out += Aa.conj().T @ (taa @ ac + tab @ bc)
        out += Ba.conj().T @ (tba @ ac + tbb @ bc)
    return out


def bilinear(A, B, T_AA, T_AB, T_BB, U, nl, x, y):
    """(y^H H x, y^H S x) without forming H or S.

    y^H H x = sum_a (A_a y)^H T^AA (A_a x) + (A_a y)^H T^AB (B_a x)
            + (B_a y)^H T^BA (A_a x) + (B_a y)^H T^BB (B_a x)
    y^H S x = sum_a (A_a y)^H (A_a x) + (U_a B_a y)^H (U_a B_a x)
    """
    h = 0j
    s = 0j
    for _, rs, ts, n in _atoms(nl):
        Aa, Ba, u = A[rs], B[rs], U[rs]
        taa, tab, tbb = _blk(T_AA, ts, n), _blk(T_AB, ts, n), _blk(T_BB, ts, n)
        ax, ay, bx, by = Aa @ x, Aa @ y, Ba @ x, Ba @ y
        h += np.vdot(ay, taa @ ax) + np.vdot(ay, tab @ bx)
        h += np.vdot(by, tab.conj().T @ ax) + np.vdot(by, tbb @ bx)
        s += np.vdot(ay, ax) + np.vdot(u * by, u * bx)
    return h, s


# --------------------------------------------------------------------------
# Index forms (Sec. 1.1), literal loops: tiny inputs only
# --------------------------------------------------------------------------

def overlap_entrywise(A, B, U, nl):
    """(S)_{G',G} = sum_a sum_{lm} conj(A^{a,G'}_{lm}) A^{a,G}_{lm}
                                  + conj(B^{a,G'}_{lm}) B^{a,G}_{lm} ||u_l^a||^2."""
    n_g = A.shape[1]
    S = np.zeros((n_g, n_g), dtype=np.complex128)
    for gp in range(n_g):
        for g in range(n_g):
            acc = 0j
            for _, rs, _, n in _atoms(nl):
                for L in range(rs.start, rs.stop):
                    w = abs(U[L]) ** 2
                    acc += np.conj(A[L, gp]) * A[L, g] + np.conj(B[L, gp]) * B[L, g] * w
            S[gp, g] = acc
    return S


def hamiltonian_entrywise(A, B, T_AA, T_AB, T_BB, nl):
    """(H)_{G',G} = sum_a sum_{L',L} sum_{X,Y in {A,B}} conj(X^{a,G'}_{L'}) T^{[XY]}_{L',L;a} Y^{a,G}_L."""
    n_g = A.shape[1]
    H = np.zeros((n_g, n_g), dtype=np.complex128)
    for _, rs, ts, n in _atoms(nl):
        T = {
            ("A", "A"): _blk(T_AA, ts, n),
            ("A", "B"): _blk(T_AB, ts, n),
            ("B", "A"): _blk(T_AB, ts, n).conj().T,
            ("B", "B"): _blk(T_BB, ts, n),
        }
        C = {"A": A[rs], "B": B[rs]}
        for gp in range(n_g):
            for g in range(n_g):
                acc = 0j
                for (x, y), t in T.items():
                    for lp in range(n):
                        for l in range(n):
                            acc += np.conj(C[x][lp, gp]) * t[lp, l] * C[y][l, g]
                H[gp, g] += acc
    return H


# --------------------------------------------------------------------------
# Per-atom steps of Alg. 1
# --------------------------------------------------------------------------

def cholesky_lower(T):
    """Cholesky T = C C^H, C lower with positive real diagonal (Alg. 1, its try step).

    Reads only the lower triangle of T. Returns (C, info): info = 0 on
    success, else the 1-based index j of the first pivot
    d_j = T_jj - sum_{k<j} |C_jk|^2 that is not > 0 (NaN included); C is then
    valid only in its first j-1 columns.
    """
    T = np.asarray(T, dtype=np.complex128)
    n = T.shape[0]
    C = np.zeros_like(T)
    for j in range(n):                       # column by column (left-looking)
        cj = C[j, :j]
        d = T[j, j].real - float(np.sum(cj.real ** 2 + cj.imag ** 2))
        if not d > 0.0:
            return C, j + 1
        cjj = np.sqrt(d)
        C[j, j] = cjj
        # C_ij = (T_ij - sum_{k<j} C_ik conj(C_jk)) / C_jj   for all i > j
        C[j + 1:, j] = (T[j + 1:, j] - C[j + 1:, :j] @ np.conj(cj)) / cjj
    return C, 0


def atom_products(A, B, T_AA, T_AB, T_BB, nl, info=None):
    """The per-atom operands of Alg. 1, stacked like A.

    Z_a = T^BA_a A_a + 1/2 T^BB_a B_a                      (first loop)
    Y_a = C_a^H A_a           if T^AA_a has a Cholesky factor (second loop)
    X_a = T^AA_a A_a          otherwise
    Returns (Z, W, info) where W holds Y_a or X_a in atom a's rows and info is
    the per-atom failure index (computed with cholesky_lower unless given).
    """
    Z = np.zeros_like(A)
    W = np.zeros_like(A)
    infos = []
    for a, rs, ts, n in _atoms(nl):
        Aa, Ba = A[rs], B[rs]
        taa, tab, tbb = _blk(T_AA, ts, n), _blk(T_AB, ts, n), _blk(T_BB, ts, n)
        Z[rs] = tab.conj().T @ Aa + 0.5 * (tbb @ Ba)
        if info is None:
            C, inf = cholesky_lower(taa)
        else:
            inf = int(info[a])
            C = cholesky_lower(taa)[0] if inf == 0 else None
        infos.append(inf)
        if inf == 0:
            W[rs] = C.conj().T @ Aa
        else:
            W[rs] = taa @ Aa
    return Z, W, np.asarray(infos, dtype=np.int32)
