// Reduction of the generalized eigenproblem H x = lambda S x (Sec. 1.1) to
// standard form, the step after the build:
//     S = L L^H  (L lower, positive real diagonal),   Ht = L^{-1} H L^{-H}.
//
// Blocked in panels of NB = 64 columns/rows, the O(N^3) work on the complex
// FP64 MFMA tile engine (zmfma_tile.h):
//   Cholesky, per panel k (rows/cols kb .. kb+nb):
//     k_gep_chol_diag   factor the diagonal block in LDS (chol_packed)
//     k_gep_trsm (0)    panel rows below: L_ik = S_ik L_kk^{-H}, stored both
//                       in L and, conjugate-transposed, in LH = L^H
//     k_gep_update      trailing lower triangle: S_ij -= L_ik L_jk^H
//   X = L^{-1} H, then Ht = L^{-1} X^H (= L^{-1} H L^{-H} for Hermitian H),
//   each a blocked forward substitution, per panel k:
//     k_gep_trsm (1)    X_k = L_kk^{-1} X_k (rows kb .. kb+nb, all columns)
//     k_gep_update      X_i -= L_ik X_k for the rows below
//   k_gep_conj_t        X^H between the two substitutions
//   mirror              Ht := lower(Ht) + its conjugate transpose (exactly
//                       Hermitian, real diagonal)
// The updates read L's panel columns as rows of LH, which is the
// contraction-by-rows layout the tile engine takes, so no update needs a
// transposed operand.
#include "hs_internal.h"
#include "prep_atom.h"
#include "zmfma_tile.h"

namespace hs {

namespace {

constexpr int GNB = 64;           // panel width
constexpr int GT = 256;           // threads of the small kernels
using GepCfg = TileCfg<128, 128, 16, 2, 4>;

__global__ void k_gep_info_clear(int *info) { *info = 0; }

// L := lower(S) (upper zero), X := H
__global__ void __launch_bounds__(256)
k_gep_init(const double2 *__restrict__ H, const double2 *__restrict__ S, double2 *__restrict__ L,
           double2 *__restrict__ X, int N) {
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= (long long)N * N) return;
    const int i = (int)(e / N), j = (int)(e % N);
    L[e] = j <= i ? S[e] : double2{0.0, 0.0};
    X[e] = H[e];
}

// Cholesky of the diagonal block (rows/cols kb .. kb+nb of L) in place.
__global__ void __launch_bounds__(GT)
k_gep_chol_diag(double2 *__restrict__ L, int N, int kb, int nb, int *__restrict__ info) {
    __shared__ double2 P[GNB * (GNB + 1) / 2];
    __shared__ double diag[GNB];
    const int tid = threadIdx.x;
    for (int e = tid; e < nb * nb; e += GT) {
        const int r = e / nb, c = e % nb;
        if (c <= r) P[pidx(r, c)] = L[(long long)(kb + r) * N + kb + c];
    }
    __syncthreads();
    const int inf = chol_packed<GT>(P, diag, nb);
    for (int e = tid; e < nb * nb; e += GT) {
        const int r = e / nb, c = e % nb;
        if (c < r) L[(long long)(kb + r) * N + kb + c] = P[pidx(r, c)];
        else if (c == r) L[(long long)(kb + r) * N + kb + c] = double2{diag[r], 0.0};
    }
    if (tid == 0 && inf != 0 && *info == 0) *info = kb + inf;
}

// Forward substitution with the diagonal block L_kk on 64 right-hand-side
// columns per block.
//   mode 0 (Cholesky panel): column i = t0 + .. of the RHS is conj(L[i][kb..]),
//          the solution x gives LH[kb + c][i] = x_c and L[i][kb + c] = conj(x_c);
//   mode 1 (substitution): column j of the RHS is X[kb..][j], overwritten.
__global__ void __launch_bounds__(GT)
k_gep_trsm(double2 *__restrict__ L, double2 *__restrict__ LH, double2 *__restrict__ X, int N,
           int kb, int nb, int mode) {
    __shared__ double2 P[GNB * (GNB + 1) / 2];
    __shared__ double2 Y[GNB][GNB];   // [row c][RHS column]
    const int tid = threadIdx.x;
    const int t0 = kb + nb;
    const int base = (mode == 0 ? t0 : 0) + blockIdx.x * GNB;   // first RHS column
    for (int e = tid; e < nb * nb; e += GT) {
        const int r = e / nb, c = e % nb;
        if (c <= r) P[pidx(r, c)] = L[(long long)(kb + r) * N + kb + c];
    }
    if (mode == 0) {
        for (int e = tid; e < GNB * GNB; e += GT) {   // consecutive c per row
            const int col = e / GNB, c = e % GNB;
            const int i = base + col;
            double2 v = {0.0, 0.0};
            if (i < N && c < nb) {
                v = L[(long long)i * N + kb + c];
                v.y = -v.y;
            }
            Y[c][col] = v;
        }
    } else {
        for (int e = tid; e < GNB * GNB; e += GT) {   // consecutive columns per row
            const int c = e / GNB, col = e % GNB;
            const int j = base + col;
            Y[c][col] = (j < N && c < nb) ? X[(long long)(kb + c) * N + j] : double2{0.0, 0.0};
        }
    }
    __syncthreads();
    const int col = tid % GNB, rg = tid / GNB;
    for (int j = 0; j < nb; ++j) {
        if (tid < GNB) {
            const double d = P[pidx(j, j)].x;
            Y[j][col].x /= d;
            Y[j][col].y /= d;
        }
        __syncthreads();
        const double2 xj = Y[j][col];
        for (int r = j + 1 + rg; r < nb; r += GT / GNB) {
            const double2 l = P[pidx(r, j)];
            double2 y = Y[r][col];
            y.x -= l.x * xj.x - l.y * xj.y;
            y.y -= l.x * xj.y + l.y * xj.x;
            Y[r][col] = y;
        }
        __syncthreads();
    }
    if (mode == 0) {
        for (int e = tid; e < GNB * GNB; e += GT) {
            const int c = e / GNB, cl = e % GNB;
            const int i = base + cl;
            if (i < N && c < nb) LH[(long long)(kb + c) * N + i] = Y[c][cl];
        }
        for (int e = tid; e < GNB * GNB; e += GT) {
            const int cl = e / GNB, c = e % GNB;
            const int i = base + cl;
            if (i < N && c < nb) {
                double2 v = Y[c][cl];
                v.y = -v.y;
                L[(long long)i * N + kb + c] = v;
            }
        }
    } else {
        for (int e = tid; e < GNB * GNB; e += GT) {
            const int c = e / GNB, cl = e % GNB;
            const int j = base + cl;
            if (j < N && c < nb) X[(long long)(kb + c) * N + j] = Y[c][cl];
        }
    }
}

// C[i][j] -= sum_{c < nb} conj(P[c][i]) Q[c][j], P = rows kb .. of LH, Q =
// rows kb .. of Qm (LH itself for the Cholesky update, X for a
// substitution; C may be Qm: the rows read and written are disjoint), for
// i >= t0; lower: only t0 <= j <= i (tiles of the trailing lower triangle),
// else the whole rectangle [t0, N) x [0, N).
__global__ void __launch_bounds__(GepCfg::NT)
k_gep_update(const double2 *LH, const double2 *Qm, double2 *C, int N, int kb, int nb, int lower,
             int ntc) {
    using Cfg = GepCfg;
    __shared__ double2 lds[Cfg::LDS_ELEMS];
    const int t0 = kb + nb;
    int ti, tj;
    if (lower) {   // blockIdx.x -> (ti, tj), tj <= ti, row-major lower triangle
        const int t = blockIdx.x;
        int r = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
        while ((r + 1) * (r + 2) / 2 <= t) ++r;
        while (r * (r + 1) / 2 > t) --r;
        ti = r;
        tj = t - r * (r + 1) / 2;
    } else {
        ti = blockIdx.x / ntc;
        tj = blockIdx.x % ntc;
    }
    const int m0 = t0 + ti * Cfg::BM;
    const int n0 = (lower ? t0 : 0) + tj * Cfg::BN;
    if (m0 >= N || n0 >= N) return;

    Segs<1, false, false> t;
    t.nseg = 1;
    t.len = nb;
    t.ldp = N;
    t.ldq = N;
    t.P[0] = LH + (long long)kb * N;
    t.Q[0] = Qm + (long long)kb * N;
    t.palt = nullptr;
    t.sel = nullptr;
    t.qscale = nullptr;
    Acc<Cfg> acc;
    ztile_run<Cfg>(t, m0, N, n0, N, acc, lds);
#pragma unroll
    for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
        for (int j = 0; j < Cfg::TN; ++j) {
            const int g = n0 + acc_col<Cfg>(j);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gp = m0 + acc_row<Cfg>(i, v);
                if (gp < N && g < N && (!lower || g <= gp)) {
                    double2 *o = C + (long long)gp * N + g;
                    double2 r = *o;
                    r.x -= acc.re[i][j][v];
                    r.y -= acc.im[i][j][v];
                    *o = r;
                }
            }
        }
}

// Y = X^H through 32 x 32 LDS tiles
__global__ void __launch_bounds__(256)
k_gep_conj_t(const double2 *__restrict__ X, double2 *__restrict__ Y, int N) {
    __shared__ double2 tile[32][33];
    const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
    const int bx = blockIdx.x, by = blockIdx.y;   // source tile rows by, cols bx
    for (int r = ty; r < 32; r += 8) {
        const int gr = by * 32 + r, gc = bx * 32 + tx;
        if (gr < N && gc < N) tile[r][tx] = X[(long long)gr * N + gc];
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int gr = bx * 32 + r, gc = by * 32 + tx;   // destination (gr, gc) = conj(X[gc][gr])
        if (gr < N && gc < N) {
            double2 v = tile[tx][r];
            v.y = -v.y;
            Y[(long long)gr * N + gc] = v;
        }
    }
}

hipError_t forward_substitution(double2 *L, double2 *LH, double2 *X, int N, hipStream_t st) {
    using Cfg = GepCfg;
    for (int kb = 0; kb < N; kb += GNB) {
        const int nb = N - kb < GNB ? N - kb : GNB;
        hipLaunchKernelGGL(k_gep_trsm, dim3((N + GNB - 1) / GNB), dim3(GT), 0, st, L, LH, X, N, kb,
                           nb, 1);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        const int t0 = kb + nb;
        if (t0 >= N) continue;
        const int ntr = (N - t0 + Cfg::BM - 1) / Cfg::BM, ntc = (N + Cfg::BN - 1) / Cfg::BN;
        hipLaunchKernelGGL(k_gep_update, dim3(ntr * ntc), dim3(Cfg::NT), 0, st, LH, X, X, N, kb, nb,
                           0, ntc);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

size_t gep_workspace_bytes(int N) {
    const size_t m = 16 * (size_t)N * (size_t)N;
    return 2 * ((m + 255) / 256 * 256) + 256;   // LH, X, info slot
}

hipError_t launch_gep(const double2 *H, const double2 *S, int N, double2 *L, double2 *Ht,
                      int *info, char *ws, hipStream_t st) {
    using Cfg = GepCfg;
    const size_t m = (16 * (size_t)N * (size_t)N + 255) / 256 * 256;
    double2 *LH = reinterpret_cast<double2 *>(ws);
    double2 *X = reinterpret_cast<double2 *>(ws + m);
    if (!info) info = reinterpret_cast<int *>(ws + 2 * m);
    const long long nn = (long long)N * N;
    hipLaunchKernelGGL(k_gep_init, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, st, H, S, L,
                       X, N);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gep_info_clear, dim3(1), dim3(1), 0, st, info);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    for (int kb = 0; kb < N; kb += GNB) {
        const int nb = N - kb < GNB ? N - kb : GNB;
        hipLaunchKernelGGL(k_gep_chol_diag, dim3(1), dim3(GT), 0, st, L, N, kb, nb, info);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        const int t0 = kb + nb;
        if (t0 >= N) continue;
        hipLaunchKernelGGL(k_gep_trsm, dim3((N - t0 + GNB - 1) / GNB), dim3(GT), 0, st, L, LH, X,
                           N, kb, nb, 0);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        const int nt = (N - t0 + Cfg::BM - 1) / Cfg::BM;
        hipLaunchKernelGGL(k_gep_update, dim3(nt * (nt + 1) / 2), dim3(Cfg::NT), 0, st, LH, LH, L,
                           N, kb, nb, 1, 0);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if ((e = forward_substitution(L, LH, X, N, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_gep_conj_t, dim3((N + 31) / 32, (N + 31) / 32), dim3(256), 0, st, X, Ht,
                       N);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = forward_substitution(L, LH, Ht, N, st)) != hipSuccess) return e;
    return launch_mirror1(Ht, N, st);
}

}  // namespace hs
