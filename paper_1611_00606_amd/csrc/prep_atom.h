// Per-atom preparation as a block-level device routine, shared by the
// one-block-per-atom launch (k_prep) and the persistent batched launch
// (k_batch).
//
// Cholesky of T^AA_a with failure detection (Alg. 1, the try step of the
// second loop; Sec. 2 explains that T^AA_a is HPD in theory but the
// factorization may fail numerically), and the operand forms used by the
// per-atom products.
//
// The lower triangle of T^AA_a is held packed (row-major lower, element (i,k)
// at i(i+1)/2 + k) in LDS: for N_L = 128 that is 8256 complex values =
// 129 KiB, inside gfx950's 160 KiB of LDS per CU. The factorization
// (chol_packed) is right-looking; a pivot that is not > 0 (NaN included)
// stops it and sets info = j+1, the LAPACK zpotrf convention.
#pragma once

#include "hs_internal.h"
#include "../../include/hs_build.h"

namespace hs {

constexpr int PACKED_MAX = HS_MAX_NL * (HS_MAX_NL + 1) / 2;
// LDS the routine needs: packed triangle, then the diagonal of C (doubles)
constexpr int PREP_LDS_BYTES = PACKED_MAX * 16 + HS_MAX_NL * 8;

__device__ __forceinline__ int pidx(int i, int k) { return i * (i + 1) / 2 + k; }

// Publishes this block's global writes to every other block on the device,
// then sets *flag (a 0 -> 1 ready flag) with release semantics.
__device__ __forceinline__ void publish(int *flag) {
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(flag, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Hermitian n x n block (row-major, element (i,k)) from the lower triangle of
// the stored block t, scaled by s; Im of the diagonal dropped.
template <int NT>
__device__ __forceinline__ void hermitian_from_lower(const double2 *__restrict__ t, int n, double s,
                                                     double2 *__restrict__ m) {
    const int nn = n * n;
    for (int e = threadIdx.x; e < nn; e += NT) {
        const int i = e / n, k = e - (e / n) * n;
        double2 v;
        if (k < i) v = t[(long long)i * n + k];
        else if (k > i) {
            v = t[(long long)k * n + i];
            v.y = -v.y;
        } else {
            v.x = t[(long long)i * n + i].x;
            v.y = 0.0;
        }
        v.x *= s;
        v.y *= s;
        m[e] = v;
    }
}

// Right-looking Cholesky of the packed lower triangle L (n x n, element
// (i,k) at pidx(i,k)) in LDS by one block of NT threads (every thread calls
// it). At step j the pivot d_j = T_jj - sum_{k<j} |C_jk|^2 has already been
// accumulated into the diagonal entry; the column below it is divided by
// sqrt(d_j) and the trailing triangle receives -C_ij conj(C_kj). On return
// the entries below the diagonal hold C, diag[j] = C_jj, and the result is
// 0 or the 1-based index of the first pivot that is not > 0 (NaN included),
// at which the factorization stopped.
template <int NT>
__device__ __forceinline__ int chol_packed(double2 *L, double *diag, int n) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    constexpr int NW = NT / 64;
    int info = 0;
    for (int j = 0; j < n; ++j) {
        const double dj = L[pidx(j, j)].x;
        if (!(dj > 0.0)) {
            info = j + 1;
            break;
        }
        const double cjj = sqrt(dj);
        if (tid == 0) diag[j] = cjj;
        for (int i = j + 1 + tid; i < n; i += NT) {
            double2 v = L[pidx(i, j)];
            v.x /= cjj;
            v.y /= cjj;
            L[pidx(i, j)] = v;
        }
        __syncthreads();
        for (int i = j + 1 + wave; i < n; i += NW) {
            const double2 cij = L[pidx(i, j)];
            for (int k = j + 1 + lane; k <= i; k += 64) {
                const double2 ckj = L[pidx(k, j)];
                double2 t = L[pidx(i, k)];
                // t -= cij * conj(ckj)
                t.x -= cij.x * ckj.x + cij.y * ckj.y;
                t.y -= cij.y * ckj.x - cij.x * ckj.y;
                L[pidx(i, k)] = t;
            }
        }
        __syncthreads();
    }
    return info;
}

// Preparation of atom a by one block of NT threads (every thread calls it):
//   M2_a = 1/2 T_BB,a (Hermitian), d, sel[0..2K) rows of a; then *flag_m2
//   (if not null) is set;
//   Cholesky of T_AA,a: M1_a = C_a (lower, zero above) on success, else
//   T_AA,a (Hermitian); sel[2K + r] = (info != 0); info_out[a] = info; then
//   *flag_m1 (if not null) is set.
// L: LDS of PREP_LDS_BYTES.
template <int NT>
__device__ __forceinline__ void prep_atom(const Atoms &at, int a, const double2 *__restrict__ T_AA,
                                          const double2 *__restrict__ T_BB,
                                          const double2 *__restrict__ U, double2 *__restrict__ M1,
                                          double2 *__restrict__ M2, double *__restrict__ d,
                                          int *__restrict__ sel, int *__restrict__ info_out,
                                          char *lds, int *flag_m2, int *flag_m1) {
    double2 *L = reinterpret_cast<double2 *>(lds);
    double *diag = reinterpret_cast<double *>(lds + PACKED_MAX * 16);

    const int tid = threadIdx.x;

    const int r0 = at.row_off[a];
    const int n = at.row_off[a + 1] - r0;
    const long long t0 = at.t_off[a];
    const double2 *taa = T_AA + t0;
    const int K = at.K;

    hermitian_from_lower<NT>(T_BB + t0, n, 0.5, M2 + t0);
    for (int l = tid; l < n; l += NT) {
        const double2 u = U[r0 + l];
        d[r0 + l] = 1.0;
        d[K + r0 + l] = u.x * u.x + u.y * u.y;
        sel[r0 + l] = 0;
        sel[K + r0 + l] = 0;
    }
    if (flag_m2) publish(flag_m2);

    // lower triangle of T_AA,a into LDS, eight loads in flight per thread
    const int nn = n * n;
    constexpr int BATCH = 8;
    for (int e0 = 0; e0 < nn; e0 += BATCH * NT) {
        double2 v[BATCH];
#pragma unroll
        for (int b = 0; b < BATCH; ++b) {
            const int e = e0 + b * NT + tid;
            v[b] = taa[e < nn ? e : nn - 1];   // clamped: every load in bounds
        }
#pragma unroll
        for (int b = 0; b < BATCH; ++b) {
            const int e = e0 + b * NT + tid;
            if (e < nn) {
                const int i = e / n, k = e - (e / n) * n;
                if (k <= i) L[pidx(i, k)] = v[b];
            }
        }
    }
    __syncthreads();

    const int info = chol_packed<NT>(L, diag, n);

    double2 *m1 = M1 + t0;
    if (info == 0) {
        for (int e = tid; e < nn; e += NT) {
            const int i = e / n, k = e % n;
            double2 v = {0.0, 0.0};
            if (k < i) v = L[pidx(i, k)];
            else if (k == i) v.x = diag[i];
            m1[e] = v;
        }
    } else {
        hermitian_from_lower<NT>(taa, n, 1.0, m1);
    }
    for (int l = tid; l < n; l += NT) sel[2 * K + r0 + l] = info != 0;
    if (tid == 0) info_out[a] = info;
    if (flag_m1) publish(flag_m1);
    // the LDS triangle may be reused by the caller after this barrier
    __syncthreads();
}

}  // namespace hs
