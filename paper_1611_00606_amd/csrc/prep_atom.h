// Per-atom preparation as a block-level device routine, shared by the
// one-block-per-atom launch (k_prep) and the persistent batched launch
// (k_batch).
//
// Cholesky of T^AA_a with failure detection (Alg. 1, the try step of the
// second loop; Sec. 2 explains that T^AA_a is HPD in theory but the
// factorization may fail numerically), and the operand forms used by the
// per-atom products.
//
// The lower triangle of T^AA_a is spread over the block's registers (entry
// e = i(i+1)/2 + k of the packed triangle, k <= i, in slot e / NT of thread
// e % NT; for N_L = 128, 17 entries per thread of a 512-thread block); only
// the current column passes through LDS. The factorization (chol_atom) is
// right-looking with one barrier per column; a pivot that is not > 0 (NaN
// included) stops it and sets info = j+1, the LAPACK zpotrf convention.
#pragma once

#include "hs_internal.h"
#include "../../include/hs_build.h"

namespace hs {

constexpr int PACKED_MAX = HS_MAX_NL * (HS_MAX_NL + 1) / 2;
// LDS the routine needs: two column buffers of HS_MAX_NL complex values
constexpr int PREP_LDS_BYTES = 2 * HS_MAX_NL * 16;

// Publishes this block's global writes to every other block on the device,
// then sets *flag (a ready flag, 0 until then) to value (nonzero) with
// release semantics.
__device__ __forceinline__ void publish(int *flag, int value) {
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(flag, value, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
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

// Right-looking Cholesky of the n x n Hermitian block t (row-major; its lower
// triangle is read) by one block of NT threads (every thread calls it), the
// triangle held in registers as described above. Before step j every entry
// (i, k), k >= j, holds L_ik = t_ik - sum_{m<j} C_im conj(C_km), and column j
// (rows i >= j) is also in the LDS buffer col[j & 1]. Step j tests the pivot
// L_jj, turns column j into C_ij = L_ij / sqrt(L_jj), subtracts
// C_ij conj(C_kj) from every entry (i, k) with k > j, and writes the updated
// column j + 1 into col[(j + 1) & 1] for the next step. Returns 0, having
// written C to m (lower triangle and real diagonal, zero above), or the
// 1-based index of the first pivot that is not > 0 (NaN included), at which
// the factorization stopped, leaving m unwritten.
template <int NT>
__device__ __forceinline__ int chol_atom(const double2 *__restrict__ t, int n, double2 *col,
                                         double2 *__restrict__ m) {
    constexpr int NS = (PACKED_MAX + NT - 1) / NT;
    int tid = threadIdx.x;
    // opaque to the compiler, so that the slot decoding below is not hoisted
    // out of a caller's loop (where it would hold registers throughout)
    asm volatile("" : "+v"(tid));
    const int ntri = n * (n + 1) / 2;
    double2 v[NS];
    int ik[NS];   // i << 8 | k of each slot's entry, -1 for none
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int e = s * NT + tid;
        int i = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
        if (i * (i + 1) / 2 > e) --i;
        if ((i + 1) * (i + 2) / 2 <= e) ++i;
        ik[s] = e < ntri ? i << 8 | (e - i * (i + 1) / 2) : -1;
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int i = ik[s] >> 8, k = ik[s] & 255;
        v[s] = ik[s] < 0 ? double2{0.0, 0.0} : t[i * n + k];
        if (ik[s] >= 0 && k == 0) col[i] = v[s];
    }
    __syncthreads();
    for (int j = 0; j < n; ++j) {
        const double2 *cj = col + (j & 1) * HS_MAX_NL;
        double2 *cn = col + ((j + 1) & 1) * HS_MAX_NL;
        const double ljj = cj[j].x;
        if (!(ljj > 0.0)) return j + 1;   // the same value in every thread
        const double rs = 1.0 / sqrt(ljj);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            // decoded anew each step rather than kept decoded in registers
            asm volatile("" : "+v"(ik[s]));
            const int i = ik[s] >> 8, k = ik[s] & 255;
            if (ik[s] < 0 || k < j) continue;
            if (k == j) {
                v[s].x *= rs;
                v[s].y *= rs;
            } else {
                const double2 a = cj[i], b = cj[k];
                const double ax = a.x * rs, ay = a.y * rs, bx = b.x * rs, by = b.y * rs;
                // v -= C_ij conj(C_kj)
                v[s].x -= ax * bx + ay * by;
                v[s].y -= ay * bx - ax * by;
                if (k == j + 1) cn[i] = v[s];
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        if (ik[s] < 0) continue;
        const int i = ik[s] >> 8, k = ik[s] & 255;
        m[i * n + k] = k == i ? double2{v[s].x, 0.0} : v[s];
    }
    for (int e = tid; e < n * n; e += NT)
        if (e % n > e / n) m[e] = double2{0.0, 0.0};
    return 0;
}

// Preparation of atom a by one block of NT threads (every thread calls it):
//   M2_a = 1/2 T_BB,a (Hermitian), d, sel[0..2K) rows of a; then *flag_m2
//   (if not null) is set to 1;
//   Cholesky of T_AA,a: M1_a = C_a (lower, zero above) on success, else
//   T_AA,a (Hermitian); sel[2K + r] = (info != 0); info_out[a] = info; then
//   *flag_m1 (if not null) is set to 1 on success, 2 on failure.
// lds: PREP_LDS_BYTES of LDS.
template <int NT>
__device__ __forceinline__ void prep_atom(const Atoms &at, int a, const double2 *__restrict__ T_AA,
                                          const double2 *__restrict__ T_BB,
                                          const double2 *__restrict__ U, double2 *__restrict__ M1,
                                          double2 *__restrict__ M2, double *__restrict__ d,
                                          int *__restrict__ sel, int *__restrict__ info_out,
                                          char *lds, int *flag_m2, int *flag_m1) {
    double2 *col = reinterpret_cast<double2 *>(lds);

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
    if (flag_m2) publish(flag_m2, 1);

    double2 *m1 = M1 + t0;
    const int info = chol_atom<NT>(taa, n, col, m1);
    if (info != 0) hermitian_from_lower<NT>(taa, n, 1.0, m1);
    for (int l = tid; l < n; l += NT) sel[2 * K + r0 + l] = info != 0;
    if (tid == 0) info_out[a] = info;
    if (flag_m1) publish(flag_m1, info != 0 ? 2 : 1);
    // the LDS column buffers may be reused by the caller after this barrier
    __syncthreads();
}

}  // namespace hs
