// Per-atom preparation: Cholesky of T^AA_a with failure detection (Alg. 1,
// the try step of the second loop; Sec. 2 explains that T^AA_a is HPD in
// theory but the factorization may fail numerically), and the operand forms
// used by the per-atom products.
//
// One 256-thread block per atom. The lower triangle of T^AA_a is held packed
// (row-major lower, element (i,k) at i(i+1)/2 + k) in LDS: for N_L = 128 that
// is 8256 complex values = 129 KiB, inside gfx950's 160 KiB of LDS per CU.
// The factorization is right-looking: at step j the pivot
// d_j = T_jj - sum_{k<j} |C_jk|^2 has already been accumulated into the
// diagonal entry, the column below it is divided by sqrt(d_j), and the
// trailing lower triangle receives the rank-1 update -C_ij conj(C_kj).
// A pivot that is not > 0 (NaN included) stops the factorization and sets
// info = j+1, the LAPACK zpotrf convention.
#include "hs_internal.h"
#include "../../include/hs_build.h"

namespace hs {

namespace {

constexpr int PREP_THREADS = 256;
constexpr int PACKED_MAX = HS_MAX_NL * (HS_MAX_NL + 1) / 2;

__device__ __forceinline__ int pidx(int i, int k) { return i * (i + 1) / 2 + k; }

__global__ void __launch_bounds__(PREP_THREADS)
k_prep(Atoms at, const double2 *__restrict__ T_AA, const double2 *__restrict__ T_BB,
       const double2 *__restrict__ U, double2 *__restrict__ M1, double2 *__restrict__ M2,
       double *__restrict__ d, int *__restrict__ sel, int *__restrict__ info_out) {
    __shared__ double2 L[PACKED_MAX];
    __shared__ double diag[HS_MAX_NL];

    const int a = blockIdx.x;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    constexpr int NW = PREP_THREADS / 64;

    const int r0 = at.row_off[a];
    const int n = at.row_off[a + 1] - r0;
    const long long t0 = at.t_off[a];
    const double2 *taa = T_AA + t0;

    // lower triangle of T_AA,a into LDS, eight loads in flight per thread
    const int nn = n * n;
    constexpr int BATCH = 8;
    for (int e0 = 0; e0 < nn; e0 += BATCH * PREP_THREADS) {
        double2 v[BATCH];
#pragma unroll
        for (int b = 0; b < BATCH; ++b) {
            const int e = e0 + b * PREP_THREADS + tid;
            v[b] = taa[e < nn ? e : nn - 1];   // clamped: every load in bounds
        }
#pragma unroll
        for (int b = 0; b < BATCH; ++b) {
            const int e = e0 + b * PREP_THREADS + tid;
            if (e < nn) {
                const int i = e / n, k = e - (e / n) * n;
                if (k <= i) L[pidx(i, k)] = v[b];
            }
        }
    }
    __syncthreads();

    int info = 0;
    for (int j = 0; j < n; ++j) {
        const double dj = L[pidx(j, j)].x;
        if (!(dj > 0.0)) {
            info = j + 1;
            break;
        }
        const double cjj = sqrt(dj);
        if (tid == 0) diag[j] = cjj;
        for (int i = j + 1 + tid; i < n; i += PREP_THREADS) {
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

    double2 *m1 = M1 + t0;
    double2 *m2 = M2 + t0;
    const double2 *tbb = T_BB + t0;
    if (info == 0) {
        for (int e = tid; e < nn; e += PREP_THREADS) {
            const int i = e / n, k = e % n;
            double2 v = {0.0, 0.0};
            if (k < i) v = L[pidx(i, k)];
            else if (k == i) v.x = diag[i];
            m1[e] = v;
        }
    } else {
        for (int e = tid; e < nn; e += PREP_THREADS) {
            const int i = e / n, k = e % n;
            double2 v;
            if (k < i) v = taa[(long long)i * n + k];
            else if (k > i) {
                v = taa[(long long)k * n + i];
                v.y = -v.y;
            } else {
                v.x = taa[(long long)i * n + i].x;
                v.y = 0.0;
            }
            m1[e] = v;
        }
    }
    for (int e = tid; e < nn; e += PREP_THREADS) {
        const int i = e / n, k = e % n;
        double2 v;
        if (k < i) v = tbb[(long long)i * n + k];
        else if (k > i) {
            v = tbb[(long long)k * n + i];
            v.y = -v.y;
        } else {
            v.x = tbb[(long long)i * n + i].x;
            v.y = 0.0;
        }
        v.x *= 0.5;
        v.y *= 0.5;
        m2[e] = v;
    }
    const int K = at.K;
    for (int l = tid; l < n; l += PREP_THREADS) {
        const double2 u = U[r0 + l];
        d[r0 + l] = 1.0;
        d[K + r0 + l] = u.x * u.x + u.y * u.y;
        sel[r0 + l] = 0;
        sel[K + r0 + l] = 0;
        sel[2 * K + r0 + l] = info != 0;
    }
    if (tid == 0) info_out[a] = info;
}

}  // namespace

hipError_t launch_prep(const Atoms &at, const double2 *T_AA, const double2 *T_BB,
                       const double2 *U, double2 *M1, double2 *M2, double *d,
                       int *sel, int *info, hipStream_t st) {
    hipLaunchKernelGGL(k_prep, dim3(at.n_atoms), dim3(PREP_THREADS), 0, st, at, T_AA, T_BB, U,
                       M1, M2, d, sel, info);
    return hipGetLastError();
}

}  // namespace hs
