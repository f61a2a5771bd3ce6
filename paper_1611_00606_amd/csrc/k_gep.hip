// Reduction of the generalized eigenproblem H x = lambda S x (Sec. 1.1) to
// standard form, the step after the build:
//     S = L L^H  (L lower, positive real diagonal),   Ht = L^{-1} H L^{-H}.
//
// The O(N^3) work runs as products on the complex FP64 MFMA tile engine with
// direct global -> LDS loads (zmfma_direct.h):
//   factor, right-looking over panels of LB = 128 columns (lookahead on a
//   second stream):
//     k_gep_leaf                        Cholesky of the diagonal block and the
//                                       inverse M11 = L11^{-1} (one workgroup)
//     LH21 = M11 S21^H                  (= L21^H, the panel)
//     S22 -= L21 L21^H                  lower triangle, contraction over 128
//   invert, recursive over the same blocks (split at m):
//     M21 = -M22 (L21 M11)              M = L^{-1}
//   then, with MH = M^H = L^{-H} (upper triangular), below N = 4096
//     V  = H MH                         (= (L^{-1} H)^H for Hermitian H)
//     Ht = V^H MH                       lower triangle, then mirrored
//   and from N = 4096 on, with HL the lower triangle of H (half diagonal),
//     WH = HL^H MH                      (= (M HL)^H, upper triangular)
//     Ht = WH^H MH + M WH               two-term lower triangle, mirrored
//
// Work: N^3/3 complex multiply-adds for the factor and its inverse; then
// N^3/2 for V and N^3/6 for the lower triangle of Ht (triangular operands
// skip their zero blocks), N^3 in all = 8 N^3 real flops; or, in the
// two-term form, N^3/6 for WH and N^3/3 for Ht, 5N^3/6 in all = 20/3 N^3
// real flops. The minimal count of the reduction (LAPACK's zpotrf + zhegst)
// is 16/3 N^3. The explicit inverse of L is the usual choice for this
// reduction in FLAPW eigensolvers; its error grows with cond(L) =
// cond(S)^{1/2} like that of the substitutions.
//
// Once the factorization passes the top split of the inverse's recursion,
// the leading block's inverse and the matching columns of the result run on
// a third stream beside it.
//
// Storage (all N x N row-major complex): L (output; working copy of S's
// lower triangle during the factorization), LH (panels L21^H, then V),
// M = L^{-1} and MH = L^{-H} (zero outside their triangles), W (S21^H,
// L21 M11), Ht (output).
#include <algorithm>
#include <cstdint>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "hs_internal.h"
#include "zmfma_direct.h"
#include "zmfma_tile.h"

namespace hs {

namespace {

using MmCfg = TileCfg<128, 128, 16, 2, 4>;

// Share of the compute units (in quarters) the work moved off the
// factorization's critical path may occupy.
#ifndef HS_GEP_BG_QUARTERS
#define HS_GEP_BG_QUARTERS 3
#endif

// product flags
constexpr int MM_PU = 1;      // P upper triangular: k <= row of C
constexpr int MM_QL = 2;      // Q lower triangular: k >= column of C
constexpr int MM_QU = 4;      // Q upper triangular: k <= column of C
constexpr int MM_LOWER = 8;   // only C's lower triangle (square region)
constexpr int MM_MASK = 16;   // only elements on or below the diagonal (any region)
constexpr int MM_PL = 32;     // P lower triangular: k >= row of C
constexpr int MM_UPPER = 64;  // only C's upper triangle (square region); zeros below it
// epilogue
constexpr int OP_STORE = 0, OP_NEG = 1, OP_SUB = 2;

// One product, or several independent ones on the same three matrices
// (the nodes of one level of the inverse's recursion) in one launch.
struct MmJob {
    int i0, i1, j0, j1;       // C rows (P columns), C columns (Q columns)
    int k0, k1;               // contraction rows of P and Q
    int ntr, ntc;             // tile rows / columns of the rectangle
    int start;                // first block of this job
    int flags;                // MM_* of this job
};
constexpr int MM_JOBS = 32;

struct MmArgs {
    const double2 *P, *Q;
    const double2 *P2, *Q2;   // second term, same rectangle and contraction range
    double2 *C;
    int N;                    // leading dimension of P, Q, C
    int op;
    int njobs;
    int total;                // tiles over all jobs (blocks loop over them)
    MmJob job[MM_JOBS];
};

// C[i][j] (op)= sum_k conj(P[k][i]) Q[k][j] over each job's rectangle, in
// absolute indices; the triangular flags trim each tile's contraction range
// to the rows where both operands can be nonzero. G3: 3 real products per
// complex product (the 3M form of the tile engine).
template <int NSEG, bool G3>
__device__ __forceinline__ void mm_tile(const MmArgs &args, int tile, double2 *lds) {
    using Cfg = MmCfg;
    const int N = args.N;
    int jb = 0;
#pragma unroll
    for (int t = 1; t < MM_JOBS; ++t)
        if (t < args.njobs && tile >= args.job[t].start) jb = t;
    const int flags = args.job[jb].flags;
    const int bid = tile - args.job[jb].start;
    const int ntr = args.job[jb].ntr, ntc = args.job[jb].ntc;
    const int i0 = args.job[jb].i0, i1 = args.job[jb].i1;
    const int j0 = args.job[jb].j0, j1 = args.job[jb].j1;
    // Tiles whose contraction is longest go first (the triangular flags
    // make it depend on the tile row or column).
    int ti, tj;
    if (flags & MM_UPPER) {   // upper triangle, tj >= ti, by diagonals from the far corner
        int r = (int)((sqrt(8.0 * bid + 1.0) - 1.0) * 0.5);
        while ((r + 1) * (r + 2) / 2 <= bid) ++r;
        while (r * (r + 1) / 2 > bid) --r;
        ti = bid - r * (r + 1) / 2;
        tj = ti + ntr - 1 - r;
    } else if (flags & MM_LOWER) {   // lower triangle, tj <= ti
        const bool byc = flags & MM_QU;   // contraction grows with tj: last columns first
        const int t = byc ? bid : ntr * (ntr + 1) / 2 - 1 - bid;
        int r = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
        while ((r + 1) * (r + 2) / 2 <= t) ++r;
        while (r * (r + 1) / 2 > t) --r;
        if (byc) {   // column ntr-1-r, its r+1 tiles from the diagonal down
            tj = ntr - 1 - r;
            ti = tj + (t - r * (r + 1) / 2);
        } else {     // reversed row-major
            ti = r;
            tj = t - r * (r + 1) / 2;
        }
    } else if ((flags & MM_PL) && (flags & MM_QU)) {   // longest: largest tj - ti first
        int rem = bid, c = ntc - 1;
        for (;; --c) {   // diagonals tj - ti = c, from the far corner
            const int lo = c < 0 ? -c : 0;
            const int hi = ntr < ntc - c ? ntr : ntc - c;
            const int cnt = hi > lo ? hi - lo : 0;
            if (rem < cnt || c <= -ntr) {
                ti = lo + rem;
                break;
            }
            rem -= cnt;
        }
        tj = ti + c;
    } else if (flags & MM_PU) {   // longest: last tile rows
        ti = ntr - 1 - bid / ntc;
        tj = bid % ntc;
    } else if (flags & MM_QU) {   // longest: last tile columns
        tj = ntc - 1 - bid / ntr;
        ti = bid % ntr;
    } else {                      // MM_QL: first tile columns
        tj = bid / ntr;
        ti = bid % ntr;
    }
    const int m0 = i0 + ti * Cfg::BM;
    const int n0 = j0 + tj * Cfg::BN;
    if (m0 >= i1 || n0 >= j1) return;
    int klo = args.job[jb].k0, khi = args.job[jb].k1;
    if (flags & MM_PU) khi = min(khi, m0 + Cfg::BM);
    if (flags & MM_QU) khi = min(khi, n0 + Cfg::BN);
    if (flags & MM_QL) klo = max(klo, n0);
    if (flags & MM_PL) klo = max(klo, m0);

    Segs<NSEG, false, false> t;
    t.nseg = NSEG;
    t.len = khi > klo ? khi - klo : 0;
    t.ldp = N;
    t.ldq = N;
    const long long k0 = (long long)(t.len ? klo : 0) * N;
    t.P[0] = args.P + k0;
    t.Q[0] = args.Q + k0;
    if constexpr (NSEG == 2) {
        t.P[1] = args.P2 + k0;
        t.Q[1] = args.Q2 + k0;
    }
    t.palt = nullptr;
    t.sel = nullptr;
    t.qscale = nullptr;
    Acc<Cfg> acc;
    ztile_direct<Cfg, NSEG, false, false, G3>(t, m0, i1, n0, j1, acc, lds);

    const bool lower = flags & (MM_LOWER | MM_MASK);
    const bool upper = flags & MM_UPPER;
    const int op = args.op;
    double2 *C = args.C;
#pragma unroll
    for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
        for (int j = 0; j < Cfg::TN; ++j) {
            const int g = n0 + acc_col<Cfg>(j);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gp = m0 + acc_row<Cfg>(i, v);
                if (gp < i1 && g < j1 && (!lower || g <= gp)) {
                    double2 *o = C + (long long)gp * N + g;
                    const bool z = upper && g < gp;
                    const double re = z ? 0.0 : acc.re[i][j][v], im = z ? 0.0 : acc.im[i][j][v];
                    if (op == OP_SUB) {
                        double2 r = *o;
                        r.x -= re;
                        r.y -= im;
                        *o = r;
                    } else if (op == OP_NEG) {
                        *o = double2{-re, -im};
                    } else {
                        *o = double2{re, im};
                    }
                }
            }
        }
}

// Blocks loop over the tiles (a launch may have fewer blocks than tiles when
// it runs beside latency-critical work).
template <int NSEG, bool G3>
__global__ void __launch_bounds__(MmCfg::NT) k_gep_mm(const MmArgs args) {
    __shared__ double2 lds[MmCfg::LDS_ELEMS];
    for (int tile = blockIdx.x; tile < args.total; tile += gridDim.x) {
        mm_tile<NSEG, G3>(args, tile, lds);
        __syncthreads();   // LDS is reused by the next tile
    }
}

// Leaf: Cholesky of the diagonal block [kb, kb + nb) (nb <= LB = 128) of the
// working matrix (lower triangle in L) and the inverse of the factor, by one
// workgroup of 8 waves. The block, padded to 128 x 128 with the identity,
// sits in LDS as the 36 lower 16 x 16 tiles (rows XOR-swizzled, so that the
// MFMA fragment loads and the accumulator stores hit distinct banks).
//   factor, right-looking over 16-column panels P:
//     wave 0: Cholesky of the diagonal tile in registers (lane r holds row
//             r; values broadcast with readlane), for P > 0 right after its
//             own update of that tile in the previous panel's trailing step;
//     panel:  L_IP = C_IP L_PP^{-H}            by substitution, one thread
//             per row of the panel;
//     update: C_IJ -= L_IP L_JP^H, P < J <= I   tiles spread over waves
//             1..7 (wave 0 takes tile (P+1, P+1), then factors it).
//   inverse X = L^{-1}, in place: every wave inverts one diagonal tile, then
//     for block rows I = 1..7: X_IJ = -X_II sum_{J<=K<I} L_IK X_KJ, J < I.
// A pivot that is not > 0 (NaN included) records kb + j + 1 in *info unless an
// earlier block failed (the outputs are undefined then). Writes the block of
// L, of M = X (lower) and of MH = X^H (upper).
constexpr int LB = 128;
constexpr int LT = LB / 16;               // tiles per side
constexpr int LNT = LT * (LT + 1) / 2;    // lower tiles

__device__ __forceinline__ double2 *ltile(double2 *T, int I, int K) {
    return T + (I * (I + 1) / 2 + K) * 256;
}
__device__ __forceinline__ int lsw(int a, int b) { return a * 16 + (b ^ a); }

// value of v in lane `src` (wave-uniform src)
__device__ __forceinline__ double bcast(double v, int src) {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)u, src);
    const int hi = __builtin_amdgcn_readlane((int)(u >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Lanes 0..15 hold the rows of a 16 x 16 Hermitian tile (lower triangle
// used); on return the rows of its Cholesky factor. Returns 0 or the
// 1-based index of the first pivot that is not > 0. Each step's pivot comes
// from lane j by readlane; 1/sqrt of it from the hardware estimate refined by
// two Newton steps (y += y (1 - d y^2) / 2; the estimate is good to far more
// than the 2^-13 two steps need for full precision), and sqrt(d) = d / sqrt(d);
// the scaled entries l_kj broadcast with readlane.
__device__ __forceinline__ int chol16(double2 (&a)[16], int lane) {
    int inf = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const double d = bcast(a[j].x, j);
        if (!(d > 0.0) && inf == 0) inf = j + 1;
        double rc = __builtin_amdgcn_rsq(d);
        rc = fma(0.5 * rc, fma(-d * rc, rc, 1.0), rc);
        rc = fma(0.5 * rc, fma(-d * rc, rc, 1.0), rc);
        const double c = d * rc;
        a[j] = lane == j ? double2{c, 0.0} : double2{a[j].x * rc, a[j].y * rc};
#pragma unroll
        for (int k = j + 1; k < 16; ++k) {   // a_rk -= l_rj conj(l_kj)
            const double lx = bcast(a[j].x, k), ly = bcast(a[j].y, k);
            a[k].x -= a[j].x * lx + a[j].y * ly;
            a[k].y -= a[j].y * lx - a[j].x * ly;
        }
    }
    return inf;
}

// Column (lane & 15) of the inverse of the lower-triangular 16 x 16 tile D
// (in LDS): x_i = (delta_ic - sum_{k<i} l_ik x_k) / l_ii, the factor read with
// broadcast loads (the same address in every lane).
__device__ __forceinline__ void inv16(const double2 *D, double2 (&x)[16], int lane) {
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        double2 t = double2{(lane & 15) == i ? 1.0 : 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < i; ++k) {
            const double2 l = D[lsw(i, k)];   // l_ik
            t.x -= l.x * x[k].x - l.y * x[k].y;
            t.y -= l.x * x[k].y + l.y * x[k].x;
        }
        const double rd = 1.0 / D[lsw(i, i)].x;
        x[i] = double2{t.x * rd, t.y * rd};
    }
}

struct Cacc {
    v4d re, im;
};

// c += A B^H for 16 x 16 tiles (c[i][j] += sum_k A[i][k] conj(B[j][k]))
__device__ __forceinline__ void mma_abh(Cacc &c, const double2 *A, const double2 *B, int lane) {
#pragma unroll
    for (int k0 = 0; k0 < 16; k0 += 4) {
        const double2 x = A[lsw(lane & 15, k0 + (lane >> 4))];
        const double2 y = B[lsw(lane & 15, k0 + (lane >> 4))];
        c.re = __builtin_amdgcn_mfma_f64_16x16x4f64(x.x, y.x, c.re, 0, 0, 0);
        c.re = __builtin_amdgcn_mfma_f64_16x16x4f64(x.y, y.y, c.re, 0, 0, 0);
        c.im = __builtin_amdgcn_mfma_f64_16x16x4f64(x.y, y.x, c.im, 0, 0, 0);
        c.im = __builtin_amdgcn_mfma_f64_16x16x4f64(x.x, -y.y, c.im, 0, 0, 0);
    }
}

// c += A B for 16 x 16 tiles
__device__ __forceinline__ void mma_ab(Cacc &c, const double2 *A, const double2 *B, int lane) {
#pragma unroll
    for (int k0 = 0; k0 < 16; k0 += 4) {
        const double2 x = A[lsw(lane & 15, k0 + (lane >> 4))];
        const double2 y = B[lsw(k0 + (lane >> 4), lane & 15)];
        c.re = __builtin_amdgcn_mfma_f64_16x16x4f64(x.x, y.x, c.re, 0, 0, 0);
        c.re = __builtin_amdgcn_mfma_f64_16x16x4f64(x.y, -y.y, c.re, 0, 0, 0);
        c.im = __builtin_amdgcn_mfma_f64_16x16x4f64(x.x, y.y, c.im, 0, 0, 0);
        c.im = __builtin_amdgcn_mfma_f64_16x16x4f64(x.y, y.x, c.im, 0, 0, 0);
    }
}

__device__ __forceinline__ void acc_zero(Cacc &c) {
    c.re = v4d{0.0, 0.0, 0.0, 0.0};
    c.im = v4d{0.0, 0.0, 0.0, 0.0};
}

// lower-triangle tile t of an n x n tile grid -> (i, j), j <= i
__device__ __forceinline__ void tri_decode(int t, int &i, int &j) {
    i = 0;
    while ((i + 1) * (i + 2) / 2 <= t) ++i;
    j = t - i * (i + 1) / 2;
}

__global__ void __launch_bounds__(512)
k_gep_leaf(double2 *__restrict__ L, double2 *__restrict__ M, double2 *__restrict__ MH, int N,
           int kb, int nb, int *__restrict__ info) {
    __shared__ double2 T[LNT * 256];   // 144 KiB
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);

    // stage: element (i, k), k <= i, of the padded block (loads issued together)
    for (int c = 0; c < LB * LB / 512; c += 8) {
        double2 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = tid + 512 * (c + u), i = e / LB, k = e % LB;
            v[u] = double2{i == k ? 1.0 : 0.0, 0.0};
            if (k <= i && i < nb) v[u] = L[(long long)(kb + i) * N + kb + k];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = tid + 512 * (c + u), i = e / LB, k = e % LB;
            if (k <= i) ltile(T, i >> 4, k >> 4)[lsw(i & 15, k & 15)] = v[u];
        }
    }
    __syncthreads();

    int inf = 0;
    // Cholesky of diagonal tile P by wave 0
    const auto diag = [&](int P) {
        double2 *D = ltile(T, P, P);
        double2 a[16];
        const int r = lane & 15;
#pragma unroll
        for (int k = 0; k < 16; ++k) a[k] = D[lsw(r, k)];
        const int f = chol16(a, lane);
        if (f != 0 && inf == 0 && 16 * P + f <= nb) inf = 16 * P + f;
        if (lane < 16) {
#pragma unroll
            for (int k = 0; k < 16; ++k) D[lsw(lane, k)] = a[k];
        }
    };
    // C_IJ -= L_IP L_JP^H for the t-th tile of the trailing triangle of panel P
    const auto trail = [&](int P, int t) {
        int ti, tj;
        tri_decode(t, ti, tj);
        const int I = P + 1 + ti, J = P + 1 + tj;
        Cacc c;
        acc_zero(c);
        mma_abh(c, ltile(T, I, P), ltile(T, J, P), lane);
        double2 *C = ltile(T, I, J);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            double2 &o = C[lsw(4 * v + (lane >> 4), lane & 15)];
            o.x -= c.re[v];
            o.y -= c.im[v];
        }
    };
    if (w == 0) diag(0);
    __syncthreads();
    for (int P = 0; P < LT; ++P) {
        // panel: row r of L_IP solves x L_PP^H = C_IP[r] by substitution,
        // x_j = (c_j - sum_{k<j} x_k conj(l_jk)) / l_jj, one thread per row
        if (tid < (LT - 1 - P) * 16) {
            const double2 *D = ltile(T, P, P);
            double2 *C = ltile(T, P + 1 + (tid >> 4), P);
            const int rr = tid & 15;
            double rd[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) rd[j] = 1.0 / D[lsw(j, j)].x;
            double2 x[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) x[k] = C[lsw(rr, k)];
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                double2 t = x[j];
#pragma unroll
                for (int k = 0; k < j; ++k) {   // t -= x_k conj(l_jk)
                    const double2 l = D[lsw(j, k)];
                    t.x -= x[k].x * l.x + x[k].y * l.y;
                    t.y -= x[k].y * l.x - x[k].x * l.y;
                }
                x[j] = double2{t.x * rd[j], t.y * rd[j]};
            }
#pragma unroll
            for (int k = 0; k < 16; ++k) C[lsw(rr, k)] = x[k];
        }
        __syncthreads();
        // trailing lower triangle: wave 0 updates the next diagonal tile
        // (t = 0) and factors it at once, beside the other waves' updates
        const int n = LT - 1 - P;
        if (w == 0) {
            if (n > 0) {
                trail(P, 0);
                asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
                diag(P + 1);
            }
        } else {
            for (int t = w; t < n * (n + 1) / 2; t += 7) trail(P, t);
        }
        __syncthreads();
    }
    if (tid == 0 && inf != 0 && *info == 0) *info = kb + inf;
    for (int e = tid; e < LB * LB; e += 512) {
        const int i = e / LB, k = e % LB;
        if (k <= i && i < nb)
            L[(long long)(kb + i) * N + kb + k] = ltile(T, i >> 4, k >> 4)[lsw(i & 15, k & 15)];
    }

    // inverse: diagonal tiles, one per wave
    {
        double2 *D = ltile(T, w, w);
        double2 x[16];
        inv16(D, x, lane);
        if (lane < 16) {
#pragma unroll
            for (int i = 0; i < 16; ++i) D[lsw(i, lane)] = i >= lane ? x[i] : double2{0.0, 0.0};
        }
    }
    __syncthreads();
    // block rows: X_IJ = -X_II sum_{J<=K<I} L_IK X_KJ (wave w: J = w)
    for (int I = 1; I < LT; ++I) {
        Cacc c;
        acc_zero(c);
        if (w < I)
            for (int K = w; K < I; ++K) mma_ab(c, ltile(T, I, K), ltile(T, K, w), lane);
        __syncthreads();   // row I of L fully read before it is overwritten
        if (w < I) {
            const double2 *X = ltile(T, I, I);
            Cacc o;
            acc_zero(o);
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {   // B fragment rows 4 s4 .. = accumulator element s4
                const double2 x = X[lsw(lane & 15, 4 * s4 + (lane >> 4))];
                const double br = c.re[s4], bi = c.im[s4];
                o.re = __builtin_amdgcn_mfma_f64_16x16x4f64(x.x, br, o.re, 0, 0, 0);
                o.re = __builtin_amdgcn_mfma_f64_16x16x4f64(x.y, -bi, o.re, 0, 0, 0);
                o.im = __builtin_amdgcn_mfma_f64_16x16x4f64(x.x, bi, o.im, 0, 0, 0);
                o.im = __builtin_amdgcn_mfma_f64_16x16x4f64(x.y, br, o.im, 0, 0, 0);
            }
            double2 *C = ltile(T, I, w);
#pragma unroll
            for (int v = 0; v < 4; ++v)
                C[lsw(4 * v + (lane >> 4), lane & 15)] = double2{-o.re[v], -o.im[v]};
        }
        __syncthreads();
    }
    for (int e = tid; e < LB * LB; e += 512) {
        const int i = e / LB, k = e % LB;
        if (i < nb && k < nb) {
            if (k <= i) M[(long long)(kb + i) * N + kb + k] = ltile(T, i >> 4, k >> 4)[lsw(i & 15, k & 15)];
            else {   // MH[i][k] = conj(X[k][i]), k > i
                const double2 v = ltile(T, k >> 4, i >> 4)[lsw(k & 15, i & 15)];
                MH[(long long)(kb + i) * N + kb + k] = double2{v.x, -v.y};
            }
            if (k == i) {
                const double2 v = ltile(T, i >> 4, i >> 4)[lsw(i & 15, i & 15)];
                MH[(long long)(kb + i) * N + kb + k] = double2{v.x, -v.y};
            }
        }
    }
}

// L := lower(S) (upper triangle zero), M := 0, MH := 0, LH := 0 below the
// diagonal, HL := lower(H) with half its diagonal (so that H = HL + HL^H)
__global__ void __launch_bounds__(256)
k_gep_init(const double2 *__restrict__ H, const double2 *__restrict__ S, double2 *__restrict__ L,
           double2 *__restrict__ M, double2 *__restrict__ MH, double2 *__restrict__ LH,
           double2 *__restrict__ HL, int N) {
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= (long long)N * N) return;
    const int i = (int)(e / N), j = (int)(e % N);
    const double2 z = double2{0.0, 0.0};
    double2 sv = z;
    if (j <= i) sv = S[e];
    L[e] = sv;
    M[e] = z;
    MH[e] = z;
    if (j < i) LH[e] = z;
    if (HL) {
        double2 hv = z;
        if (j <= i) hv = H[e];
        if (j == i) hv = double2{0.5 * hv.x, 0.0};
        HL[e] = hv;
    }
}

__global__ void k_gep_info_clear(int *info) { *info = 0; }

// D[j][i] = conj(X[i][j]) for i in [i0, i1), j in [j0, j1) of each job
// (blockIdx.z), through 32 x 32 LDS tiles (blockIdx.y: source tile row,
// blockIdx.x: source tile column)
struct CtJobs {
    int r[MM_JOBS][4];   // i0, i1, j0, j1
};

__global__ void __launch_bounds__(256)
k_gep_conj_t(const double2 *__restrict__ X, double2 *__restrict__ D, int N, const CtJobs jobs) {
    __shared__ double2 tile[32][33];
    const int z = blockIdx.z;
    const int i0 = jobs.r[z][0], i1 = jobs.r[z][1], j0 = jobs.r[z][2], j1 = jobs.r[z][3];
    const int si = i0 + blockIdx.y * 32, sj = j0 + blockIdx.x * 32;
    if (si >= i1 || sj >= j1) return;   // the grid covers the largest job
    const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
    for (int r = ty; r < 32; r += 8) {
        const int gr = si + r, gc = sj + tx;
        if (gr < i1 && gc < j1) tile[r][tx] = X[(long long)gr * N + gc];
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int dr = sj + r, dc = si + tx;   // D[dr][dc] = conj(X[dc][dr])
        if (dr < j1 && dc < i1) {
            double2 v = tile[tx][r];
            v.y = -v.y;
            D[(long long)dr * N + dc] = v;
        }
    }
}

struct Gep {
    double2 *L, *LH, *M, *MH, *W, *HL;
    int N;
    int *info;
    hipStream_t st;
    int cap;   // most blocks per product launch (0: one per tile)
    bool g3;   // products in the 3M form
};

#define GEP_TRY(x)                              \
    do {                                        \
        hipError_t e_ = (x);                    \
        if (e_ != hipSuccess) return e_;        \
    } while (0)

struct Rect {
    int i0, i1, j0, j1, k0, k1;
};

// ---------------------------------------------------------------------------
// Schedule check (host only). With a recorder installed the orchestration
// below runs unchanged but issues nothing: every launch is logged with its
// stream and the rectangles of each matrix it reads and writes (per output
// tile, with the tile's trimmed contraction range), every event record and
// stream wait with its stream and event. sched_check then runs a
// vector-clock pass over the log: two launches on different streams that
// touch a common 128 x 128 cell of a matrix, one of them writing, must be
// ordered by a chain of stream order and event waits.
enum SchedBuf { SB_H, SB_S, SB_L, SB_HT, SB_LH, SB_M, SB_MH, SB_W, SB_HL, SB_INFO, SB_COUNT };
const char *const kSchedBufName[SB_COUNT] = {"H", "S", "L", "Ht", "LH", "M", "MH", "W", "HL", "info"};

struct SchedAcc {
    int buf, r0, r1, c0, c1;   // element rectangle [r0, r1) x [c0, c1)
    bool write;
};
struct SchedOp {
    int kind;          // 0 launch, 1 event record, 2 stream wait
    hipStream_t st;
    hipEvent_t ev;
    const char *name;
    std::vector<SchedAcc> acc;
};
struct Sched {
    std::vector<SchedOp> ops;
    const void *base[SB_COUNT] = {};
    int drop_tag = 0;            // waits with this tag are left out (a test hook)
    uintptr_t next_event = 1;
    int buf(const void *p) const {
        for (int i = 0; i < SB_COUNT; ++i)
            if (base[i] == p) return i;
        return -1;
    }
    SchedOp &launch(hipStream_t st, const char *name) {
        ops.push_back(SchedOp{0, st, nullptr, name, {}});
        return ops.back();
    }
    void add(SchedOp &op, const void *p, int r0, int r1, int c0, int c1, bool write) {
        const int b = buf(p);
        if (b >= 0 && r1 > r0 && c1 > c0) op.acc.push_back(SchedAcc{b, r0, r1, c0, c1, write});
    }
};
thread_local Sched *g_sched = nullptr;

hipError_t ev_create(hipEvent_t *e) {
    if (g_sched) {
        *e = reinterpret_cast<hipEvent_t>(g_sched->next_event++);
        return hipSuccess;
    }
    return hipEventCreateWithFlags(e, hipEventDisableTiming);
}
void ev_destroy(hipEvent_t e) {
    if (!g_sched && e) (void)hipEventDestroy(e);
}
hipError_t ev_record(hipEvent_t e, hipStream_t st) {
    if (g_sched) {
        g_sched->ops.push_back(SchedOp{1, st, e, "record", {}});
        return hipSuccess;
    }
    return hipEventRecord(e, st);
}
// Wait sites, by tag (hs_gep_check_schedule's drop argument).
enum WaitTag {
    WT_TRANSPOSE_AFTER_BLOCK = 1,   // next S21^H after the next column block's update
    WT_PANEL_AFTER_TRANSPOSE,       // panel product after S21^H
    WT_BLOCK_AFTER_BULK,            // next column block after the previous bulk update
    WT_AHEAD_AFTER_PANEL,           // L21 and bulk update after the panel product
    WT_JOIN_AHEAD,                  // end of the factorization: lookahead stream
    WT_JOIN_TRANSPOSE,              // end of the factorization: transposes stream
    WT_FORK,                        // background stream after the top split's panel
    WT_FORK_AHEAD,                  // background stream after the pending lookahead work
    WT_END_AFTER_INVERSE,           // top split's M21 after the leading block's inverse
    WT_END_AFTER_BACKGROUND         // Ht's last rows after the background's products
};
hipError_t ev_wait(hipStream_t st, hipEvent_t e, int tag) {
    if (g_sched) {
        if (tag != g_sched->drop_tag) g_sched->ops.push_back(SchedOp{2, st, e, "wait", {}});
        return hipSuccess;
    }
    return hipStreamWaitEvent(st, e, 0);
}

// The vector-clock pass. Returns the number of unordered conflicting pairs
// of launches and describes the first few in `report`.
int sched_check(const Sched &sc, int N, std::string &report) {
    constexpr int CB = 128;
    const int nc = (N + CB - 1) / CB;
    std::vector<hipStream_t> streams;
    auto sid = [&](hipStream_t st) {
        for (size_t i = 0; i < streams.size(); ++i)
            if (streams[i] == st) return (int)i;
        streams.push_back(st);
        return (int)streams.size() - 1;
    };
    for (const SchedOp &op : sc.ops) sid(op.st);
    const int ns = (int)streams.size();
    std::vector<std::vector<int>> vc(ns, std::vector<int>(ns, 0));
    std::vector<std::pair<hipEvent_t, std::vector<int>>> evc;
    struct Last {
        int op = -1, st = 0, clk = 0;
    };
    struct CellState {
        Last w;
        std::vector<Last> r;   // latest read per stream since the last write
    };
    const size_t ncell = (size_t)SB_COUNT * nc * nc;
    std::vector<CellState> cells(ncell);
    std::vector<signed char> mark(ncell, -1);   // per launch: 0 read, 1 write
    std::vector<size_t> touched;
    std::set<std::pair<int, int>> races;
    for (int i = 0; i < (int)sc.ops.size(); ++i) {
        const SchedOp &op = sc.ops[i];
        const int s = sid(op.st);
        if (op.kind == 1) {
            bool found = false;
            for (auto &e : evc)
                if (e.first == op.ev) {
                    e.second = vc[s];
                    found = true;
                }
            if (!found) evc.push_back({op.ev, vc[s]});
            continue;
        }
        if (op.kind == 2) {
            for (auto &e : evc)
                if (e.first == op.ev)
                    for (int k = 0; k < ns; ++k) vc[s][k] = std::max(vc[s][k], e.second[k]);
            continue;
        }
        ++vc[s][s];
        const std::vector<int> &me = vc[s];
        touched.clear();
        for (const SchedAcc &a : op.acc) {
            const int cr0 = a.buf == SB_INFO ? 0 : a.r0 / CB, cr1 = a.buf == SB_INFO ? 0 : (a.r1 - 1) / CB;
            const int cc0 = a.buf == SB_INFO ? 0 : a.c0 / CB, cc1 = a.buf == SB_INFO ? 0 : (a.c1 - 1) / CB;
            for (int r = cr0; r <= cr1; ++r)
                for (int c = cc0; c <= cc1; ++c) {
                    const size_t id = ((size_t)a.buf * nc + r) * nc + c;
                    if (mark[id] < 0) touched.push_back(id);
                    mark[id] = std::max<signed char>(mark[id], a.write ? 1 : 0);
                }
        }
        auto ordered = [&](const Last &l) { return l.st == s || me[l.st] >= l.clk; };
        auto race = [&](int other, size_t id) {
            if (races.count({other, i})) return;
            if (races.size() < 5) {
                const int b = (int)(id / ((size_t)nc * nc));
                const int r = (int)(id / nc % nc), c = (int)(id % nc);
                report += std::string(sc.ops[other].name) + " and " + op.name + " on " +
                          kSchedBufName[b] + " cell (" + std::to_string(r) + ", " +
                          std::to_string(c) + "); ";
            }
            races.insert({other, i});
        };
        for (size_t id : touched) {
            CellState &cs = cells[id];
            const bool w = mark[id] == 1;
            mark[id] = -1;
            if (cs.w.op >= 0 && !ordered(cs.w)) race(cs.w.op, id);
            if (w) {
                for (const Last &l : cs.r)
                    if (!ordered(l)) race(l.op, id);
                cs.r.clear();
                cs.w = Last{i, s, me[s]};
            } else {
                bool had = false;
                for (Last &l : cs.r)
                    if (l.st == s) {
                        l = Last{i, s, me[s]};
                        had = true;
                    }
                if (!had) cs.r.push_back(Last{i, s, me[s]});
            }
        }
    }
    return (int)races.size();
}

// The footprint of one product launch, tile by tile as mm_tile trims it.
void sched_mm(const Gep &g, const MmArgs &a) {
    using Cfg = MmCfg;
    SchedOp &op = g_sched->launch(g.st, a.P2 ? "k_gep_mm<2>" : "k_gep_mm<1>");
    for (int jb = 0; jb < a.njobs; ++jb) {
        const MmJob &j = a.job[jb];
        const int flags = j.flags;
        for (int ti = 0; ti < j.ntr; ++ti)
            for (int tj = 0; tj < j.ntc; ++tj) {
                if ((flags & MM_UPPER) && tj < ti) continue;
                if ((flags & MM_LOWER) && tj > ti) continue;
                const int m0 = j.i0 + ti * Cfg::BM, n0 = j.j0 + tj * Cfg::BN;
                if (m0 >= j.i1 || n0 >= j.j1) continue;
                const int m1 = std::min(m0 + Cfg::BM, j.i1), n1 = std::min(n0 + Cfg::BN, j.j1);
                int klo = j.k0, khi = j.k1;
                if (flags & MM_PU) khi = std::min(khi, m0 + Cfg::BM);
                if (flags & MM_QU) khi = std::min(khi, n0 + Cfg::BN);
                if (flags & MM_QL) klo = std::max(klo, n0);
                if (flags & MM_PL) klo = std::max(klo, m0);
                g_sched->add(op, a.P, klo, khi, m0, m1, false);
                g_sched->add(op, a.Q, klo, khi, n0, n1, false);
                if (a.P2) {
                    g_sched->add(op, a.P2, klo, khi, m0, m1, false);
                    g_sched->add(op, a.Q2, klo, khi, n0, n1, false);
                }
                g_sched->add(op, a.C, m0, m1, n0, n1, true);
            }
    }
}

// Products over the rectangles r[0 .. n), up to MM_JOBS per launch, with
// the flags rflags[t] of each (or flags for all when rflags is null); the
// blocks take the rectangles in the order given.
hipError_t mm_batch(const Gep &g, const double2 *P, const double2 *Q, double2 *C, const Rect *r,
                    int n, int flags, int op, const double2 *P2 = nullptr,
                    const double2 *Q2 = nullptr, const int *rflags = nullptr) {
    using Cfg = MmCfg;
    for (int b = 0; b < n; b += MM_JOBS) {
        MmArgs a = {};
        a.P = P;
        a.Q = Q;
        a.P2 = P2;
        a.Q2 = Q2;
        a.C = C;
        a.N = g.N;
        a.op = op;
        long long nblk = 0;
        for (int t = b; t < n && t < b + MM_JOBS; ++t) {
            if (r[t].i1 <= r[t].i0 || r[t].j1 <= r[t].j0) continue;
            MmJob &j = a.job[a.njobs++];
            j.i0 = r[t].i0;
            j.i1 = r[t].i1;
            j.j0 = r[t].j0;
            j.j1 = r[t].j1;
            j.k0 = r[t].k0;
            j.k1 = r[t].k1;
            j.ntr = (j.i1 - j.i0 + Cfg::BM - 1) / Cfg::BM;
            j.ntc = (j.j1 - j.j0 + Cfg::BN - 1) / Cfg::BN;
            j.start = (int)nblk;
            j.flags = rflags ? rflags[t] : flags;
            if (j.flags & (MM_LOWER | MM_UPPER)) {
                if (j.i0 != j.j0 || j.i1 != j.j1) return hipErrorInvalidValue;
                nblk += (long long)j.ntr * (j.ntr + 1) / 2;
            } else {
                nblk += (long long)j.ntr * j.ntc;
            }
        }
        if (a.njobs == 0) continue;
        a.total = (int)nblk;
        if (g_sched) {
            sched_mm(g, a);
            continue;
        }
        const long long grid = g.cap > 0 && nblk > g.cap ? g.cap : nblk;
        const dim3 gd((unsigned)grid), bd(Cfg::NT);
        if (P2 && g.g3)
            hipLaunchKernelGGL((k_gep_mm<2, true>), gd, bd, 0, g.st, a);
        else if (P2)
            hipLaunchKernelGGL((k_gep_mm<2, false>), gd, bd, 0, g.st, a);
        else if (g.g3)
            hipLaunchKernelGGL((k_gep_mm<1, true>), gd, bd, 0, g.st, a);
        else
            hipLaunchKernelGGL((k_gep_mm<1, false>), gd, bd, 0, g.st, a);
        GEP_TRY(hipGetLastError());
    }
    return hipSuccess;
}

hipError_t mm(const Gep &g, const double2 *P, const double2 *Q, double2 *C, int i0, int i1,
              int j0, int j1, int k0, int k1, int flags, int op) {
    const Rect r = {i0, i1, j0, j1, k0, k1};
    return mm_batch(g, P, Q, C, &r, 1, flags, op);
}

// Transposes of the rectangles r[0 .. n), up to MM_JOBS per launch.
hipError_t conj_t_batch(const Gep &g, const double2 *X, double2 *D, const Rect *r, int n) {
    for (int b = 0; b < n; b += MM_JOBS) {
        CtJobs j = {};
        int nj = 0, gx = 0, gy = 0;
        for (int t = b; t < n && t < b + MM_JOBS; ++t) {
            if (r[t].i1 <= r[t].i0 || r[t].j1 <= r[t].j0) continue;
            j.r[nj][0] = r[t].i0;
            j.r[nj][1] = r[t].i1;
            j.r[nj][2] = r[t].j0;
            j.r[nj][3] = r[t].j1;
            gx = std::max(gx, (r[t].j1 - r[t].j0 + 31) / 32);
            gy = std::max(gy, (r[t].i1 - r[t].i0 + 31) / 32);
            ++nj;
        }
        if (nj == 0) continue;
        if (g_sched) {
            SchedOp &op = g_sched->launch(g.st, "k_gep_conj_t");
            for (int t = 0; t < nj; ++t) {
                g_sched->add(op, X, j.r[t][0], j.r[t][1], j.r[t][2], j.r[t][3], false);
                g_sched->add(op, D, j.r[t][2], j.r[t][3], j.r[t][0], j.r[t][1], true);
            }
            continue;
        }
        hipLaunchKernelGGL(k_gep_conj_t, dim3(gx, gy, nj), dim3(256), 0, g.st, X, D, g.N, j);
        GEP_TRY(hipGetLastError());
    }
    return hipSuccess;
}

hipError_t conj_t(const Gep &g, const double2 *X, double2 *D, int i0, int i1, int j0, int j1) {
    const Rect r = {i0, i1, j0, j1, 0, 0};
    return conj_t_batch(g, X, D, &r, 1);
}

// Auxiliary streams per device (0: the factorization's lookahead, 1: work
// moved off the critical path, 2: the panels' transposes; with the caller's
// stream that is one hardware queue each at the default of four per
// process); default priority,
// created once and kept for the life of the process.
hipStream_t aux_stream(int which) {
    if (g_sched) return reinterpret_cast<hipStream_t>((uintptr_t)(0x100 + which));
    static std::mutex mu;
    static hipStream_t cached[64][3] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    std::lock_guard<std::mutex> lk(mu);
    if (!cached[dev][which]) {
        hipStream_t s = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
        cached[dev][which] = s;
    }
    return cached[dev][which];
}

// Cholesky, right-looking over panels of LB columns: factor and invert the
// diagonal block, then the panel L21 = S21 L11^{-H} (as LH21 = M11 S21^H) and
// the update of the trailing lower triangle S22 -= L21 L21^H.
// Lookahead (from 4 panels on), with three streams and panels in pairs:
//   caller's    leaf, panel product; after the first panel of a pair the
//               update of the next column block with it, after the second
//               the update of the next two column blocks with both panels
//               (contraction 2 LB);
//   lookahead   L21 = LH21^H (an output only); after the second panel of a
//               pair the bulk of the update with both panels (contraction
//               2 LB), beside the next two leaves and panels;
//   transposes  the next panel's S21^H, beside the next leaf.
// The update of the two column blocks after a pair waits for the previous
// pair's bulk update (both write those blocks); the bulk update and L21
// wait for the panel they use; the next S21^H waits for the update of its
// column block.
template <class Hook>
hipError_t factor(const Gep &g, Hook after_panel) {
    const int N = g.N;
    const int np = (N + LB - 1) / LB;
    Gep ga = g, gc = g;
    hipEvent_t e_panel = nullptr, e_bulk = nullptr, e_look = nullptr, e_next = nullptr,
               e_w = nullptr;
    bool ahead = np >= 4;
    if (ahead) {
        ga.st = aux_stream(0);
        gc.st = aux_stream(2);
        ahead = ga.st != nullptr && gc.st != nullptr && ev_create(&e_panel) == hipSuccess &&
                ev_create(&e_bulk) == hipSuccess && ev_create(&e_look) == hipSuccess &&
                ev_create(&e_next) == hipSuccess && ev_create(&e_w) == hipSuccess;
    }
    // recorded events still to be waited for (no wait on an unrecorded event);
    // e_bulk: the last bulk update, e_look: everything on the lookahead stream
    bool bulk_pending = false, look_pending = false, w_pending = false;
    hipError_t err = hipSuccess;
    // S21^H of the first panel, beside the first leaf
    const auto next_s21h = [&](int c0, int c1) -> hipError_t {   // columns [c0, c1)
        GEP_TRY(ev_record(e_next, g.st));
        GEP_TRY(ev_wait(gc.st, e_next, WT_TRANSPOSE_AFTER_BLOCK));
        GEP_TRY(conj_t(gc, g.L, g.W, c1, N, c0, c1));
        GEP_TRY(ev_record(e_w, gc.st));
        w_pending = true;
        return hipSuccess;
    };
    if (ahead) err = next_s21h(0, LB);
    for (int kb = 0; kb < N && err == hipSuccess; kb += LB) {
        const int nb = N - kb < LB ? N - kb : LB;
        const int t0 = kb + nb;
        if (g_sched) {
            SchedOp &op = g_sched->launch(g.st, "k_gep_leaf");
            for (const double2 *X : {(const double2 *)g.L, (const double2 *)g.M,
                                     (const double2 *)g.MH})
                g_sched->add(op, X, kb, kb + nb, kb, kb + nb, true);
            g_sched->add(op, g.info, 0, 1, 0, 1, true);
        } else {
            hipLaunchKernelGGL(k_gep_leaf, dim3(1), dim3(512), 0, g.st, g.L, g.M, g.MH, N, kb, nb,
                               g.info);
            err = hipGetLastError();
        }
        if (err != hipSuccess || t0 >= N) break;
        if (!ahead) {
            if ((err = conj_t(g, g.L, g.W, t0, N, kb, t0)) != hipSuccess) break;  // W = S21^H
            if ((err = mm(g, g.MH, g.W, g.LH, kb, t0, t0, N, kb, t0, MM_PU, OP_STORE)) !=
                hipSuccess)
                break;                                                             // LH21 = M11 S21^H
            if ((err = after_panel(t0, nullptr)) != hipSuccess) break;
            if ((err = conj_t(g, g.LH, g.L, kb, t0, t0, N)) != hipSuccess) break; // L21
            err = mm(g, g.LH, g.LH, g.L, t0, N, t0, N, kb, t0, MM_LOWER, OP_SUB);  // S22 -= L21 L21^H
            continue;
        }
        if ((err = ev_wait(g.st, e_w, WT_PANEL_AFTER_TRANSPOSE)) != hipSuccess) break;   // W = S21^H
        w_pending = false;
        if ((err = mm(g, g.MH, g.W, g.LH, kb, t0, t0, N, kb, t0, MM_PU, OP_STORE)) != hipSuccess)
            break;                                                                 // LH21 = M11 S21^H
        // the hook also gets the lookahead stream's latest event (or null),
        // which orders that stream's pending work before anything it forks
        if ((err = after_panel(t0, look_pending ? e_look : nullptr)) != hipSuccess) break;
        const bool second = ((kb / LB) & 1) != 0;   // second panel of a pair
        const int k0 = second ? kb - LB : kb;        // first contraction row of the update
        const int t1 = N - t0 < LB ? N : t0 + LB;
        const int u1 = second ? std::min(N, t0 + 2 * LB) : t1;   // columns the caller updates
        if ((err = ev_record(e_panel, g.st)) != hipSuccess) break;
        if (second && bulk_pending &&
            (err = ev_wait(g.st, e_bulk, WT_BLOCK_AFTER_BULK)) != hipSuccess)
            break;
        if ((err = ev_wait(ga.st, e_panel, WT_AHEAD_AFTER_PANEL)) != hipSuccess) break;
        if ((err = conj_t(ga, g.LH, g.L, kb, t0, t0, N)) != hipSuccess) break;    // L21
        if (second) {
            if (u1 < N && (err = mm(ga, g.LH, g.LH, g.L, u1, N, u1, N, k0, t0, MM_LOWER,
                                    OP_SUB)) != hipSuccess)
                break;                                                             // the rest
            if ((err = ev_record(e_bulk, ga.st)) != hipSuccess) break;
            bulk_pending = true;
        }
        if ((err = ev_record(e_look, ga.st)) != hipSuccess) break;
        look_pending = true;
        if ((err = mm(g, g.LH, g.LH, g.L, t0, N, t0, u1, k0, t0, MM_MASK, OP_SUB)) != hipSuccess)
            break;                                                                 // next column block(s)
        if (t1 < N) err = next_s21h(t0, t1);
    }
    // join the other streams, also after an error
    if (look_pending) {
        const hipError_t e = ev_wait(g.st, e_look, WT_JOIN_AHEAD);
        if (err == hipSuccess) err = e;
    }
    if (w_pending) {
        const hipError_t e = ev_wait(g.st, e_w, WT_JOIN_TRANSPOSE);
        if (err == hipSuccess) err = e;
    }
    for (hipEvent_t e : {e_panel, e_bulk, e_look, e_next, e_w}) ev_destroy(e);
    return err;
}

// Inverse of the factor, M = L^{-1}, over the recursion tree of [0, N) split
// at multiples of LB (the leaves' inverses are in place): per node [a, b)
// split at m, M21 = -M22 (L21 M11) and MH12 = M21^H. The nodes of one depth
// are independent; each depth, deepest first, runs as two batched launches.
struct Node {
    int a, m, b;
};

void tree(int a, int b, int depth, std::vector<std::vector<Node>> &lv) {
    const int n = b - a;
    if (n <= LB) return;
    const int m = a + (n / 2 + LB - 1) / LB * LB;   // multiple of LB, < b
    if ((int)lv.size() <= depth) lv.resize(depth + 1);
    lv[depth].push_back(Node{a, m, b});
    tree(a, m, depth + 1, lv);
    tree(m, b, depth + 1, lv);
}

// The two products and the transpose of a set of independent nodes.
hipError_t node_w21(const Gep &g, const std::vector<Node> &nodes) {   // W21 = L21 M11
    std::vector<Rect> r;
    for (const Node &n : nodes) r.push_back(Rect{n.m, n.b, n.a, n.m, n.a, n.m});
    return mm_batch(g, g.LH, g.M, g.W, r.data(), (int)r.size(), MM_QL, OP_STORE);
}
hipError_t node_m21(const Gep &g, const std::vector<Node> &nodes) {   // M21 = -M22 W21, MH12
    std::vector<Rect> r;
    for (const Node &n : nodes) r.push_back(Rect{n.m, n.b, n.a, n.m, n.m, n.b});
    GEP_TRY(mm_batch(g, g.MH, g.W, g.M, r.data(), (int)r.size(), MM_PU, OP_NEG));
    r.clear();
    for (const Node &n : nodes) r.push_back(Rect{n.m, n.b, n.a, n.m, 0, 0});
    return conj_t_batch(g, g.M, g.MH, r.data(), (int)r.size());
}

template <class Keep>
hipError_t invert(const Gep &g, const std::vector<std::vector<Node>> &lv, Keep keep) {
    std::vector<Node> nodes;
    for (int d = (int)lv.size() - 1; d >= 0; --d) {
        nodes.clear();
        for (const Node &n : lv[d])
            if (keep(n)) nodes.push_back(n);
        if (nodes.empty()) continue;
        GEP_TRY(node_w21(g, nodes));
        GEP_TRY(node_m21(g, nodes));
    }
    return hipSuccess;
}

size_t padded(size_t bytes) { return (bytes + 255) / 256 * 256; }

// With H = HL + HL^H (HL: lower triangle of H, half its diagonal),
//   Ht = M H M^H = A B^H + B A^H,  A = M HL (lower), B = M,
// so Ht takes WH = A^H = HL^H MH (upper: WH[i][j] sums k in [i, j]) and the
// two-term lower-triangle product Ht = WH^H MH + MH^H WH (k <= j). WH is
// kept in LH, whose lower triangle is zero.

// Below this size the two-term form has too few lower-triangle tiles to fill
// the device, and Ht = V^H MH with V = H MH (N^3/2 + N^3/6 complex
// multiply-adds over full squares of tiles) is faster.
constexpr int GEP_HER2K_MIN_N = 4096;

// V[:, c0:c1) = H MH[:, c0:c1), kept in LH
hipError_t v_cols(const Gep &g, const double2 *H, int c0, int c1) {
    return mm(g, H, g.MH, g.LH, 0, g.N, c0, c1, 0, g.N, MM_QU, OP_STORE);
}

// WH[:, c0:c1) (rows i <= j): the rows above the block (longer contractions)
// and the block's upper triangle in one launch
hipError_t wh_cols(const Gep &g, int c0, int c1) {
    const int N = g.N;
    const Rect r[2] = {{0, c0, c0, c1, 0, N}, {c0, c1, c0, c1, 0, N}};
    const int f[2] = {MM_PL | MM_QU, MM_PL | MM_QU | MM_UPPER};
    return mm_batch(g, g.HL, g.MH, g.LH, r, 2, 0, OP_STORE, nullptr, nullptr, f);
}

// lower triangle of Ht, rows [r0, r1): the triangle (contractions up to
// r1) and then the rows' columns left of it (up to r0) in one launch
hipError_t her2k_rows(const Gep &g, double2 *Ht, int r0, int r1) {
    const int N = g.N;
    const Rect r[2] = {{r0, r1, r0, r1, 0, N}, {r0, r1, 0, r0, 0, N}};
    const int f[2] = {MM_QU | MM_LOWER, MM_QU};
    return mm_batch(g, g.LH, g.MH, Ht, r, 2, 0, OP_STORE, g.MH, g.LH, f);
}

}  // namespace

size_t gep_workspace_bytes(int N) {
    return 5 * padded(16 * (size_t)N * (size_t)N) + 256;   // LH, M, MH, W, HL, info slot
}

hipError_t launch_gep(const double2 *H, const double2 *S, int N, double2 *L, double2 *Ht,
                      int *info, char *ws, hipStream_t st, bool g3) {
    const bool two = N >= GEP_HER2K_MIN_N;   // Ht from WH (two-term product), else from V
    const size_t m = padded(16 * (size_t)N * (size_t)N);
    Gep g;
    g.L = L;
    g.LH = reinterpret_cast<double2 *>(ws);
    g.M = reinterpret_cast<double2 *>(ws + m);
    g.MH = reinterpret_cast<double2 *>(ws + 2 * m);
    g.W = reinterpret_cast<double2 *>(ws + 3 * m);
    g.HL = reinterpret_cast<double2 *>(ws + 4 * m);
    g.N = N;
    g.info = info ? info : reinterpret_cast<int *>(ws + 5 * m);
    g.st = st;
    g.g3 = g3;
    const long long nn = (long long)N * N;
    // Ht's upper triangle by conjugation, Im(diag) = 0
    const auto mirror = [&]() -> hipError_t {
        if (g_sched) {
            g_sched->add(g_sched->launch(st, "k_mirror"), Ht, 0, N, 0, N, true);
            return hipSuccess;
        }
        return launch_mirror1(Ht, N, st);
    };
    if (g_sched) {
        const void *b[SB_COUNT] = {H, S, L, Ht, g.LH, g.M, g.MH, g.W, g.HL, g.info};
        std::copy(b, b + SB_COUNT, g_sched->base);
        SchedOp &op = g_sched->launch(st, "k_gep_init");
        g_sched->add(op, S, 0, N, 0, N, false);
        for (const void *X : {(const void *)L, (const void *)g.M, (const void *)g.MH,
                              (const void *)g.LH})
            g_sched->add(op, X, 0, N, 0, N, true);
        if (two) {
            g_sched->add(op, H, 0, N, 0, N, false);
            g_sched->add(op, g.HL, 0, N, 0, N, true);
        }
        g_sched->add(op, g.info, 0, 1, 0, 1, true);
    } else {
        hipLaunchKernelGGL(k_gep_init, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, st, H, S,
                           L, g.M, g.MH, g.LH, two ? g.HL : nullptr, N);
        GEP_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_gep_info_clear, dim3(1), dim3(1), 0, st, g.info);
        GEP_TRY(hipGetLastError());
    }
    g.cap = 0;
    std::vector<std::vector<Node>> lv;
    tree(0, N, 0, lv);
    const auto all = [](const Node &) { return true; };
    const int np = (N + LB - 1) / LB;
    hipStream_t sb = np >= 8 ? aux_stream(1) : nullptr;
    if (!sb) {
        GEP_TRY(factor(g, [](int, hipEvent_t) { return hipSuccess; }));
        GEP_TRY(invert(g, lv, all));
        if (two) {
            GEP_TRY(wh_cols(g, 0, N));
            GEP_TRY(her2k_rows(g, Ht, 0, N));
        } else {
            GEP_TRY(v_cols(g, H, 0, N));
            GEP_TRY(mm(g, g.LH, g.MH, Ht, 0, N, 0, N, 0, N, MM_QU | MM_LOWER, OP_STORE));  // V^H MH
        }
        return mirror();
    }
    // Once the factorization has passed the top split m (the leaf and the
    // panel product LH21 of the panel ending at m are enqueued), the inverse of the
    // leading block [0, m), the top split's W21 = L21 M11, WH[:, 0:m) and the
    // rows [0, m) of Ht (or V[:, 0:m)) depend on nothing still to come: they run on a second
    // stream, with at most HS_GEP_BG_QUARTERS / 4 of the compute units, beside
    // the rest of the factorization (which no longer touches LH's columns < m).
    const Node top = lv[0][0];
    const int mt = top.m;
    Gep gb = g;
    gb.st = sb;
    gb.cap = (g_sched ? 256 : num_cus()) * HS_GEP_BG_QUARTERS / 4;
    hipEvent_t e_split = nullptr, e_inv = nullptr, e_v = nullptr;
    hipError_t err = ev_create(&e_split);
    if (err == hipSuccess) err = ev_create(&e_inv);
    if (err == hipSuccess) err = ev_create(&e_v);
    bool forked = false;
    const auto left = [mt](const Node &n) { return n.b <= mt; };
    if (err == hipSuccess)
        err = factor(g, [&](int t0, hipEvent_t e_ahead) -> hipError_t {
            if (t0 != mt) return hipSuccess;
            GEP_TRY(ev_record(e_split, st));
            GEP_TRY(ev_wait(sb, e_split, WT_FORK));
            // the previous panel's L21 = LH21^H may still read LH columns
            // >= m - LB on the lookahead stream; V (or WH) overwrites LH's
            // columns < m below
            if (e_ahead) GEP_TRY(ev_wait(sb, e_ahead, WT_FORK_AHEAD));
            forked = true;
            GEP_TRY(invert(gb, lv, left));
            GEP_TRY(node_w21(gb, {top}));   // L21 and M11 of the top split are final too
            GEP_TRY(ev_record(e_inv, sb));
            if (two) {
                GEP_TRY(wh_cols(gb, 0, mt));
                GEP_TRY(her2k_rows(gb, Ht, 0, mt));
            } else {
                GEP_TRY(v_cols(gb, H, 0, mt));
            }
            return ev_record(e_v, sb);
        });
    if (err == hipSuccess) err = invert(g, lv, [mt](const Node &n) { return n.a >= mt; });
    if (err == hipSuccess && forked) err = ev_wait(st, e_inv, WT_END_AFTER_INVERSE);
    if (err == hipSuccess) err = node_m21(g, {top});
    if (err == hipSuccess) err = two ? wh_cols(g, mt, N) : v_cols(g, H, mt, N);
    if (forked) {   // join the second stream even after an error
        const hipError_t e = ev_wait(st, e_v, WT_END_AFTER_BACKGROUND);
        if (err == hipSuccess) err = e;
    }
    if (err == hipSuccess)
        err = two ? her2k_rows(g, Ht, mt, N)
                  : mm(g, g.LH, g.MH, Ht, 0, N, 0, N, 0, N, MM_QU | MM_LOWER, OP_STORE);
    for (hipEvent_t e : {e_split, e_inv, e_v}) ev_destroy(e);
    GEP_TRY(err);
    return mirror();
}

int gep_check_schedule(int N, bool g3, int drop_tag, std::string &report) {
    Sched sc;
    sc.drop_tag = drop_tag;
    // distinct stand-in addresses; nothing is dereferenced or launched
    auto fake = [](uintptr_t a) { return reinterpret_cast<double2 *>(a); };
    char *ws = reinterpret_cast<char *>((uintptr_t)1 << 44);
    g_sched = &sc;
    const hipError_t e = launch_gep(fake((uintptr_t)1 << 40), fake((uintptr_t)2 << 40), N,
                                    fake((uintptr_t)3 << 40), fake((uintptr_t)4 << 40), nullptr, ws,
                                    reinterpret_cast<hipStream_t>((uintptr_t)0x10), g3);
    g_sched = nullptr;
    if (e != hipSuccess) {
        report = "orchestration returned an error";
        return -1;
    }
    return sched_check(sc, N, report);
}

}  // namespace hs
