// Split-precision form of the large reductions (the five stacked products of
// Alg. 1: zher2k, the two zherk of S, the failure-branch zgemm and the HPD
// zherk): FP64 operands are cut into FP16 slices, the
// slice products run on FP16 MFMA with FP32 accumulation, and the slices are
// recombined in FP64. The per-atom Cholesky, the HPD test and the per-atom
// products stay in FP64 (they produce the Z, W operands sliced here).
//
// Slicing (error-free): for each operand column n let e[n] be the exponent
// with max_k max(|Re X[k][n]|, |Im X[k][n]|) < 2^e[n]. The scaled values
// x = X 2^-e lie in (-1, 1) and are written exactly as
//     x = sig_1 2^-b1 + sum_{s=2..NSL} sig_s 2^-(b1 + b (s-1)) + r
// with b1 bits in the first slice and b bits in the others:
// sig_1 = rint(2^b1 x) in [-2^b1, 2^b1], then sig_s = rint(2^b r_{s-1}) in
// [-2^(b-1), 2^(b-1)] (r_s the running remainder, |r_NSL| <=
// 2^-(b1 + b (NSL-1) + 1); every step is exact in FP64). With b1, b <= 10
// every sig_s is an integer that FP16 holds exactly. The weight of a pair
// (s, t) is 2^-(2 b1 + b (s + t - 2)): it depends on s + t only, so pairs of
// one level c = s + t share an accumulator.
//
// Complex products without extra passes: along the contraction index the real
// and imaginary parts are interleaved, P' = (p_re, p_im), Q'_re = (q_re, q_im)
// and Q'_im = (q_im, -q_re), so that Re conj(p) q = P'.Q'_re and
// Im conj(p) q = P'.Q'_im; one FP16 MFMA K-step of 32 then covers 16 complex
// contraction rows. Q'_im is formed from Q'_re in registers.
//
// Accumulation: the slice pairs (s, t) with s + t <= NSL + 1 are summed into
// one FP32 accumulator per level c = s + t and, every FLUSH stages (16
// complex rows each) and at the end of each (P, Q) segment, combined in FP64:
//     acc += 2^(eP[m] + eQ[n] - 2 b1) (L_2 + 2^-b L_3 + 2^-2b L_4 + ...)
// and cleared. Default scheme (b1 = 8, b = 9, NSL = 4, FLUSH = 4, i.e. 64
// rows = 128 real products per pair between flushes):
//   level 2: |sig_1 sig_1| <= 2^16, sum <= 2^7 * 2^16 = 2^23: exact;
//   level 3: two pairs <= 2^8 * 2^8 each, sum <= 2^24: exact;
//   levels 4, 5 (weights 2^-18, 2^-27 relative to level 2) may round, at
//   2^-24 of their own size, i.e. below 2^-42 of the leading terms.
// Products of FP16 integers are exact in FP32 and, within one MFMA, partial
// sums of a level stay below 2^24, so the MFMA's internal order is immaterial.
// Errors left: the remainders (2^-36 of the column maxima), the dropped pairs
// (s + t > 5, at most 2^-37), and FP64 rounding; relative to a typical
// product (entries a few standard deviations below their column maximum)
// about 2^-32.
#include "hs_internal.h"
#include "zmfma_tile.h"

#ifndef HS_SPLIT_NSL
#define HS_SPLIT_NSL 4
#endif
#ifndef HS_SPLIT_BITS1
#define HS_SPLIT_BITS1 8
#endif
#ifndef HS_SPLIT_BITS
#define HS_SPLIT_BITS 9
#endif
#ifndef HS_SPLIT_FLUSH
#define HS_SPLIT_FLUSH 4
#endif
#ifndef HS_SPLIT_WM
#define HS_SPLIT_WM 4
#endif
#ifndef HS_SPLIT_WN
#define HS_SPLIT_WN 2
#endif

namespace hs {

namespace {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int NSL = HS_SPLIT_NSL;      // slices per value
constexpr int SBITS1 = HS_SPLIT_BITS1; // bits of the first slice
constexpr int SBITS = HS_SPLIT_BITS;   // bits of the other slices
constexpr int NLEV = NSL;              // levels c = 2 .. NSL + 1
static_assert(SBITS1 <= 10 && SBITS <= 10, "slices must be integers FP16 holds exactly");

// ---------------------------------------------------------------------------
// Column maxima. A positive double's bit pattern orders like the double, so
// the per-column maximum of |Re|, |Im| is reduced with an integer atomicMax
// (order-independent, hence deterministic) over blocks of 64 columns x 64
// rows; k_zero_u64 clears the maxima first (a kernel, not a memset, so the
// sequence stays valid inside a captured graph).

constexpr int CROWS = 64;   // rows per k_colmax block

__global__ void __launch_bounds__(256) k_zero_u64(unsigned long long *p, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

__device__ __forceinline__ double2 slice_src_row(const SliceSrc &src, int k, int n_g, int n) {
    const double2 *row = src.X;
    if (src.sel && src.sel[k]) row = src.Xalt;
    double2 v = row[(long long)k * n_g + n];
    if (src.rscale) {
        const double w = sqrt(src.rscale[k]);
        v.x *= w;
        v.y *= w;
    }
    return v;
}

__global__ void __launch_bounds__(256)
k_colmax(SliceSrc src, int K, int n_g) {
    __shared__ double red[4][64];
    const int c = threadIdx.x & 63, rg = threadIdx.x >> 6;
    const int n = blockIdx.x * 64 + c;
    const int ncl = n < n_g ? n : n_g - 1;
    const int k0 = blockIdx.y * CROWS;
    double m = 0.0;
#pragma unroll 4
    for (int k = k0 + rg; k < k0 + CROWS; k += 4) {
        if (k < K) {
            const double2 v = slice_src_row(src, k, n_g, ncl);
            m = fmax(m, fmax(fabs(v.x), fabs(v.y)));
        }
    }
    red[rg][c] = m;
    __syncthreads();
    if (rg == 0 && n < n_g) {
        m = fmax(fmax(red[0][c], red[1][c]), fmax(red[2][c], red[3][c]));
        atomicMax(src.mx + n, (unsigned long long)__double_as_longlong(m));
    }
}

// exponent e with column max < 2^e (0 for an all-zero column)
__device__ __forceinline__ int col_exp(const unsigned long long *mx, int n) {
    const double m = __longlong_as_double((long long)mx[n]);
    int e = 0;
    if (m > 0.0) frexp(m, &e);
    return e;
}

// ---------------------------------------------------------------------------
// Slices. One thread per (group of 4 complex rows, column): 8 interleaved
// real values -> NSL slices of 8 halves, written to S[s][g][n][0..7].

__global__ void __launch_bounds__(256)
k_slice(SliceSrc src, int K, int n_g, int groups) {
    const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
    const int n = (int)(idx % n_g);
    const int g = (int)(idx / n_g);
    if (g >= groups) return;
    const double sc = ldexp(1.0, -col_exp(src.mx, n));
    double x[8];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int k = 4 * g + q;
        double2 v = {0.0, 0.0};
        if (k < K) v = slice_src_row(src, k, n_g, n);
        x[2 * q] = v.x * sc;
        x[2 * q + 1] = v.y * sc;
    }
    const long long plane = (long long)groups * n_g * 8;   // halves per slice
    _Float16 *out = src.S + ((long long)g * n_g + n) * 8;
#pragma unroll
    for (int s = 0; s < NSL; ++s) {
        h8 h;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const double t = x[j] * (double)(1 << (s == 0 ? SBITS1 : SBITS));
            const double sig = rint(t);
            x[j] = t - sig;
            h[j] = (_Float16)sig;
        }
        *reinterpret_cast<h8 *>(out + s * plane) = h;
    }
}

// ---------------------------------------------------------------------------
// Slice GEMM over lower-triangle tiles of H and S.

constexpr int SBM = 64;                 // tile rows (g')
constexpr int SBN = 64;                 // tile cols (g)
constexpr int SWM = HS_SPLIT_WM, SWN = HS_SPLIT_WN;
constexpr int SNT = 64 * SWM * SWN;
constexpr int SWTM = SBM / SWM, SWTN = SBN / SWN;   // wave tile
constexpr int STM = SWTM / 16;          // 16-row blocks per wave
constexpr int STN = SWTN / 16;          // 16-col blocks per wave
constexpr int SGRP = 4;                 // groups (of 4 complex rows) per stage = 16 rows
constexpr int FLUSH = HS_SPLIT_FLUSH;   // stages per flush
// exactness of the two leading levels between flushes (2 * 16 * FLUSH real
// products per pair): level 2 one pair of |sig_1| <= 2^b1, level 3 two
// pairs of |sig_1| <= 2^b1 times |sig_2| <= 2^(b-1)
constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x / 2); }
static_assert((32 * FLUSH) == (1 << ilog2(32 * FLUSH)), "FLUSH is a power of two");
static_assert(2 * SBITS1 + ilog2(32 * FLUSH) <= 24, "level 2 exact in FP32");
static_assert(SBITS1 + SBITS - 1 + 1 + ilog2(32 * FLUSH) <= 24, "level 3 exact in FP32");
constexpr int SBAND = 8;
// LDS per operand per stage: NSL slices x SGRP groups x 64 columns x 16 B
constexpr int LDS_OP = NSL * SGRP * 64;   // in units of 16 B
constexpr int LD_ITEMS = (LDS_OP + SNT - 1) / SNT;
static_assert(SBM == 64 && SBN == 64, "loader assumes 64-column tiles");
static_assert(SWTM % 16 == 0 && SWTN % 16 == 0, "wave tiling");

struct SplitSeg {
    const _Float16 *P, *Q;                  // slices [NSL][groups][n_g][8]
    const unsigned long long *mP, *mQ;      // column maxima (bit patterns) [n_g]
};

struct SplitArgs {
    SplitSeg h[3];
    SplitSeg s[2];
    double2 *H, *S;
    int n_g, groups;         // groups = K padded to 16, over 4
    int nt, ntri, ntri8;
};

__device__ __forceinline__ void sband_tile(int t, int nt, int &ti, int &tj) {
    int c0 = 0;
    for (;;) {
        const int m = nt - c0;
        if (m <= 0) {
            ti = tj = -1;
            return;
        }
        const int w = m < SBAND ? m : SBAND;
        const int tri = w * (w + 1) / 2;
        const int cnt = tri + (m - w) * w;
        if (t < cnt) {
            if (t < tri) {
                int r = 0;
                while ((r + 1) * (r + 2) / 2 <= t) ++r;
                ti = c0 + r;
                tj = c0 + (t - r * (r + 1) / 2);
            } else {
                const int u = t - tri;
                ti = c0 + w + u / w;
                tj = c0 + u % w;
            }
            return;
        }
        t -= cnt;
        c0 += SBAND;
    }
}

struct Acc64 {
    double re[STM][STN][4];
    double im[STM][STN][4];
};

// One (P, Q) segment into the FP64 accumulators. The segment is taken by
// value: a reference into the by-value kernel argument would move the whole
// argument block into scratch memory.
__device__ __forceinline__ void split_segment(const SplitSeg sg, int n_g, int groups, int m0,
                                              int n0, Acc64 &acc, uint4 *lds) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave % SWM, wn = wave / SWM;

    // loader: NSL*SGRP*64 16-byte items per operand per stage, item
    // id -> (slice, group, column) = (id / 256, (id / 64) % 4, id % 64); each
    // thread moves up to LD_ITEMS of them (indices clamped, extra ones unused)
    const int col = tid & 63;
    const int pm = m0 + col, qn = n0 + col;
    const bool pok = pm < n_g, qok = qn < n_g;
    const int pmc = pok ? pm : n_g - 1, qnc = qok ? qn : n_g - 1;
    const long long plane = (long long)groups * n_g;   // 16-byte items per slice
    const uint4 *Pg = reinterpret_cast<const uint4 *>(sg.P);
    const uint4 *Qg = reinterpret_cast<const uint4 *>(sg.Q);
    uint4 rp[LD_ITEMS], rq[LD_ITEMS];
    const int nstage = groups / SGRP;
    auto fetch = [&](int st) {
        const int st_c = st < nstage ? st : nstage - 1;   // clamped (unused past the end)
#pragma unroll
        for (int j = 0; j < LD_ITEMS; ++j) {
            const int idv = tid + j * SNT;
            const int id = idv < LDS_OP ? idv : LDS_OP - 1;
            const int s = id >> 8, gi = (id >> 6) & 3;
            const long long g = (long long)st_c * SGRP + gi;
            rp[j] = Pg[s * plane + g * n_g + pmc];
            rq[j] = Qg[s * plane + g * n_g + qnc];
        }
    };
    // per-component selects (an aggregate select becomes an address select
    // that sends the staging registers to scratch)
    auto stash = [&](int buf) {
        uint4 *lp = lds + buf * 2 * LDS_OP;
        uint4 *lq = lp + LDS_OP;
#pragma unroll
        for (int j = 0; j < LD_ITEMS; ++j) {
            const int id = tid + j * SNT;
            if (id >= LDS_OP) continue;
            uint4 a, b;
            a.x = pok ? rp[j].x : 0u;
            a.y = pok ? rp[j].y : 0u;
            a.z = pok ? rp[j].z : 0u;
            a.w = pok ? rp[j].w : 0u;
            b.x = qok ? rq[j].x : 0u;
            b.y = qok ? rq[j].y : 0u;
            b.z = qok ? rq[j].z : 0u;
            b.w = qok ? rq[j].w : 0u;
            lp[id] = a;
            lq[id] = b;
        }
    };

    // column scales of this lane's accumulator rows (g') and columns (g),
    // with the 2^-2b1 weight of the first level folded in
    double sP[STM][4], sQ[STN];
#pragma unroll
    for (int i = 0; i < STM; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int m = m0 + wm * SWTM + i * 16 + 4 * (lane >> 4) + v;
            sP[i][v] = ldexp(1.0, col_exp(sg.mP, m < n_g ? m : n_g - 1) - 2 * SBITS1);
        }
#pragma unroll
    for (int j = 0; j < STN; ++j) {
        const int n = n0 + wn * SWTN + j * 16 + (lane & 15);
        sQ[j] = ldexp(1.0, col_exp(sg.mQ, n < n_g ? n : n_g - 1));
    }

    f4 lre[STM][STN][NLEV], lim[STM][STN][NLEV];
    auto clear = [&]() {
#pragma unroll
        for (int i = 0; i < STM; ++i)
#pragma unroll
            for (int j = 0; j < STN; ++j)
#pragma unroll
                for (int c = 0; c < NLEV; ++c) {
                    lre[i][j][c] = f4{0.f, 0.f, 0.f, 0.f};
                    lim[i][j][c] = f4{0.f, 0.f, 0.f, 0.f};
                }
    };
    constexpr double STEP = 1.0 / (double)(1 << SBITS);
    auto flush = [&]() {
#pragma unroll
        for (int i = 0; i < STM; ++i)
#pragma unroll
            for (int j = 0; j < STN; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const double w = sP[i][v] * sQ[j];
                    double tr = (double)lre[i][j][NLEV - 1][v];
                    double ti = (double)lim[i][j][NLEV - 1][v];
#pragma unroll
                    for (int c = NLEV - 2; c >= 0; --c) {
                        tr = fma(tr, STEP, (double)lre[i][j][c][v]);
                        ti = fma(ti, STEP, (double)lim[i][j][c][v]);
                    }
                    acc.re[i][j][v] = fma(tr, w, acc.re[i][j][v]);
                    acc.im[i][j][v] = fma(ti, w, acc.im[i][j][v]);
                }
        clear();
    };

    clear();
    if (nstage == 0) return;
    fetch(0);
    stash(0);
    __syncthreads();

    const int lg = lane >> 4, lc = lane & 15;
    for (int st = 0; st < nstage; ++st) {
        fetch(st + 1);
        const uint4 *lp = lds + (st & 1) * 2 * LDS_OP;
        const uint4 *lq = lp + LDS_OP;
        h8 a[STM][NSL], bre[STN][NSL];
#pragma unroll
        for (int s = 0; s < NSL; ++s) {
#pragma unroll
            for (int i = 0; i < STM; ++i) {
                const uint4 u = lp[(s * SGRP + lg) * 64 + wm * SWTM + i * 16 + lc];
                a[i][s] = __builtin_bit_cast(h8, u);
            }
#pragma unroll
            for (int j = 0; j < STN; ++j) {
                const uint4 u = lq[(s * SGRP + lg) * 64 + wn * SWTN + j * 16 + lc];
                bre[j][s] = __builtin_bit_cast(h8, u);
            }
        }
#pragma unroll
        for (int t = 0; t < NSL; ++t)
#pragma unroll
            for (int j = 0; j < STN; ++j) {
                const h8 b = bre[j][t];
                h8 bi;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    bi[2 * q] = b[2 * q + 1];
                    bi[2 * q + 1] = -b[2 * q];
                }
#pragma unroll
                for (int s = 0; s + t < NLEV; ++s) {   // levels (s+1)+(t+1) <= NSL+1
                    const int c = s + t;
#pragma unroll
                    for (int i = 0; i < STM; ++i) {
                        lre[i][j][c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[i][s], b, lre[i][j][c], 0, 0, 0);
                        lim[i][j][c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[i][s], bi, lim[i][j][c], 0, 0, 0);
                    }
                }
            }
        stash((st + 1) & 1);
        if ((st + 1) % FLUSH == 0 || st + 1 == nstage) flush();
        __syncthreads();
    }
}

__global__ void __launch_bounds__(SNT)
k_split_reduce(SplitArgs args) {
    __shared__ uint4 lds[2 * 2 * LDS_OP];   // 2 buffers x (P, Q)

    int b = blockIdx.x;
    const bool isH = b < args.ntri8;
    if (!isH) b -= args.ntri8;
    const int per_xcd = args.ntri8 / 8;
    const int t = (b % 8) * per_xcd + b / 8;
    if (t >= args.ntri) return;
    int ti, tj;
    sband_tile(t, args.nt, ti, tj);
    if (ti < 0) return;
    const int m0 = ti * SBM, n0 = tj * SBN;
    const int n_g = args.n_g;

    Acc64 acc;
#pragma unroll
    for (int i = 0; i < STM; ++i)
#pragma unroll
        for (int j = 0; j < STN; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc.re[i][j][v] = acc.im[i][j][v] = 0.0;

    if (isH) {
        const SplitSeg h0 = args.h[0], h1 = args.h[1], h2 = args.h[2];
        split_segment(h0, n_g, args.groups, m0, n0, acc, lds);
        split_segment(h1, n_g, args.groups, m0, n0, acc, lds);
        split_segment(h2, n_g, args.groups, m0, n0, acc, lds);
    } else {
        const SplitSeg s0 = args.s[0], s1 = args.s[1];
        split_segment(s0, n_g, args.groups, m0, n0, acc, lds);
        split_segment(s1, n_g, args.groups, m0, n0, acc, lds);
    }

    double2 *out = isH ? args.H : args.S;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave % SWM, wn = wave / SWM;
#pragma unroll
    for (int j = 0; j < STN; ++j) {
        const int g = n0 + wn * SWTN + j * 16 + (lane & 15);
#pragma unroll
        for (int i = 0; i < STM; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gp = m0 + wm * SWTM + i * 16 + 4 * (lane >> 4) + v;
                if (gp < n_g && g <= gp)
                    out[(long long)gp * n_g + g] = double2{acc.re[i][j][v], acc.im[i][j][v]};
            }
    }
}

}  // namespace

size_t split_slice_bytes(int K, int n_g) {
    const long long groups = (long long)((K + 15) / 16) * 4;
    return (size_t)NSL * groups * n_g * 16;
}

hipError_t launch_slice(const SliceSrc &src, int K, int n_g, hipStream_t st) {
    const int groups = (K + 15) / 16 * 4;
    hipLaunchKernelGGL(k_zero_u64, dim3((n_g + 255) / 256), dim3(256), 0, st, src.mx, n_g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_colmax, dim3((n_g + 63) / 64, (K + CROWS - 1) / CROWS), dim3(256), 0, st,
                       src, K, n_g);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const long long items = (long long)groups * n_g;
    hipLaunchKernelGGL(k_slice, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, st, src, K,
                       n_g, groups);
    return hipGetLastError();
}

hipError_t launch_split_reduce(int K, int n_g, const SliceView (&hseg)[3][2],
                               const SliceView (&sseg)[2][2], double2 *H, double2 *S,
                               hipStream_t st) {
    SplitArgs a;
    for (int i = 0; i < 3; ++i)
        a.h[i] = SplitSeg{hseg[i][0].S, hseg[i][1].S, hseg[i][0].mx, hseg[i][1].mx};
    for (int i = 0; i < 2; ++i)
        a.s[i] = SplitSeg{sseg[i][0].S, sseg[i][1].S, sseg[i][0].mx, sseg[i][1].mx};
    a.H = H;
    a.S = S;
    a.n_g = n_g;
    a.groups = (K + 15) / 16 * 4;
    a.nt = (n_g + SBM - 1) / SBM;
    a.ntri = a.nt * (a.nt + 1) / 2;
    a.ntri8 = (a.ntri + 7) / 8 * 8;
    hipLaunchKernelGGL(k_split_reduce, dim3(2 * a.ntri8), dim3(SNT), 0, st, a);
    return hipGetLastError();
}

}  // namespace hs
