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
#include "split_common.h"
#include "zmfma_tile.h"

namespace hs {

namespace {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 bh8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int NSL = 4;                 // slices per value
constexpr int SBITS1 = 8;              // bits of the first slice
constexpr int SBITS = 9;               // bits of the other slices
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

// ---------------------------------------------------------------------------
// Slices. One thread per (group of 4 complex rows, column): 8 interleaved
// real values -> NSL slices of 8 halves, written to S[s][g][n][0..7].

// BF: the slices are written as BF16 instead of FP16. Every slice is an
// integer of magnitude <= 256, which both formats hold exactly (BF16 has 8
// significant bits), so the two forms carry the same values and the
// reduction's FP32 sums of their exact products are the same numbers.
template <bool BF>
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
        unsigned short b[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const double t = x[j] * (double)(1 << (s == 0 ? SBITS1 : SBITS));
            const double sig = rint(t);
            x[j] = t - sig;
            h[j] = (_Float16)sig;
            // BF16 of an integer of at most 9 bits: the float's upper half, exactly
            b[j] = (unsigned short)(__builtin_bit_cast(unsigned, (float)sig) >> 16);
        }
        if constexpr (BF) {
            uint4 w;
            w.x = b[0] | ((unsigned)b[1] << 16);
            w.y = b[2] | ((unsigned)b[3] << 16);
            w.z = b[4] | ((unsigned)b[5] << 16);
            w.w = b[6] | ((unsigned)b[7] << 16);
            *reinterpret_cast<uint4 *>(out + s * plane) = w;
        } else {
            *reinterpret_cast<h8 *>(out + s * plane) = h;
        }
    }
}

// ---------------------------------------------------------------------------
// Slice GEMM over lower-triangle tiles of H and S.

constexpr int SBM = 64;                 // tile rows (g')
constexpr int SBN = 64;                 // tile cols (g)
constexpr int SWM = 2, SWN = 4;         // waves
constexpr int SNT = 64 * SWM * SWN;
constexpr int SWTM = SBM / SWM, SWTN = SBN / SWN;   // wave tile
constexpr int STM = SWTM / 16;          // 16-row blocks per wave
constexpr int STN = SWTN / 16;          // 16-col blocks per wave
constexpr int SGRP = 4;                 // groups (of 4 complex rows) per stage = 16 rows
constexpr int FLUSH = 4;                // stages per flush
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

struct Acc64 {
    double re[STM][STN][4];
    double im[STM][STN][4];
};

// One (P, Q) segment into the FP64 accumulators (BF: BF16 slices on BF16
// MFMA). The segment is taken by
// value: a reference into the by-value kernel argument would move the whole
// argument block into scratch memory.
template <bool BF>
__device__ __forceinline__ void split_segment(const SplitSeg sg, int n_g, int groups, int m0,
                                              int n0, Acc64 &acc, uint4 *lds) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave % SWM, wn = wave / SWM;

    const long long plane = (long long)groups * n_g;   // 16-byte items per slice
    const int nstage = groups / SGRP;
    // direct global -> LDS loads, 64 columns each: wave w loads group w % 4
    // of every slice of operand w / 4 (P for waves 0-3, Q for 4-7); columns
    // past the edge read the last column (they only feed outputs past N_G)
    static_assert(SNT == 512 && SGRP == 4, "direct loader assumes 8 waves, 4 groups");
    const int grp_w = wave % SGRP, op_w = wave / SGRP;
    int ldc = (op_w == 0 ? m0 : n0) + lane;
    ldc = ldc < n_g ? ldc : n_g - 1;
    const unsigned ldvo = (unsigned)ldc * 16u;
    const uint4 *ldrows = reinterpret_cast<const uint4 *>(op_w == 0 ? sg.P : sg.Q);
    auto issue = [&](uint4 *buf, int st) __attribute__((always_inline)) {
        const uint4 *rows = ldrows + (long long)(st * SGRP + grp_w) * n_g;
        uint4 *dst = buf + op_w * LDS_OP + grp_w * 64;
#pragma unroll
        for (int s = 0; s < NSL; ++s)
            __builtin_amdgcn_global_load_lds(
                reinterpret_cast<const uint4 *>(reinterpret_cast<const char *>(rows + s * plane) + ldvo),
                dst + s * SGRP * 64, 16, 0, 0);
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

    const int lg = lane >> 4, lc = lane & 15;
    // slice products of one stage from LDS (P slices at lp, Q slices at lq)
    auto compute = [&](const uint4 *lp, const uint4 *lq) __attribute__((always_inline)) {
        uint4 a[STM][NSL], bre[STN][NSL];
#pragma unroll
        for (int s = 0; s < NSL; ++s) {
#pragma unroll
            for (int i = 0; i < STM; ++i) a[i][s] = lp[(s * SGRP + lg) * 64 + wm * SWTM + i * 16 + lc];
#pragma unroll
            for (int j = 0; j < STN; ++j) bre[j][s] = lq[(s * SGRP + lg) * 64 + wn * SWTN + j * 16 + lc];
        }
#pragma unroll
        for (int t = 0; t < NSL; ++t)
#pragma unroll
            for (int j = 0; j < STN; ++j) {
                const uint4 b = bre[j][t];
                uint4 bi;
                if constexpr (BF) {
                    // (re, im) half pairs -> (im, -re): swap the halves of each
                    // word, then flip the sign bit of the new high half
                    auto im_word = [](unsigned w) { return ((w >> 16) | (w << 16)) ^ 0x80000000u; };
                    bi = uint4{im_word(b.x), im_word(b.y), im_word(b.z), im_word(b.w)};
                } else {
                    const h8 bh = __builtin_bit_cast(h8, b);
                    h8 bih;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        bih[2 * q] = bh[2 * q + 1];
                        bih[2 * q + 1] = -bh[2 * q];
                    }
                    bi = __builtin_bit_cast(uint4, bih);
                }
#pragma unroll
                for (int s = 0; s + t < NLEV; ++s) {   // levels (s+1)+(t+1) <= NSL+1
                    const int c = s + t;
#pragma unroll
                    for (int i = 0; i < STM; ++i) {
                        if constexpr (BF) {
                            const bh8 x = __builtin_bit_cast(bh8, a[i][s]);
                            lre[i][j][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                x, __builtin_bit_cast(bh8, b), lre[i][j][c], 0, 0, 0);
                            lim[i][j][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                x, __builtin_bit_cast(bh8, bi), lim[i][j][c], 0, 0, 0);
                        } else {
                            const h8 x = __builtin_bit_cast(h8, a[i][s]);
                            lre[i][j][c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                                x, __builtin_bit_cast(h8, b), lre[i][j][c], 0, 0, 0);
                            lim[i][j][c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                                x, __builtin_bit_cast(h8, bi), lim[i][j][c], 0, 0, 0);
                        }
                    }
                }
            }
    };

    clear();
    if (nstage == 0) return;
    issue(lds, 0);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    for (int st = 0; st < nstage; ++st) {
        // the buffer being computed and the one being loaded are distinct:
        // saying so (restrict) keeps the compiler from waiting for the direct
        // loads before the stage's LDS reads
        auto stage = [&](const uint4 *__restrict__ cur, uint4 *__restrict__ nxt)
                         __attribute__((always_inline)) {
            if (st + 1 < nstage) issue(nxt, st + 1);
            compute(cur, cur + LDS_OP);
        };
        stage(lds + (st & 1) * 2 * LDS_OP, lds + ((st + 1) & 1) * 2 * LDS_OP);
        if ((st + 1) % FLUSH == 0 || st + 1 == nstage) flush();
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
    }
}

template <bool BF>
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
    sband_tile(t, args.nt, ti, tj, SBAND);
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
        split_segment<BF>(h0, n_g, args.groups, m0, n0, acc, lds);
        split_segment<BF>(h1, n_g, args.groups, m0, n0, acc, lds);
        split_segment<BF>(h2, n_g, args.groups, m0, n0, acc, lds);
    } else {
        const SplitSeg s0 = args.s[0], s1 = args.s[1];
        split_segment<BF>(s0, n_g, args.groups, m0, n0, acc, lds);
        split_segment<BF>(s1, n_g, args.groups, m0, n0, acc, lds);
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


// ===========================================================================
// INT8 form (HS_SPLIT_I8). Same scaling and complex interleaving, integer
// slices of 7 bits on V_MFMA_I32_16X16X64_I8 with exact INT32 accumulation.
//
// Slicing: with e[n] such that max |X[.][n]| * 128/127 < 2^e[n], x = X 2^-e
// lies in (-127/128, 127/128) and
//     x = sum_{s=1..5} sig_s 128^-s + r,   sig_1 = rint(128 x) in [-127, 127],
//     sig_s = rint(128 r_{s-1}) in [-64, 64] (s >= 2),  |r| <= 2^-36,
// every value an int8. A pair (s, t) weighs 128^-(s + t); the 15 pairs with
// s + t <= 6 go into five INT32 level accumulators (c = 2..6). A level sums
// at most 5 pairs of |sig sig'| <= 127 * 64 or 64 * 64 (level 2: 127^2), at
// most 28544 < 2^15 per real product, so a level stays exact for 2^16 real
// products: the accumulators are combined in FP64 (Horner, scaled by
// 2^(eP + eQ - 14)) only at the end of each (P, Q) segment and every 32768
// complex rows, into FP64 accumulators held in registers across the
// segments of the output tile (a fixed order: deterministic); each output
// element is stored to memory once, after its last segment. No FP64 work
// sits in the K loop.
//
// Errors left: remainders (2^-36 of the column maxima on each side),
// dropped pairs (s + t = 7: four pairs of |sig sig'| <= 2^12 at 2^-49, i.e.
// 2^-35), FP64 rounding.
//
// Tiles: 64 x 64, 8 waves (2 x 4 waves of 32 x 16). A stage is 32 complex
// rows (one MFMA K step of 64 int8). Operand slices go straight from global
// memory to LDS (16-byte direct loads of 64 columns; 40 per stage) through
// two 40 KiB LDS buffers (the next stage loads while the current one is
// multiplied), so no staging registers are needed.

typedef int i4 __attribute__((ext_vector_type(4)));

constexpr int NSL8 = 5;                  // slices per value
constexpr int NLEV8 = 5;                 // levels c = 2 .. 6
constexpr int B8 = 64;                   // tile rows (g') and columns (g)
constexpr int W8M = 2, W8N = 4;          // waves
constexpr int NT8 = 64 * W8M * W8N;
constexpr int T8M = B8 / W8M / 16, T8N = B8 / W8N / 16;   // 16x16 blocks per wave
constexpr int GRP8 = 4;                  // groups of 8 complex rows per stage = 32 rows
constexpr int OP8_ITEMS = NSL8 * GRP8 * B8;   // 16-byte items per operand and stage
constexpr int BUF8 = 2 * OP8_ITEMS;
constexpr int FLUSH8 = 1024;                  // stages (32768 complex rows) per flush
constexpr int BAND8 = 8;
static_assert((long long)FLUSH8 * 64 * 28544 < (1LL << 31), "levels exact in INT32");

// exponent e with column max * 128/127 < 2^e (0 for an all-zero column)
__device__ __forceinline__ int col_exp8(const unsigned long long *mx, int n) {
    const double m = __longlong_as_double((long long)mx[n]);
    int e = 0;
    if (m > 0.0) frexp(m * (128.0 / 127.0), &e);
    return e;
}

// One thread per (group of 8 complex rows, column): 16 interleaved real
// values -> 5 slices of 16 int8, written to S8[s][g][n][0..15].
__global__ void __launch_bounds__(256)
k_slice8(SliceSrc src, int K, int n_g, int groups) {
    const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
    const int n = (int)(idx % n_g);
    const int g = (int)(idx / n_g);
    if (g >= groups) return;
    const double sc = ldexp(1.0, -col_exp8(src.mx, n));
    double x[16];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int k = 8 * g + q;
        double2 v = {0.0, 0.0};
        if (k < K) v = slice_src_row(src, k, n_g, n);
        x[2 * q] = v.x * sc;
        x[2 * q + 1] = v.y * sc;
    }
    const long long plane = (long long)groups * n_g;   // 16-byte items per slice
    uint4 *out = reinterpret_cast<uint4 *>(src.S) + (long long)g * n_g + n;
#pragma unroll
    for (int s = 0; s < NSL8; ++s) {
        unsigned w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const double t = x[j] * 128.0;
            double sig = rint(t);
            sig = fmin(fmax(sig, -127.0), 127.0);
            x[j] = t - sig;
            w[j >> 2] |= ((unsigned)(int)sig & 0xffu) << (8 * (j & 3));
        }
        out[s * plane] = uint4{w[0], w[1], w[2], w[3]};
    }
}

struct Split8Seg {
    const uint4 *P, *Q;                     // slices [5][groups][n_g] x 16 B
    const unsigned long long *mP, *mQ;      // column maxima [n_g]
};

struct Split8Args {
    Split8Seg h[3];
    Split8Seg s[2];
    double2 *H, *S;
    int n_g, groups;          // groups of 8 complex rows, a multiple of GRP8
    int nt, ntri, ntri8;
};

// FP64 sums of a wave's outputs across the segments of its tile.
struct Acc8 {
    double re[T8M][T8N][4];
    double im[T8M][T8N][4];
};

// One (P, Q) segment into the FP64 accumulators. first: the segment's first
// flush writes instead of adding. The segment is taken by value for the
// same reason as split_segment.
__device__ __forceinline__ void split8_segment(const Split8Seg sg, int n_g, int groups, int m0,
                                               int n0, bool first, Acc8 &acc, uint4 *bufs0,
                                               uint4 *bufs1) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave % W8M, wn = wave / W8M;
    const long long plane = (long long)groups * n_g;
    const int nstage = groups / GRP8;

    // direct loads of stage st into buf, 64 columns each (40 loads): wave w
    // loads group w % 4 of every slice of operand w / 4 (P for waves 0-3, Q
    // for 4-7); columns past the edge read the last column (they only feed
    // outputs past N_G, which are not stored)
    static_assert(NT8 == 512, "the loader assumes 8 waves");
    const int grp_w = wave % GRP8;
    const int op_w = wave / GRP8;
    int ldc = (op_w == 0 ? m0 : n0) + lane;
    ldc = ldc < n_g ? ldc : n_g - 1;
    // per-lane byte offset (32-bit) from wave-uniform row bases: the loads
    // then take the scalar-base form and need no 64-bit address registers
    const unsigned ldvo = (unsigned)ldc * 16u;
    const uint4 *ldrows = op_w == 0 ? sg.P : sg.Q;
    auto issue = [&](uint4 *buf, int st) __attribute__((always_inline)) {
        const uint4 *rows = ldrows + (long long)(st * GRP8 + grp_w) * n_g;
        uint4 *dst = buf + op_w * OP8_ITEMS + grp_w * B8;
#pragma unroll
        for (int s = 0; s < NSL8; ++s)
            __builtin_amdgcn_global_load_lds(
                reinterpret_cast<const uint4 *>(reinterpret_cast<const char *>(rows + s * plane) + ldvo),
                dst + s * GRP8 * B8, 16, 0, 0);
    };

    i4 lre[T8M][T8N][NLEV8], lim[T8M][T8N][NLEV8];
    auto clear = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < T8M; ++i)
#pragma unroll
            for (int j = 0; j < T8N; ++j)
#pragma unroll
                for (int c = 0; c < NLEV8; ++c) {
                    lre[i][j][c] = i4{0, 0, 0, 0};
                    lim[i][j][c] = i4{0, 0, 0, 0};
                }
    };
    const int lg = lane >> 4, lc = lane & 15;
    auto compute = [&](const uint4 *buf) __attribute__((always_inline)) {
        const uint4 *lp = buf;
        const uint4 *lq = buf + OP8_ITEMS;
        i4 a[T8M][NSL8];
#pragma unroll
        for (int s = 0; s < NSL8; ++s)
#pragma unroll
            for (int i = 0; i < T8M; ++i)
                a[i][s] = __builtin_bit_cast(i4, lp[(s * GRP8 + lg) * B8 + wm * (B8 / W8M) + i * 16 + lc]);
#pragma unroll
        for (int t = 0; t < NSL8; ++t)
#pragma unroll
            for (int j = 0; j < T8N; ++j) {
                // one Q fragment (and its Im form) live at a time: otherwise
                // the scheduler hoists all of them and the accumulators spill
                __builtin_amdgcn_sched_barrier(0);
                const uint4 u = lq[(t * GRP8 + lg) * B8 + wn * (B8 / W8N) + j * 16 + lc];
                const i4 b = __builtin_bit_cast(i4, u);
                const i4 bi = i4{(int)im_pairs(u.x), (int)im_pairs(u.y), (int)im_pairs(u.z),
                                 (int)im_pairs(u.w)};
#pragma unroll
                for (int s = 0; s + t < NLEV8; ++s) {   // levels (s+1)+(t+1) <= 6
                    const int c = s + t;
#pragma unroll
                    for (int i = 0; i < T8M; ++i) {
                        lre[i][j][c] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[i][s], b, lre[i][j][c], 0, 0, 0);
                        lim[i][j][c] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[i][s], bi, lim[i][j][c], 0, 0, 0);
                    }
                }
            }
    };
    // levels -> FP64, scaled, into the accumulator tile
    auto flush = [&](bool write) __attribute__((always_inline)) {
#pragma unroll
        for (int j = 0; j < T8N; ++j) {
            const int c = wn * (B8 / W8N) + j * 16 + lc;
            const int g = n0 + c;
            const int eq = col_exp8(sg.mQ, g < n_g ? g : n_g - 1);
#pragma unroll
            for (int i = 0; i < T8M; ++i)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = wm * (B8 / W8M) + i * 16 + 4 * lg + v;
                    const int gp = m0 + r;
                    const double w = ldexp(1.0, col_exp8(sg.mP, gp < n_g ? gp : n_g - 1) + eq - 14);
                    double tr = (double)lre[i][j][NLEV8 - 1][v];
                    double ti = (double)lim[i][j][NLEV8 - 1][v];
#pragma unroll
                    for (int lv = NLEV8 - 2; lv >= 0; --lv) {
                        tr = fma(tr, 1.0 / 128.0, (double)lre[i][j][lv][v]);
                        ti = fma(ti, 1.0 / 128.0, (double)lim[i][j][lv][v]);
                    }
                    if (write) {
                        acc.re[i][j][v] = tr * w;
                        acc.im[i][j][v] = ti * w;
                    } else {
                        acc.re[i][j][v] += tr * w;
                        acc.im[i][j][v] += ti * w;
                    }
                }
        }
        clear();
    };

    clear();
    if (nstage == 0) return;
    issue(bufs0, 0);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    for (int c0 = 0; c0 < nstage; c0 += FLUSH8) {
        const int c1 = nstage < c0 + FLUSH8 ? nstage : c0 + FLUSH8;
        for (int st = c0; st < c1; ++st) {
            // the buffer being computed and the one being loaded are
            // distinct: saying so (restrict) keeps the compiler from waiting
            // for the direct loads before every LDS read of the stage
            auto stage = [&](const uint4 *__restrict__ cur, uint4 *__restrict__ nxt)
                             __attribute__((always_inline)) {
                if (st + 1 < nstage) issue(nxt, st + 1);
                compute(cur);
            };
            stage((st & 1) ? bufs1 : bufs0, (st & 1) ? bufs0 : bufs1);
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            __syncthreads();
        }
        flush(first);
        first = false;
    }
}

__global__ void __launch_bounds__(NT8)
k_split8_reduce(Split8Args args) {
    __shared__ uint4 bufA[BUF8];
    __shared__ uint4 bufB[BUF8];

    int b = blockIdx.x;
    const bool isH = b < args.ntri8;
    if (!isH) b -= args.ntri8;
    const int per_xcd = args.ntri8 / 8;
    const int t = (b % 8) * per_xcd + b / 8;
    if (t >= args.ntri) return;
    int ti, tj;
    sband_tile(t, args.nt, ti, tj, BAND8);
    if (ti < 0) return;
    const int n_g = args.n_g;
    const int m0 = ti * B8, n0 = tj * B8;

    Acc8 acc;
    if (isH) {
        const Split8Seg h0 = args.h[0], h1 = args.h[1], h2 = args.h[2];
        split8_segment(h0, n_g, args.groups, m0, n0, true, acc, bufA, bufB);
        split8_segment(h1, n_g, args.groups, m0, n0, false, acc, bufA, bufB);
        split8_segment(h2, n_g, args.groups, m0, n0, false, acc, bufA, bufB);
    } else {
        const Split8Seg s0 = args.s[0], s1 = args.s[1];
        split8_segment(s0, n_g, args.groups, m0, n0, true, acc, bufA, bufB);
        split8_segment(s1, n_g, args.groups, m0, n0, false, acc, bufA, bufB);
    }

    double2 *out = isH ? args.H : args.S;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave % W8M, wn = wave / W8M;
#pragma unroll
    for (int j = 0; j < T8N; ++j) {
        const int g = n0 + wn * (B8 / W8N) + j * 16 + (lane & 15);
#pragma unroll
        for (int i = 0; i < T8M; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gp = m0 + wm * (B8 / W8M) + i * 16 + 4 * (lane >> 4) + v;
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

hipError_t launch_colmax(const SliceSrc &src, int K, int n_g, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_u64, dim3((n_g + 255) / 256), dim3(256), 0, st, src.mx, n_g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_colmax, dim3((n_g + 63) / 64, (K + CROWS - 1) / CROWS), dim3(256), 0, st,
                       src, K, n_g);
    return hipGetLastError();
}

hipError_t launch_slice(const SliceSrc &src, int K, int n_g, hipStream_t st, bool bf16) {
    const int groups = (K + 15) / 16 * 4;
    hipError_t e = launch_colmax(src, K, n_g, st);
    if (e != hipSuccess) return e;
    const long long items = (long long)groups * n_g;
    if (bf16)
        hipLaunchKernelGGL(k_slice<true>, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, st,
                           src, K, n_g, groups);
    else
        hipLaunchKernelGGL(k_slice<false>, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, st,
                           src, K, n_g, groups);
    return hipGetLastError();
}

hipError_t launch_split_reduce(int K, int n_g, const SliceView (&hseg)[3][2],
                               const SliceView (&sseg)[2][2], double2 *H, double2 *S,
                               hipStream_t st, bool bf16) {
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
    if (bf16) hipLaunchKernelGGL(k_split_reduce<true>, dim3(2 * a.ntri8), dim3(SNT), 0, st, a);
    else hipLaunchKernelGGL(k_split_reduce<false>, dim3(2 * a.ntri8), dim3(SNT), 0, st, a);
    return hipGetLastError();
}

size_t split8_slice_bytes(int K, int n_g) {
    const long long groups = (long long)((K + 31) / 32) * GRP8;
    return (size_t)NSL8 * groups * n_g * 16;
}

hipError_t launch_slice8(const SliceSrc &src, int K, int n_g, hipStream_t st) {
    const int groups = (K + 31) / 32 * GRP8;
    hipError_t e = launch_colmax(src, K, n_g, st);
    if (e != hipSuccess) return e;
    const long long items = (long long)groups * n_g;
    hipLaunchKernelGGL(k_slice8, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, st, src, K,
                       n_g, groups);
    return hipGetLastError();
}

hipError_t launch_split8_reduce(int K, int n_g, const SliceView (&hseg)[3][2],
                                const SliceView (&sseg)[2][2], double2 *H, double2 *S,
                                hipStream_t st) {
    auto u4 = [](const _Float16 *p) { return reinterpret_cast<const uint4 *>(p); };
    Split8Args a;
    for (int i = 0; i < 3; ++i)
        a.h[i] = Split8Seg{u4(hseg[i][0].S), u4(hseg[i][1].S), hseg[i][0].mx, hseg[i][1].mx};
    for (int i = 0; i < 2; ++i)
        a.s[i] = Split8Seg{u4(sseg[i][0].S), u4(sseg[i][1].S), sseg[i][0].mx, sseg[i][1].mx};
    a.H = H;
    a.S = S;
    a.n_g = n_g;
    a.groups = (K + 31) / 32 * GRP8;
    a.nt = (n_g + B8 - 1) / B8;
    a.ntri = a.nt * (a.nt + 1) / 2;   // blocks per output
    a.ntri8 = (a.ntri + 7) / 8 * 8;
    hipLaunchKernelGGL(k_split8_reduce, dim3(2 * a.ntri8), dim3(NT8), 0, st, a);
    return hipGetLastError();
}

}  // namespace hs
