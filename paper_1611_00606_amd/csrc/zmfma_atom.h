// Complex-double MFMA tile engine of the per-atom products (k_atom, k_batch):
// one tile of C = sum_s P_s^H Q_s with the operands moved global -> LDS by
// 16-byte direct loads (global_load_lds_dwordx4; lane l lands at base + 16 l),
// as in zmfma_direct.h, but shaped for the per-atom operands:
//
// * the tile's rows are the atom's N_L output rows (up to 128, in blocks of
//   16) and its columns 128 or 256 plane-wave columns, so one tile usually
//   covers every row of an atom: the A and B columns of a tile are read once
//   instead of once per 32-row tile;
// * the P rows (the atom's N_L x N_L blocks) are N_L entries long: a P row is
//   loaded as 64-column pieces with the columns past N_L clamped to the last
//   one (they only feed output rows past N_L, which are not stored);
// * triangular P (W_a = C_a^H A_a with C_a lower triangular): output row l
//   only needs contraction rows k >= l, so a 16-row block of outputs skips the
//   stages below its first row (those would add exact zeros);
// * a last stage whose second half holds no contraction rows skips it.
//
// Waves: 2 x 4; wave w takes block row w / 4 and block column w % 4, so each
// SIMD (waves w and w + 4) holds one wave of each block row and the
// triangle's skipped stages shorten every SIMD's work alike.
#pragma once

#include "zmfma_tile.h"

namespace hs {

template <int TM_, int TN_, int BK_>
struct AtomCfg {
    static constexpr int WM = 2, WN = 4;
    static constexpr int NT = 64 * WM * WN;
    static constexpr int TM = TM_, TN = TN_, BK = BK_;
    static constexpr int WTM = 16 * TM, WTN = 16 * TN;   // wave tile
    static constexpr int BM = WM * WTM, BN = WN * WTN;   // tile
    static constexpr int BMS = (BM + 63) / 64 * 64;      // LDS row width of P
    static constexpr int BNS = BN;                       // LDS row width of Q
    static constexpr int PH = BMS / 64, QH = BNS / 64;   // 64-column loads per row
    static constexpr int STAGE = BK * (BMS + BNS);       // complex elements per stage
    static constexpr int LDS_ELEMS = 2 * STAGE;
    static_assert(BN % 64 == 0, "64-column loads of Q");
    static_assert(BK == 8 || BK == 16, "each wave loads BK / 8 rows of a stage");
    static_assert(BK % 8 == 0 && (BK / 4) % 2 == 0, "K steps per stage must be even");
};

// Output coordinates of accumulator element v of block (i, j) for this lane
// (V_MFMA_F64_16X16X4_F64: result element v of lane l is D[4 v + l / 16][l % 16]).
template <class C>
__device__ __forceinline__ int atom_row(int i, int v) {
    const int wave = threadIdx.x >> 6;
    return (wave / C::WN) * C::WTM + i * 16 + 4 * v + ((threadIdx.x & 63) >> 4);
}
template <class C>
__device__ __forceinline__ int atom_col(int j) {
    const int wave = threadIdx.x >> 6;
    return (wave % C::WN) * C::WTN + j * 16 + (threadIdx.x & 15);
}

// tri: P is triangular in the sense above, with the tile's first output row
// at contraction row 0 (the caller starts the contraction at the tile's first
// row).
template <class C, int NSEG>
__device__ __forceinline__ void ztile_atom(const Segs<NSEG, false, false> &t, int m0, int mlim,
                                           int n0, int nlim, bool tri, Acc<C> &acc,
                                           double2 *lds) {
    static_assert(C::NT == 512, "8 waves");
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave / C::WN;
    const int wn = wave % C::WN;

#pragma unroll
    for (int i = 0; i < C::TM; ++i)
#pragma unroll
        for (int j = 0; j < C::TN; ++j) {
            acc.re[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
            acc.im[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
        }

    const int ktot = t.nseg * t.len;
    const int nst = (ktot + C::BK - 1) / C::BK;
    if (nst == 0) return;
    // with P triangular, this wave's block row i starts at output row
    // wm WTM + 16 i (a multiple of BK) and needs contraction rows from there
    // on: its first stage is sbase + i SPB
    const int sbase = wm * C::WTM / C::BK;
    constexpr int SPB = 16 / C::BK;   // stages per 16-row block

    unsigned pvo[C::PH], qvo[C::QH];
#pragma unroll
    for (int h = 0; h < C::PH; ++h) {
        const int c = m0 + 64 * h + lane;
        pvo[h] = (unsigned)(c < mlim ? c : mlim - 1) * 16u;
    }
#pragma unroll
    for (int h = 0; h < C::QH; ++h) {
        const int c = n0 + 64 * h + lane;
        qvo[h] = (unsigned)(c < nlim ? c : nlim - 1) * 16u;
    }
    auto at = [](const double2 *row, unsigned vo) __attribute__((always_inline)) {
        return reinterpret_cast<const double2 *>(reinterpret_cast<const char *>(row) + vo);
    };
    // rows w (and w + 8) of stage st into buf
    auto issue = [&](double2 *buf, int st) __attribute__((always_inline)) {
        double2 *lp = buf;
        double2 *lq = buf + C::BK * C::BMS;
#pragma unroll
        for (int k = 0; k < C::BK / 8; ++k) {
            const int r = wave + 8 * k;
            const int kk = st * C::BK + r;
            if (kk < ktot) {
                const int s = (NSEG > 1 && kk >= t.len) ? 1 : 0;
                const long long row = kk - s * t.len;
                const double2 *prow = pick<NSEG>(t.P, s) + row * t.ldp;
                const double2 *qrow = pick<NSEG>(t.Q, s) + row * t.ldq;
#pragma unroll
                for (int h = 0; h < C::PH; ++h)
                    __builtin_amdgcn_global_load_lds(at(prow, pvo[h]), lp + r * C::BMS + 64 * h, 16, 0, 0);
#pragma unroll
                for (int h = 0; h < C::QH; ++h)
                    __builtin_amdgcn_global_load_lds(at(qrow, qvo[h]), lq + r * C::BNS + 64 * h, 16, 0, 0);
            } else {
#pragma unroll
                for (int h = 0; h < C::PH; ++h) lp[r * C::BMS + 64 * h + lane] = double2{0.0, 0.0};
#pragma unroll
                for (int h = 0; h < C::QH; ++h) lq[r * C::BNS + 64 * h + lane] = double2{0.0, 0.0};
            }
        }
    };

    const int lr = lane >> 4;   // contraction row within a K step of 4
    const int lc = lane & 15;   // column within a 16-wide block
    auto ldfrag = [&](const double2 *lp, const double2 *lq, int k4, double2 (&a)[C::TM],
                      double2 (&b)[C::TN]) __attribute__((always_inline)) {
        const int kr = k4 * 4 + lr;
#pragma unroll
        for (int i = 0; i < C::TM; ++i) a[i] = lp[kr * C::BMS + wm * C::WTM + i * 16 + lc];
#pragma unroll
        for (int j = 0; j < C::TN; ++j) b[j] = lq[kr * C::BNS + wn * C::WTN + j * 16 + lc];
    };
    // the 4 TM TN real MFMAs of one K step (block rows with on[i] only), in
    // four passes over the blocks so that two MFMAs into one accumulator are
    // 2 TM TN - 1 MFMAs apart
    auto mma = [&](const bool (&on)[C::TM], const double2 (&a)[C::TM], const double2 (&b)[C::TN])
                   __attribute__((always_inline)) {
        double nbr[C::TN];
#pragma unroll
        for (int j = 0; j < C::TN; ++j) nbr[j] = -b[j].x;
#pragma unroll
        for (int i = 0; i < C::TM; ++i)
            if (on[i])
#pragma unroll
                for (int j = 0; j < C::TN; ++j)
                    acc.re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].x, b[j].x, acc.re[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < C::TM; ++i)
            if (on[i])
#pragma unroll
                for (int j = 0; j < C::TN; ++j)
                    acc.im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].x, b[j].y, acc.im[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < C::TM; ++i)
            if (on[i])
#pragma unroll
                for (int j = 0; j < C::TN; ++j)
                    acc.re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].y, b[j].y, acc.re[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < C::TM; ++i)
            if (on[i])
#pragma unroll
                for (int j = 0; j < C::TN; ++j)
                    acc.im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].y, nbr[j], acc.im[i][j], 0, 0, 0);
    };
    // one LDS fragment read, then a few MFMAs, for the next step's TM + TN
    // reads (1% faster than the scheduler's own order)
    auto interleave = [&]() __attribute__((always_inline)) {
        constexpr int NR = C::TM + C::TN;
        constexpr int NM = 4 * C::TM * C::TN;
        constexpr int PER = NM / (NR + 1);
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x008, PER, 0);
        }
        __builtin_amdgcn_sched_group_barrier(0x008, NM - NR * PER, 0);
    };
    // block row i of this wave takes part in stage st from its first stage
    // on (every stage when P is not triangular)
    auto compute = [&](const double2 *lp, const double2 *lq, int st) __attribute__((always_inline)) {
        // the last stage's second half holds no contraction rows: skip it
        const bool full = ktot - st * C::BK > C::BK / 2;
        bool on[C::TM];
#pragma unroll
        for (int i = 0; i < C::TM; ++i) on[i] = !tri || st >= sbase + i * SPB;
        double2 fa0[C::TM], fb0[C::TN], fa1[C::TM], fb1[C::TN];
        ldfrag(lp, lq, 0, fa0, fb0);
#pragma unroll
        for (int k4 = 0; k4 < C::BK / 4; k4 += 2) {
            if (k4 >= C::BK / 8 && !full) break;
            ldfrag(lp, lq, k4 + 1, fa1, fb1);
            mma(on, fa0, fb0);
            interleave();
            if (k4 + 2 < C::BK / 4) ldfrag(lp, lq, k4 + 2, fa0, fb0);
            mma(on, fa1, fb1);
            if (k4 + 2 < C::BK / 4) interleave();
        }
    };

    issue(lds, 0);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    for (int s = 0; s < nst; ++s) {
        // the buffer being computed and the one being loaded are distinct:
        // saying so (restrict) keeps the compiler from waiting for the
        // direct loads before every LDS read of the stage
        auto stage = [&](const double2 *__restrict__ cur, double2 *__restrict__ nxt)
                         __attribute__((always_inline)) {
            if (s + 1 < nst) issue(nxt, s + 1);
            compute(cur, cur + C::BK * C::BMS, s);
        };
        stage(lds + (s & 1) * C::STAGE, lds + ((s + 1) & 1) * C::STAGE);
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
    }
}

}  // namespace hs
