// Complex-double MFMA tile engine with direct global -> LDS operand loads,
// for the large reductions (k_reduce). Same contraction and accumulator
// layout as ztile_run in zmfma_tile.h (C = sum_s P_s^H Q_s over
// concatenated segments, 4 real V_MFMA_F64_16X16X4_F64 per complex step), but
// the operand rows move from global memory straight into LDS with 16-byte
// loads (global_load_lds_dwordx4: lane l of a wave lands at base + 16 l), so
// no staging registers and no LDS-store instructions sit in the K loop.
//
// One stage is BK = 16 contraction rows of P (BM columns) and Q (BN
// columns). Wave w loads rows w and w + 8 of both, 64 columns per load, so
// every load's row is wave-uniform: its segment, its row pointer and the
// failure-branch selector (SEL: P row taken from palt; the selectors are
// loaded a stage ahead) are scalar work.
// Columns past the edge read the last column (they only feed outputs past
// the edge, which are not stored); rows past the end of the contraction are
// written as zeros with ordinary LDS stores (only the last stage has any).
// The per-row scale of Q (SCALE) is applied to the Q fragment in registers,
// from a value prefetched one stage ahead. Two LDS buffers: the next stage
// loads while the current one is multiplied; the buffers are handed to the
// stage body as distinct (restrict) pointers, without which the compiler
// waits for the loads before the stage's LDS reads.
//
// G3: the complex product in 3 real products instead of 4 (the 3M or Gauss
// form): per contraction row, with p = pr + i pi and q = qr + i qi,
//   T1 += pr qr,   T2 += pi qi,   T3 += (pr - pi)(qr + qi)
// and at the end Re = T1 + T2, Im = T3 - T1 + T2, which is conj(p) q summed.
// T1 and T2 live in acc.re and acc.im until the final fold. The real part is
// the same sum as in the 4-product form; the imaginary part's rounding error
// is bounded by the unit roundoff times |pr - pi||qr + qi| + |pr||qr| +
// |pi||qi| (summed over the contraction) instead of |pr||qi| + |pi||qr|.
// Three accumulator sets of a 64x32 wave tile take 192 of the 256 registers
// a wave has at two waves per SIMD, so the fragments are not double-buffered.
#pragma once

#include "zmfma_tile.h"

namespace hs {

template <class C, int NSEG, bool SEL, bool SCALE, bool G3 = false>
__device__ __forceinline__ void ztile_direct(const Segs<NSEG, SEL, SCALE> &t, int m0, int mlim,
                                             int n0, int nlim, Acc<C> &acc, double2 *lds) {
    static_assert(C::BK == 16 && C::NT == 512, "8 waves load rows w and w + 8 of a 16-row stage");
    static_assert(C::BM % 64 == 0 && C::BN % 64 == 0, "64-column loads");
    constexpr int PH = C::BM / 64, QH = C::BN / 64;   // loads per row
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave % C::WM;
    const int wn = wave / C::WM;

#pragma unroll
    for (int i = 0; i < C::TM; ++i)
#pragma unroll
        for (int j = 0; j < C::TN; ++j) {
            acc.re[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
            acc.im[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
        }
    v4d t3[G3 ? C::TM : 1][G3 ? C::TN : 1];
    if constexpr (G3) {
#pragma unroll
        for (int i = 0; i < C::TM; ++i)
#pragma unroll
            for (int j = 0; j < C::TN; ++j) t3[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
    }

    const int ktot = t.nseg * t.len;
    const int nst = (ktot + C::BK - 1) / C::BK;
    if (nst == 0) return;

    // per-lane byte offsets of the loaded columns (clamped at the edge)
    unsigned pvo[PH], qvo[QH];
#pragma unroll
    for (int h = 0; h < PH; ++h) {
        const int c = m0 + 64 * h + lane;
        pvo[h] = (unsigned)(c < mlim ? c : mlim - 1) * 16u;
    }
#pragma unroll
    for (int h = 0; h < QH; ++h) {
        const int c = n0 + 64 * h + lane;
        qvo[h] = (unsigned)(c < nlim ? c : nlim - 1) * 16u;
    }
    auto at = [](const double2 *row, unsigned vo) __attribute__((always_inline)) {
        return reinterpret_cast<const double2 *>(reinterpret_cast<const char *>(row) + vo);
    };
    // failure-branch selectors of this wave's rows w and w + 8, loaded one
    // stage before the rows themselves: a selector loaded and used at once
    // held every stage's loads (and so its MFMAs) for a memory round trip
    int selv[2] = {0, 0};
    auto load_sel = [&](int st) __attribute__((always_inline)) {
        if constexpr (SEL) {
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int kk = st * C::BK + wave + 8 * k;
                selv[k] = kk < ktot ? t.sel[kk] : 0;
            }
        }
    };
    // rows w and w + 8 of stage st into buf (selectors from load_sel(st))
    auto issue = [&](double2 *buf, int st) __attribute__((always_inline)) {
        double2 *lp = buf;
        double2 *lq = buf + C::BK * C::BM;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int r = wave + 8 * k;
            const int kk = st * C::BK + r;
            if (kk < ktot) {
                int s = 0;
#pragma unroll
                for (int i = 1; i < NSEG; ++i) s += (i < t.nseg && kk >= i * t.len) ? 1 : 0;
                const long long row = kk - s * t.len;
                const double2 *prow = pick<NSEG>(t.P, s);
                if constexpr (SEL)
                    if (selv[k]) prow = t.palt;
                const double2 *qrow = pick<NSEG>(t.Q, s);
                prow += row * t.ldp;
                qrow += row * t.ldq;
#pragma unroll
                for (int h = 0; h < PH; ++h)
                    __builtin_amdgcn_global_load_lds(at(prow, pvo[h]), lp + r * C::BM + 64 * h, 16, 0, 0);
#pragma unroll
                for (int h = 0; h < QH; ++h)
                    __builtin_amdgcn_global_load_lds(at(qrow, qvo[h]), lq + r * C::BN + 64 * h, 16, 0, 0);
            } else {
#pragma unroll
                for (int h = 0; h < PH; ++h) lp[r * C::BM + 64 * h + lane] = double2{0.0, 0.0};
#pragma unroll
                for (int h = 0; h < QH; ++h) lq[r * C::BN + 64 * h + lane] = double2{0.0, 0.0};
            }
        }
    };

    const int lr = lane >> 4;   // contraction row within a K step of 4
    const int lc = lane & 15;   // column within a 16-wide block
    // Q scales of this lane's rows in the 4 K steps of a stage
    double qs[C::BK / 4], qs_next[C::BK / 4];
    auto load_scales = [&](double (&dst)[C::BK / 4], int st) __attribute__((always_inline)) {
        if constexpr (SCALE) {
#pragma unroll
            for (int k4 = 0; k4 < C::BK / 4; ++k4) {
                const int kk = st * C::BK + 4 * k4 + lr;
                dst[k4] = t.qscale[kk < ktot ? kk : ktot - 1];
            }
        }
    };

    auto ldfrag = [&](const double2 *lp, const double2 *lq, int k4, double2 (&a)[C::TM],
                      double2 (&b)[C::TN]) __attribute__((always_inline)) {
        const int kr = k4 * 4 + lr;
#pragma unroll
        for (int i = 0; i < C::TM; ++i) a[i] = lp[kr * C::BM + wm * C::WTM + i * 16 + lc];
#pragma unroll
        for (int j = 0; j < C::TN; ++j) {
            b[j] = lq[kr * C::BN + wn * C::WTN + j * 16 + lc];
            if constexpr (SCALE) {
                b[j].x *= qs[k4];
                b[j].y *= qs[k4];
            }
        }
    };
    auto mma = [&](const double2 (&a)[C::TM], const double2 (&b)[C::TN]) __attribute__((always_inline)) {
        if constexpr (G3) {
            double sb[C::TN];
#pragma unroll
            for (int j = 0; j < C::TN; ++j) sb[j] = b[j].x + b[j].y;
#pragma unroll
            for (int i = 0; i < C::TM; ++i)
#pragma unroll
                for (int j = 0; j < C::TN; ++j)
                    acc.re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].x, b[j].x, acc.re[i][j], 0, 0, 0);
#pragma unroll
            for (int i = 0; i < C::TM; ++i)
#pragma unroll
                for (int j = 0; j < C::TN; ++j)
                    acc.im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].y, b[j].y, acc.im[i][j], 0, 0, 0);
#pragma unroll
            for (int i = 0; i < C::TM; ++i) {
                const double sa = a[i].x - a[i].y;
#pragma unroll
                for (int j = 0; j < C::TN; ++j)
                    t3[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(sa, sb[j], t3[i][j], 0, 0, 0);
            }
            return;
        }
        double nbr[C::TN];
#pragma unroll
        for (int j = 0; j < C::TN; ++j) nbr[j] = -b[j].x;
#pragma unroll
        for (int i = 0; i < C::TM; ++i)
#pragma unroll
            for (int j = 0; j < C::TN; ++j)
                acc.re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].x, b[j].x, acc.re[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < C::TM; ++i)
#pragma unroll
            for (int j = 0; j < C::TN; ++j)
                acc.im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].x, b[j].y, acc.im[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < C::TM; ++i)
#pragma unroll
            for (int j = 0; j < C::TN; ++j)
                acc.re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].y, b[j].y, acc.re[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < C::TM; ++i)
#pragma unroll
            for (int j = 0; j < C::TN; ++j)
                acc.im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].y, nbr[j], acc.im[i][j], 0, 0, 0);
    };
    auto interleave = [&]() __attribute__((always_inline)) {
        constexpr int NR = C::TM + C::TN;
        constexpr int NM = (G3 ? 3 : 4) * C::TM * C::TN;
        constexpr int PER = NM / (NR + 1);
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x008, PER, 0);
        }
        __builtin_amdgcn_sched_group_barrier(0x008, NM - NR * PER, 0);
    };
    static_assert((C::BK / 4) % 2 == 0, "K steps per stage must be even");
    auto compute = [&](const double2 *lp, const double2 *lq) __attribute__((always_inline)) {
        if constexpr (G3) {
#pragma unroll
            for (int k4 = 0; k4 < C::BK / 4; ++k4) {
                double2 fa[C::TM], fb[C::TN];
                ldfrag(lp, lq, k4, fa, fb);
                mma(fa, fb);   // no interleave hints: the free schedule is faster here
            }
            return;
        }
        double2 fa0[C::TM], fb0[C::TN], fa1[C::TM], fb1[C::TN];
        ldfrag(lp, lq, 0, fa0, fb0);
#pragma unroll
        for (int k4 = 0; k4 < C::BK / 4; k4 += 2) {
            ldfrag(lp, lq, k4 + 1, fa1, fb1);
            mma(fa0, fb0);
            interleave();
            if (k4 + 2 < C::BK / 4) ldfrag(lp, lq, k4 + 2, fa0, fb0);
            mma(fa1, fb1);
            if (k4 + 2 < C::BK / 4) interleave();
        }
    };

    constexpr int BUF = C::BK * (C::BM + C::BN);
    load_scales(qs, 0);
    load_sel(0);
    issue(lds, 0);
    load_sel(1);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    for (int s = 0; s < nst; ++s) {
        auto stage = [&](const double2 *__restrict__ cur, double2 *__restrict__ nxt)
                         __attribute__((always_inline)) {
            if (s + 1 < nst) {
                issue(nxt, s + 1);
                load_scales(qs_next, s + 1);
                load_sel(s + 2);
            }
            compute(cur, cur + C::BK * C::BM);
        };
        stage(lds + (s & 1) * BUF, lds + ((s + 1) & 1) * BUF);
        if constexpr (SCALE) {
#pragma unroll
            for (int k4 = 0; k4 < C::BK / 4; ++k4) qs[k4] = qs_next[k4];
        }
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
    }
    if constexpr (G3) {
#pragma unroll
        for (int i = 0; i < C::TM; ++i)
#pragma unroll
            for (int j = 0; j < C::TN; ++j) {
                const v4d t1 = acc.re[i][j], t2 = acc.im[i][j];
                acc.re[i][j] = t1 + t2;
                acc.im[i][j] = (t3[i][j] - t1) + t2;
            }
    }
}

}  // namespace hs
