// Complex-double MFMA tile engine for gfx950 (CDNA4).
//
// Computes one BM x BN tile of   C = sum_s P_s^H Q_s   where every operand is
// a row-major complex matrix whose rows are the contraction index and whose
// columns are the output index (this is how the stacked per-atom operands of
// Alg. 1 are laid out: Z, B, Y, X, A are [K][N_G], and the T blocks are
// [N_L][N_L]). Segments (P_s, Q_s) of equal length are concatenated along the
// contraction index, so one K-loop covers e.g. Z^H B + B^H Z + Y^H Y of the H
// reduction.
//
// One complex multiply-add conj(p) q is 4 real FP64 MFMA products:
//   Re += p.re q.re + p.im q.im,   Im += p.re q.im - p.im q.re
// issued as V_MFMA_F64_16X16X4_F64 on 16x16 output blocks with a K step of 4.
//
// Staging: the K-loop advances BK contraction rows at a time. Each stage of P
// (BK x BM) and Q (BK x BN) is fetched from global memory into registers one
// stage ahead, then written to one of two LDS buffers, so the global loads of
// stage s+1 overlap the MFMAs of stage s and a single barrier per stage
// suffices. The fetch is branch-free: addresses are clamped into the operands
// and every load is issued unconditionally; rows past the end and columns
// past the edge are zeroed when the registers are written to LDS, and the
// per-row Q scale is applied there too, so no load waits on another. Per-row
// metadata (the P-row selector and the Q scale) is itself loaded one stage
// earlier than the rows it describes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hs {

typedef double v4d __attribute__((ext_vector_type(4)));

// NSEG segments of `len` rows each (nseg <= NSEG of them active), forming
// the contraction index kk = s * len + r. Row r of segment s contributes
// conj(P_s[r][m]) * w * Q_s[r][n] to C[m][n] with
//   P_s[r] replaced by palt[r] where sel[kk] != 0     (SEL)
//   w = qscale[kk], else 1                              (SCALE)
// sel and qscale cover the whole contraction index (nseg * len entries), so
// reading them needs no test of the segment.
template <int NSEG, bool SEL, bool SCALE>
struct Segs {
    const double2 *P[NSEG];
    const double2 *Q[NSEG];
    int nseg;
    int len;
    long long ldp, ldq;   // row strides, in complex elements
    const double2 *palt;
    const int *sel;
    const double *qscale;
};

template <int BM_, int BN_, int BK_, int WM_, int WN_>
struct TileCfg {
    static constexpr int BM = BM_, BN = BN_, BK = BK_, WM = WM_, WN = WN_;
    static constexpr int NT = 64 * WM * WN;            // threads per block
    static constexpr int WTM = BM / WM, WTN = BN / WN; // wave tile
    static constexpr int TM = WTM / 16, TN = WTN / 16; // 16x16 blocks per wave
    static constexpr int RPP = NT / BM, RPQ = NT / BN; // rows per load pass
    static constexpr int PE = BK / RPP, QE = BK / RPQ; // loads per thread per stage
    static constexpr int LDS_ELEMS = 2 * BK * (BM + BN);
    static_assert(BM % (16 * WM) == 0 && BN % (16 * WN) == 0, "wave tiling");
    static_assert(NT % BM == 0 && NT % BN == 0, "loader needs NT multiple of BM, BN");
    static_assert(BK % RPP == 0 && BK % RPQ == 0 && BK % 4 == 0, "stage depth");
    static_assert(BM % 16 == 0 && BN % 16 == 0, "16-wide MFMA blocks");
    // With BM (BN) a multiple of the 64-lane wave, every P (Q) row a thread
    // loads is the same for its whole wave, so that row bookkeeping runs on
    // the scalar unit (see ztile_run); narrower tiles keep it per lane.
    static constexpr bool PUNI = BM % 64 == 0, QUNI = BN % 64 == 0;
};

template <class C>
struct Acc {
    v4d re[C::TM][C::TN];
    v4d im[C::TM][C::TN];
};

// Segment of contraction row kk and the row within it (row 0 of segment 0
// when kk is past the end, so that addresses stay inside the operands).
template <int NSEG, bool SEL, bool SCALE>
__device__ __forceinline__ void seg_of(const Segs<NSEG, SEL, SCALE> &t, int kk, int &seg, int &r,
                                       bool &valid) {
    valid = kk < t.nseg * t.len;
    int s = 0;
#pragma unroll
    for (int i = 1; i < NSEG; ++i) s += (i < t.nseg && kk >= i * t.len) ? 1 : 0;
    seg = valid ? s : 0;
    r = valid ? kk - s * t.len : 0;
}

// v[seg], formed arithmetically: a chain of selects between pointers read
// from the table is turned into one load at a selected address, which moves
// the whole table into scratch memory.
template <int NSEG>
__device__ __forceinline__ const double2 *pick(const double2 *const (&v)[NSEG], int seg) {
    const uintptr_t base = reinterpret_cast<uintptr_t>(v[0]);
    uintptr_t p = base;
#pragma unroll
    for (int i = 1; i < NSEG; ++i) p += (seg == i) ? reinterpret_cast<uintptr_t>(v[i]) - base : 0;
    return reinterpret_cast<const double2 *>(p);
}

// Main loop. P columns [m0, m0+BM) and Q columns [n0, n0+BN) are read, with
// columns >= mlim / nlim read as zero (mlim, nlim >= 1).
template <class C, int NSEG, bool SEL, bool SCALE>
__device__ __forceinline__ void ztile_run(const Segs<NSEG, SEL, SCALE> &t, int m0, int mlim,
                                          int n0, int nlim, Acc<C> &acc, double2 *lds) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave % C::WM;
    const int wn = wave / C::WM;

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

    // loader coordinates: fixed column per thread, rows strided by RPP / RPQ;
    // out-of-range columns are clamped for the load and zeroed at the store.
    // When BM is a multiple of 64, tid / BM is uniform across a wave:
    // declaring it so moves segment lookup, row pointers and metadata loads
    // to SGPRs/SALU.
    const int pc = tid % C::BM;
    const int pr0 = C::PUNI ? __builtin_amdgcn_readfirstlane(tid / C::BM) : tid / C::BM;
    const int qc = tid % C::BN;
    const int qr0 = C::QUNI ? __builtin_amdgcn_readfirstlane(tid / C::BN) : tid / C::BN;
    const bool pcol_ok = (m0 + pc) < mlim;
    const bool qcol_ok = (n0 + qc) < nlim;
    const int pcol = pcol_ok ? m0 + pc : mlim - 1;
    const int qcol = qcol_ok ? n0 + qc : nlim - 1;

    double2 rp[C::PE], rq[C::QE];   // staged operand values
    bool pv[C::PE], qv[C::QE];      // staged validity
    double qs[C::QE];               // staged Q scale
    int msel[C::PE];                // metadata of the next stage: P selector
    double mqs[C::QE];              // metadata of the next stage: Q scale
#pragma unroll
    for (int i = 0; i < C::PE; ++i) msel[i] = 0;
#pragma unroll
    for (int i = 0; i < C::QE; ++i) {
        mqs[i] = 1.0;
        qs[i] = 1.0;
    }

    // metadata (selector, scale) of stage `stage` into msel / mqs; indices
    // past the end are clamped (those rows are zeroed at the store anyway)
    auto meta = [&](int stage) {
        const int kb = stage * C::BK;
        if constexpr (SEL) {
#pragma unroll
            for (int i = 0; i < C::PE; ++i) {
                const int kk = kb + pr0 + i * C::RPP;
                msel[i] = t.sel[kk < ktot ? kk : ktot - 1];
            }
        }
        if constexpr (SCALE) {
#pragma unroll
            for (int i = 0; i < C::QE; ++i) {
                const int kk = kb + qr0 + i * C::RPQ;
                mqs[i] = t.qscale[kk < ktot ? kk : ktot - 1];
            }
        }
    };
    // operand rows of stage `stage` into registers (uses msel / mqs of that stage)
    auto fetch = [&](int stage) {
        const int kb = stage * C::BK;
#pragma unroll
        for (int i = 0; i < C::PE; ++i) {
            int seg, r;
            bool valid;
            seg_of(t, kb + pr0 + i * C::RPP, seg, r, valid);
            const double2 *p = pick<NSEG>(t.P, seg);
            if constexpr (SEL) {
                const uintptr_t pp = reinterpret_cast<uintptr_t>(p);
                p = reinterpret_cast<const double2 *>(
                    pp + (msel[i] ? reinterpret_cast<uintptr_t>(t.palt) - pp : 0));
            }
            rp[i] = p[(long long)r * t.ldp + pcol];
            pv[i] = valid && pcol_ok;
        }
#pragma unroll
        for (int i = 0; i < C::QE; ++i) {
            int seg, r;
            bool valid;
            seg_of(t, kb + qr0 + i * C::RPQ, seg, r, valid);
            const double2 *q = pick<NSEG>(t.Q, seg);
            rq[i] = q[(long long)r * t.ldq + qcol];
            qv[i] = valid && qcol_ok;
            if constexpr (SCALE) qs[i] = mqs[i];
        }
    };
    // (selects are per scalar component: a select between two double2
    // aggregates is turned into a select of addresses, which forces the
    // staging arrays into scratch memory)
    auto stash = [&](int buf) {
        double2 *lp = lds + buf * C::BK * (C::BM + C::BN);
        double2 *lq = lp + C::BK * C::BM;
#pragma unroll
        for (int i = 0; i < C::PE; ++i) {
            double2 v;
            v.x = pv[i] ? rp[i].x : 0.0;
            v.y = pv[i] ? rp[i].y : 0.0;
            lp[(pr0 + i * C::RPP) * C::BM + pc] = v;
        }
#pragma unroll
        for (int i = 0; i < C::QE; ++i) {
            double2 v;
            v.x = qv[i] ? rq[i].x : 0.0;
            v.y = qv[i] ? rq[i].y : 0.0;
            if constexpr (SCALE) {
                v.x *= qs[i];
                v.y *= qs[i];
            }
            lq[(qr0 + i * C::RPQ) * C::BN + qc] = v;
        }
    };

    // Loads of the stages after the last one are issued too (their indices
    // are clamped, so they stay in bounds, and their rows are never used):
    // a conditional load would leave a join in the loop at which the compiler
    // waits for every outstanding load, including the prefetch.
    meta(0);
    fetch(0);
    meta(1);
    stash(0);
    __syncthreads();

    const int lr = lane >> 4;   // contraction row within a K step of 4
    const int lc = lane & 15;   // column within a 16-wide block

    // LDS fragments of K step k4 (4 contraction rows) for this wave.
    auto ldfrag = [&](const double2 *lp, const double2 *lq, int k4, double2 (&a)[C::TM],
                      double2 (&b)[C::TN]) {
        const int kr = k4 * 4 + lr;
#pragma unroll
        for (int i = 0; i < C::TM; ++i) a[i] = lp[kr * C::BM + wm * C::WTM + i * 16 + lc];
#pragma unroll
        for (int j = 0; j < C::TN; ++j) b[j] = lq[kr * C::BN + wn * C::WTN + j * 16 + lc];
    };
    // The 4 TM TN real MFMAs of one K step.
    auto mma = [&](const double2 (&a)[C::TM], const double2 (&b)[C::TN]) {
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
    // Interleave the next step's TM+TN fragment reads with this step's
    // 4 TM TN MFMAs (one LDS read, then a few MFMAs), instead of letting the
    // scheduler hoist every read of the stage ahead of the MFMAs.
    auto interleave = [&]() {
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
    static_assert((C::BK / 4) % 2 == 0, "K steps per stage must be even");

    for (int s = 0; s < nst; ++s) {
        fetch(s + 1);
        meta(s + 2);
        const double2 *lp = lds + (s & 1) * C::BK * (C::BM + C::BN);
        const double2 *lq = lp + C::BK * C::BM;
        double2 fa0[C::TM], fb0[C::TN], fa1[C::TM], fb1[C::TN];
        // The last stage can hold fewer than BK valid rows (the rest are
        // zero-filled): when its second half holds none, its two K steps
        // are skipped (they would add exact zeros). Short contractions - the
        // per-atom products - save part of a stage this way.
        const bool full = ktot - s * C::BK > C::BK / 2;
        ldfrag(lp, lq, 0, fa0, fb0);
#pragma unroll
        for (int k4 = 0; k4 < C::BK / 4; k4 += 2) {
            if (k4 >= C::BK / 8 && !full) break;
            ldfrag(lp, lq, k4 + 1, fa1, fb1);
            mma(fa0, fb0);
            interleave();
            if (k4 + 2 < C::BK / 4) ldfrag(lp, lq, k4 + 2, fa0, fb0);
            mma(fa1, fb1);
            if (k4 + 2 < C::BK / 4) interleave();
        }
        stash((s + 1) & 1);
        __syncthreads();
    }
}

// Output coordinates of accumulator element v of block (i, j) for this lane.
// Operand layouts of V_MFMA_F64_16X16X4_F64: lane l holds A[l % 16][l / 16]
// and B[l / 16][l % 16]; result element v of lane l is D[4 v + l / 16][l % 16]
// (measured on gfx950 with a one-wave probe of known integer operands).
template <class C>
__device__ __forceinline__ int acc_row(int i, int v) {
    const int wave = threadIdx.x >> 6;
    return (wave % C::WM) * C::WTM + i * 16 + 4 * v + ((threadIdx.x & 63) >> 4);
}
template <class C>
__device__ __forceinline__ int acc_col(int j) {
    const int wave = threadIdx.x >> 6;
    return (wave / C::WM) * C::WTN + j * 16 + (threadIdx.x & 15);
}

}  // namespace hs
