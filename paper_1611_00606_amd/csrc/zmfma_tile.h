// Complex-double MFMA tile engine for gfx950 (CDNA4).
//
// Computes one BM x BN tile of   C = sum_s P_s^H Q_s   where every operand is
// a row-major complex matrix whose rows are the contraction index and whose
// columns are the output index (this is how the stacked per-atom operands of
// Alg. 1 are laid out: Z, B, Y, X, A are [K][N_G], and the T blocks are
// [N_L][N_L]). Segments (P_s, Q_s) are concatenated along the contraction
// index, so one K-loop covers e.g. Z^H B + B^H Z + Y^H Y of the H reduction.
//
// One complex multiply-add conj(p) q is 4 real FP64 MFMA products:
//   Re += p.re q.re + p.im q.im,   Im += p.re q.im - p.im q.re
// issued as V_MFMA_F64_16X16X4_F64 on 16x16 output blocks with a K step of 4.
//
// Staging: the K-loop advances BK contraction rows at a time. Each stage of P
// (BK x BM) and Q (BK x BN) is fetched from global memory into registers one
// stage ahead, then written to one of two LDS buffers, so the global loads of
// stage s+1 overlap the MFMAs of stage s and a single barrier per stage
// suffices.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hs {

typedef double v4d __attribute__((ext_vector_type(4)));

// One contraction segment. Row r (0 <= r < rows) of the segment contributes
// conj(P[r][m]) * qscale[r] * Q[r][n] to C[m][n]. Where `sel` is given and
// sel[r] != 0, row r of P is taken from `Palt` instead of `P`.
struct Seg {
    const double2 *P;
    const double2 *Palt;
    const int *sel;
    const double2 *Q;
    const double *qscale;
    int rows;
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
};

template <class C>
struct Acc {
    v4d re[C::TM][C::TN];
    v4d im[C::TM][C::TN];
};

// Segment table of up to NSEG segments; row lookup is fully unrolled (no
// dynamic indexing into the table, which would go through scratch).
// All segments of a table share the row strides of P and of Q.
template <int NSEG>
struct SegTable {
    Seg s[NSEG];
    int n;
    long long ldp, ldq;   // row strides, in complex elements
};

// Resolve contraction row kk of a segment table into row pointers of P and Q
// (nullptr past the end) and the Q row scale.
template <int NSEG>
__device__ __forceinline__ void seg_row(const SegTable<NSEG> &t, int kk,
                                        const double2 *&prow, const double2 *&qrow,
                                        double &qs) {
    const double2 *p = nullptr, *q = nullptr, *palt = nullptr;
    const int *sel = nullptr;
    const double *sc = nullptr;
    int r = kk;
    bool done = false;
#pragma unroll
    for (int i = 0; i < NSEG; ++i) {
        const Seg &s = t.s[i];
        const bool here = !done && i < t.n && r < s.rows;
        p = here ? s.P : p;
        q = here ? s.Q : q;
        palt = here ? s.Palt : palt;
        sel = here ? s.sel : sel;
        sc = here ? s.qscale : sc;
        if (!done && !here && i < t.n) r -= s.rows;
        done = done || here;
    }
    if (!done) {
        prow = nullptr;
        qrow = nullptr;
        qs = 1.0;
        return;
    }
    if (sel && sel[r]) p = palt;
    prow = p + (long long)r * t.ldp;
    qrow = q + (long long)r * t.ldq;
    qs = sc ? sc[r] : 1.0;
}

// Main loop. `table` lists the segments; P columns [m0, m0+BM) and Q columns
// [n0, n0+BN) are read, with columns >= mlim / nlim read as zero.
template <class C, int NSEG>
__device__ __forceinline__ void ztile_run(const SegTable<NSEG> &table, int ktot,
                                          int m0, int mlim, int n0, int nlim,
                                          Acc<C> &acc, double2 *lds) {
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

    // loader coordinates: fixed column per thread, rows strided by RPP / RPQ
    const int pc = tid % C::BM, pr0 = tid / C::BM;
    const int qc = tid % C::BN, qr0 = tid / C::BN;
    const bool pcol_ok = (m0 + pc) < mlim;
    const bool qcol_ok = (n0 + qc) < nlim;

    double2 rp[C::PE], rq[C::QE];
    const double2 zero = {0.0, 0.0};

    auto fetch = [&](int stage) {
        const int kb = stage * C::BK;
#pragma unroll
        for (int i = 0; i < C::PE; ++i) {
            const int kk = kb + pr0 + i * C::RPP;
            const double2 *prow, *qrow;
            double qs;
            rp[i] = zero;
            if (kk < ktot) {
                seg_row(table, kk, prow, qrow, qs);
                if (pcol_ok && prow) rp[i] = prow[m0 + pc];
            }
        }
#pragma unroll
        for (int i = 0; i < C::QE; ++i) {
            const int kk = kb + qr0 + i * C::RPQ;
            const double2 *prow, *qrow;
            double qs;
            rq[i] = zero;
            if (kk < ktot) {
                seg_row(table, kk, prow, qrow, qs);
                if (qcol_ok && qrow) {
                    double2 v = qrow[n0 + qc];
                    v.x *= qs;
                    v.y *= qs;
                    rq[i] = v;
                }
            }
        }
    };
    auto stash = [&](int buf) {
        double2 *lp = lds + buf * C::BK * (C::BM + C::BN);
        double2 *lq = lp + C::BK * C::BM;
#pragma unroll
        for (int i = 0; i < C::PE; ++i) lp[(pr0 + i * C::RPP) * C::BM + pc] = rp[i];
#pragma unroll
        for (int i = 0; i < C::QE; ++i) lq[(qr0 + i * C::RPQ) * C::BN + qc] = rq[i];
    };

    const int nst = (ktot + C::BK - 1) / C::BK;
    if (nst == 0) return;
    fetch(0);
    stash(0);
    __syncthreads();

    const int lr = lane >> 4;   // contraction row within a K step of 4
    const int lc = lane & 15;   // column within a 16-wide block

    for (int s = 0; s < nst; ++s) {
        if (s + 1 < nst) fetch(s + 1);
        const double2 *lp = lds + (s & 1) * C::BK * (C::BM + C::BN);
        const double2 *lq = lp + C::BK * C::BM;
#pragma unroll
        for (int k4 = 0; k4 < C::BK / 4; ++k4) {
            const int kr = k4 * 4 + lr;
            double2 a[C::TM], b[C::TN];
            double nbr[C::TN];
#pragma unroll
            for (int i = 0; i < C::TM; ++i) a[i] = lp[kr * C::BM + wm * C::WTM + i * 16 + lc];
#pragma unroll
            for (int j = 0; j < C::TN; ++j) {
                b[j] = lq[kr * C::BN + wn * C::WTN + j * 16 + lc];
                nbr[j] = -b[j].x;
            }
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
        }
        if (s + 1 < nst) stash((s + 1) & 1);
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
