// The large stacked reductions of Alg. 1, on complex FP64 MFMA tiles:
//   H = Z^H B + B^H Z              (zher2k)
//     + A_notHPD^H X_notHPD        (failure-branch zgemm)
//     + Y_HPD^H Y_HPD              (HPD zherk)
//   S = A^H A + (U B)^H (U B)      (zherk, scaling of B by U, zherk)
// The second-loop operands are held in one stacked matrix W (Y_a or X_a in
// atom a's rows); for the rows of failing atoms the left operand is A, chosen
// per row by `sel`, so no compaction of the stacks is needed. The U scaling
// is applied to the right operand as |u|^2 while it is loaded.
//
// Only lower-triangle tiles (tile row >= tile column) are computed; one block
// per tile and output. H tiles are dispatched before S tiles (they carry 1.5x
// the contraction length). Consecutive blocks of the hardware dispatch go to
// the 8 XCDs in turn, so block b is remapped to tile index
// (b mod 8) * (tiles/8) + b/8: each XCD then walks a contiguous run of a
// banded tile order, and the blocks resident on one XCD share the column
// panels they read through that XCD's L2.
//
// With G3 every complex product takes 3 real MFMA products instead of 4 (the
// 3M form, see zmfma_direct.h): three quarters of the matrix-core work, a
// slightly larger rounding bound on the imaginary parts.
//
// k_mirror (launched separately, also after the split-precision reduction)
// completes both outputs: upper = conj(lower), Im(diag) = 0.
#include "hs_internal.h"
#include "zmfma_direct.h"

namespace hs {

namespace {

// Tile shape of the reductions: 128 x 128 outputs, stages of 16 contraction
// rows, 8 waves as 2 x 4 (64 x 32 complex outputs each).
using RedCfg = TileCfg<128, 128, 16, 2, 4>;
static_assert(RedCfg::BM == RedCfg::BN, "lower-triangle tiling needs square tiles");
constexpr int BAND = 4;   // tile columns per band of the tile order

struct RedArgs {
    const double2 *A, *B, *Z, *W;
    const int *sel;
    const double *d;
    int K;
    double2 *H;
    double2 *S;
    int n_g;
    int nt;       // tiles per dimension
    int ntri;     // lower-triangle tiles per output
    int ntri8;    // ntri rounded up to a multiple of 8
};

// Tile (i, j), j <= i, of the t-th position in the banded order: bands of
// BAND tile columns, each band walked row by row from its diagonal down.
__device__ __forceinline__ void band_tile(int t, int nt, int &ti, int &tj) {
    int c0 = 0;
    for (;;) {
        const int m = nt - c0;
        if (m <= 0) {   // t beyond the triangle: no tile
            ti = tj = -1;
            return;
        }
        const int w = m < BAND ? m : BAND;
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
        c0 += BAND;
    }
}

template <bool G3>
__global__ void __launch_bounds__(RedCfg::NT)
k_reduce(RedArgs args) {
    using C = RedCfg;
    __shared__ double2 lds[C::LDS_ELEMS];

    int b = blockIdx.x;
    const bool isH = b < args.ntri8;
    if (!isH) b -= args.ntri8;
    const int per_xcd = args.ntri8 / 8;
    const int t = (b % 8) * per_xcd + b / 8;
    if (t >= args.ntri) return;
    int ti, tj;
    band_tile(t, args.nt, ti, tj);
    if (ti < 0) return;
    const int m0 = ti * C::BM;   // rows g' of the output (columns of P)
    const int n0 = tj * C::BN;   // columns g of the output (columns of Q)

    // Segment tables are built from scalar arguments in registers: taking a
    // reference into the by-value kernel argument would copy it to scratch.
    const long long ld = args.n_g;
    Acc<C> acc;
    if (isH) {
        // Z^H B + B^H Z + (W or A)^H W
        Segs<3, true, false> t;
        t.nseg = 3;
        t.len = args.K;
        t.ldp = t.ldq = ld;
        t.P[0] = args.Z;
        t.Q[0] = args.B;
        t.P[1] = args.B;
        t.Q[1] = args.Z;
        t.P[2] = args.W;
        t.Q[2] = args.W;
        t.palt = args.A;
        t.sel = args.sel;      // [3K]: 0 on the first two segments
        t.qscale = nullptr;
        ztile_direct<C, 3, true, false, G3>(t, m0, args.n_g, n0, args.n_g, acc, lds);
    } else {
        // A^H A + B^H diag(|u|^2) B
        Segs<2, false, true> t;
        t.nseg = 2;
        t.len = args.K;
        t.ldp = t.ldq = ld;
        t.P[0] = args.A;
        t.Q[0] = args.A;
        t.P[1] = args.B;
        t.Q[1] = args.B;
        t.palt = nullptr;
        t.sel = nullptr;
        t.qscale = args.d;     // [2K]: 1 on A's rows, |u|^2 on B's rows
        ztile_direct<C, 2, false, true, G3>(t, m0, args.n_g, n0, args.n_g, acc, lds);
    }

    double2 *out = isH ? args.H : args.S;
    const int n_g = args.n_g;
#pragma unroll
    for (int i = 0; i < C::TM; ++i)
#pragma unroll
        for (int j = 0; j < C::TN; ++j) {
            const int g = n0 + acc_col<C>(j);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gp = m0 + acc_row<C>(i, v);
                if (gp < n_g && g <= gp)
                    out[(long long)gp * n_g + g] = double2{acc.re[i][j][v], acc.im[i][j][v]};
            }
        }
}

// upper := conj(lower) through a 32x32 LDS transpose; Im(diag) := 0.
constexpr int MT = 32;
__global__ void __launch_bounds__(256)
k_mirror(double2 *H, double2 *S, int n_g) {
    const int bx = blockIdx.x, by = blockIdx.y;   // destination tile: rows by, cols bx
    if (bx < by) return;
    double2 *M = blockIdx.z == 0 ? H : S;
    __shared__ double2 tile[MT][MT + 1];
    const int tx = threadIdx.x % MT, ty = threadIdx.x / MT;   // 32 x 8
    // source: lower tile rows bx*32.., cols by*32..
    for (int r = ty; r < MT; r += 8) {
        const int gr = bx * MT + r, gc = by * MT + tx;
        if (gr < n_g && gc < n_g && gc <= gr) tile[r][tx] = M[(long long)gr * n_g + gc];
    }
    __syncthreads();
    for (int r = ty; r < MT; r += 8) {
        const int gr = by * MT + r, gc = bx * MT + tx;   // destination (gr, gc), gr <= gc
        if (gr < n_g && gc < n_g) {
            if (gr < gc) {
                double2 v = tile[tx][r];
                v.y = -v.y;
                M[(long long)gr * n_g + gc] = v;
            } else if (gr == gc) {
                M[(long long)gr * n_g + gc].y = 0.0;
            }
        }
    }
}

}  // namespace

hipError_t launch_reduce(int K, int n_g, const double2 *A, const double2 *B,
                         const double2 *Z, const double2 *W, const int *sel,
                         const double *d, double2 *H, double2 *S, hipStream_t st, bool g3) {
    using C = RedCfg;
    RedArgs args;
    args.A = A;
    args.B = B;
    args.Z = Z;
    args.W = W;
    args.sel = sel;
    args.d = d;
    args.K = K;
    args.H = H;
    args.S = S;
    args.n_g = n_g;
    args.nt = (n_g + C::BM - 1) / C::BM;
    args.ntri = args.nt * (args.nt + 1) / 2;
    args.ntri8 = (args.ntri + 7) / 8 * 8;
    if (g3)
        hipLaunchKernelGGL(k_reduce<true>, dim3(2 * args.ntri8), dim3(C::NT), 0, st, args);
    else
        hipLaunchKernelGGL(k_reduce<false>, dim3(2 * args.ntri8), dim3(C::NT), 0, st, args);
    return hipGetLastError();
}

hipError_t launch_mirror(double2 *H, double2 *S, int n_g, hipStream_t st) {
    const int mt = (n_g + MT - 1) / MT;
    hipLaunchKernelGGL(k_mirror, dim3(mt, mt, 2), dim3(256), 0, st, H, S, n_g);
    return hipGetLastError();
}

hipError_t launch_mirror1(double2 *M, int n, hipStream_t st) {
    const int mt = (n + MT - 1) / MT;
    hipLaunchKernelGGL(k_mirror, dim3(mt, mt, 1), dim3(256), 0, st, M, M, n);
    return hipGetLastError();
}

}  // namespace hs
