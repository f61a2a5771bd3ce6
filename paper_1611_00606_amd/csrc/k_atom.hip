// Per-atom products of Alg. 1, as complex MFMA tiles:
//   first loop     Z_a = T^BA_a A_a + 1/2 T^BB_a B_a = T_AB,a^H A_a + M2_a^H B_a
//   second loop    W_a = M1_a^H A_a  = C_a^H A_a (success, Y_a; C_a lower
//                                    triangular, so a row tile's contraction
//                                    starts at its first row)
//                                    or T^AA_a A_a (failure, X_a)
// with M1, M2 prepared by k_prep (M2 = 1/2 T^BB_a and, on failure,
// M1 = T^AA_a, both Hermitian, so M^H = M).
//
// Each block computes a BM x BN tile of one atom's N_L x N_G output (one
// tile covers all of an atom's rows, BM >= N_L); the contraction runs over
// the atom's N_L rows (twice for Z). The grid is (N_G tiles, atoms x row
// tiles, 2 products); Z and W land in the stacked [K][N_G] layout that the
// large reductions read.
#include "hs_internal.h"
#include "zmfma_atom.h"

namespace hs {

namespace {

template <class C>
__global__ void __launch_bounds__(C::NT)
k_atom(Atoms at, int n_g, int mtiles, const double2 *__restrict__ A,
       const double2 *__restrict__ B, const double2 *__restrict__ T_AB,
       const double2 *__restrict__ M1, const double2 *__restrict__ M2,
       const int *__restrict__ sel, double2 *__restrict__ Z, double2 *__restrict__ W) {
    __shared__ double2 lds[C::LDS_ELEMS];

    const int a = blockIdx.y / mtiles;
    const int mt = blockIdx.y % mtiles;
    const int which = blockIdx.z;  // 0: Z, 1: W
    const int r0 = at.row_off[a];
    const int n = at.row_off[a + 1] - r0;
    const int m0 = mt * C::BM;
    if (m0 >= n) return;  // atom has fewer rows than this row tile (mixed N_L)
    const long long t0 = at.t_off[a];
    const int n0 = blockIdx.x * C::BN;

    const double2 *Aa = A + (long long)r0 * n_g;
    const double2 *Ba = B + (long long)r0 * n_g;
    Segs<2, false, false> tab;
    tab.ldp = n;
    tab.ldq = n_g;
    tab.len = n;
    tab.palt = nullptr;
    tab.sel = nullptr;
    tab.qscale = nullptr;
    if (which == 0) {
        tab.nseg = 2;
        tab.P[0] = T_AB + t0;
        tab.Q[0] = Aa;
        tab.P[1] = M2 + t0;
        tab.Q[1] = Ba;
    } else {
        const int k0 = w_contraction_start(sel[2 * at.K + r0] != 0, m0);
        tab.nseg = 1;
        tab.len = n - k0;
        tab.P[0] = M1 + t0 + (long long)k0 * n;
        tab.Q[0] = Aa + (long long)k0 * n_g;
        tab.P[1] = tab.P[0];
        tab.Q[1] = tab.Q[0];
    }

    const bool tri = which == 1 && sel[2 * at.K + r0] == 0;
    Acc<C> acc;
    ztile_atom<C, 2>(tab, m0, n, n0, n_g, tri, acc, lds);

    double2 *out = (which == 0 ? Z : W) + (long long)r0 * n_g;
#pragma unroll
    for (int i = 0; i < C::TM; ++i)
#pragma unroll
        for (int j = 0; j < C::TN; ++j) {
            const int g = n0 + atom_col<C>(j);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int l = m0 + atom_row<C>(i, v);
                if (l < n && g < n_g) out[(long long)l * n_g + g] = double2{acc.re[i][j][v], acc.im[i][j][v]};
            }
        }
}

template <class C>
hipError_t launch_atom_cfg(const Atoms &at, int n_g, const double2 *A, const double2 *B,
                           const double2 *T_AB, const double2 *M1, const double2 *M2,
                           const int *sel, double2 *Z, double2 *W, hipStream_t st) {
    const int mtiles = (at.max_nl + C::BM - 1) / C::BM;
    dim3 grid((n_g + C::BN - 1) / C::BN, at.n_atoms * mtiles, 2);
    hipLaunchKernelGGL(k_atom<C>, grid, dim3(C::NT), 0, st, at, n_g, mtiles, A, B, T_AB, M1,
                       M2, sel, Z, W);
    return hipGetLastError();
}

}  // namespace

// Row tile of 32, 64, 96 or 128 (the smallest that covers the largest N_L),
// 128 columns (192 for the 96-row tile, as in the batched launch's
// built-in choice).
hipError_t launch_atom(const Atoms &at, int n_g, const double2 *A, const double2 *B,
                       const double2 *T_AB, const double2 *M1, const double2 *M2,
                       const int *sel, double2 *Z, double2 *W, hipStream_t st) {
    if (at.max_nl <= 32)
        return launch_atom_cfg<AtomCfg<1, 2, 16>>(at, n_g, A, B, T_AB, M1, M2, sel, Z, W, st);
    if (at.max_nl <= 64)
        return launch_atom_cfg<AtomCfg<2, 2, 16>>(at, n_g, A, B, T_AB, M1, M2, sel, Z, W, st);
    if (at.max_nl <= 96)
        return launch_atom_cfg<AtomCfg<3, 3, 8>>(at, n_g, A, B, T_AB, M1, M2, sel, Z, W, st);
    return launch_atom_cfg<AtomCfg<4, 2, 16>>(at, n_g, A, B, T_AB, M1, M2, sel, Z, W, st);
}

}  // namespace hs
