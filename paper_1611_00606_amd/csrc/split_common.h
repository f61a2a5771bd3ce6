// Device helpers shared by the split-precision reductions (k_split.hip) and
// the modular INT8 form (k_crt.hip): the sliced operand's rows, column
// exponents, the (Re, Im) -> (Im, -Re) byte-pair form and the banded
// lower-triangle tile order.
#pragma once

#include "hs_internal.h"

namespace hs {

// Row k, column n of a sliced operand: X (or Xalt where sel[k] != 0),
// optionally scaled by sqrt(rscale[k]).
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

// exponent e with column max < 2^e (0 for an all-zero column)
__device__ __forceinline__ int col_exp(const unsigned long long *mx, int n) {
    const double m = __longlong_as_double((long long)mx[n]);
    int e = 0;
    if (m > 0.0) frexp(m, &e);
    return e;
}

// (Re, Im) int8 byte pairs -> (Im, -Re): conj(p) q's imaginary part as a dot
// product. The bytes must not hold -128.
__device__ __forceinline__ unsigned im_pairs(unsigned d) {
    typedef unsigned short us2 __attribute__((ext_vector_type(2)));
    const unsigned t = __builtin_amdgcn_perm(d, d, 0x02030001u) ^ 0xff00ff00u;
    us2 h = __builtin_bit_cast(us2, t);
    h += us2{0x0100, 0x0100};   // per 16-bit half: high byte ~b + 1 = -b, no carry across
    return __builtin_bit_cast(unsigned, h);
}

// Tile (i, j), j <= i, at position t of the banded order over an nt x nt
// lower triangle of tiles: bands of `band` tile columns, each band walked
// from its diagonal triangle down; (-1, -1) past the end.
__device__ __forceinline__ void sband_tile(int t, int nt, int &ti, int &tj, int band) {
    int c0 = 0;
    for (;;) {
        const int m = nt - c0;
        if (m <= 0) {
            ti = tj = -1;
            return;
        }
        const int w = m < band ? m : band;
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
        c0 += band;
    }
}

}  // namespace hs
