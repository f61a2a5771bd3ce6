// Modular INT8 form of the large reductions (HS_SPLIT_I8_CRT): the five
// stacked products of Alg. 1 (the zher2k, the two zherk of S, the
// failure-branch zgemm and the HPD zherk) computed exactly on integers.
//
// Operands. For each column n of a sliced operand X let e[n] be the exponent
// with max_k max(|Re X[k][n]|, |Im X[k][n]|) < 2^e[n], and
//     X'[k][n] = rint(X[k][n] 2^(b - 1 - e[n]))        (|X'| <= 2^(b-1))
// for the real and the imaginary parts. This rounding is the form's only
// error: at most 2^-b of the column maximum per element.
//
// Products. With real and imaginary parts interleaved along the contraction,
// P'' = (p_re, p_im), Q''_re = (q_re, q_im) and Q''_im = (q_im, -q_re), the
// real and the imaginary part of conj(P')^T Q' are each one dot product of 2K
// integers, so |Re|, |Im| <= 2K 2^(2b - 2). Both are computed modulo NMOD
// pairwise coprime odd moduli m_i <= 255: the operands' residues in symmetric
// form (|r| <= (m - 1) / 2 <= 127, so a residue and its negation are int8),
// INT8 MFMA products summed exactly in INT32 and reduced to a symmetric
// residue at the end of the segment. With M = prod m_i (about 2^86.8) and b
// chosen so that 2K 2^(2b - 2) <= (M - 1) / 2, the residues fix each integer
// uniquely in the symmetric range of M.
//
// Reconstruction (Chinese remainder theorem in Garner's mixed-radix form):
//     X = v_0 + m_0 (v_1 + m_1 (v_2 + ... + m_9 v_10)),
//     v_i = (r_i - sum_{j<i} v_j W_j) W_i^-1  mod m_i,   W_j = m_0 ... m_{j-1},
// with symmetric digits v_i, computed exactly in FP32 (every intermediate is
// an integer below 2^24) and evaluated by Horner's rule in FP64. Each
// segment's integer is scaled by 2^(eP + eQ - 2 (b - 1)) and the segments of
// H (three) and of S (two) are added in FP64.
//
// The scheme is the modular-integer emulation of floating-point matrix
// products of Ozaki, Uchino and Imamura ("Ozaki scheme II", 2025). Against
// the INT8 slice pairs of HS_SPLIT_I8 (15 INT8 products per complex product)
// it needs one per modulus (11), and the INT32 sums of a modulus need no
// per-level accumulators, so a wave holds a four times larger output tile.
#include "hs_internal.h"
#include "split_common.h"

namespace hs {

namespace {

typedef int i4 __attribute__((ext_vector_type(4)));

constexpr int NMOD = 11;
constexpr int CRT_MOD[NMOD] = {255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 217};
constexpr int CRT_BMAX = 36;   // |X'| <= 2^35: exact in FP64, and b = 36 for K up to about 5e4
constexpr int NSEG = 5;        // H: (Z,B), (B,Z), (P3,W); S: (A,A), (Bs,Bs)

// Garner constants, symmetric: w[i][j] = W_j mod m_i (j < i), u[i] = W_i^-1 mod m_i.
constexpr int sym_mod_c(long long x, int m) {
    long long r = x % m;
    if (r < 0) r += m;
    return r > m / 2 ? (int)(r - m) : (int)r;
}
constexpr int inv_mod_c(long long a, int m) {
    a %= m;
    if (a < 0) a += m;
    for (int x = 1; x < m; ++x)
        if (a * x % m == 1) return x;
    return 0;
}
struct GarnerTab {
    int w[NMOD][NMOD];
    int u[NMOD];
    int wu[NMOD][NMOD];   // w[i][j] u[i] mod m_i, symmetric
};
constexpr GarnerTab make_garner() {
    GarnerTab t{};
    for (int i = 0; i < NMOD; ++i) {
        long long wm = 1;   // W_j mod m_i
        for (int j = 0; j < i; ++j) {
            t.w[i][j] = sym_mod_c(wm, CRT_MOD[i]);
            wm = wm * CRT_MOD[j] % CRT_MOD[i];
        }
        t.u[i] = sym_mod_c(inv_mod_c(wm, CRT_MOD[i]), CRT_MOD[i]);
        for (int j = 0; j < i; ++j) t.wu[i][j] = sym_mod_c((long long)t.w[i][j] * t.u[i], CRT_MOD[i]);
    }
    return t;
}
constexpr GarnerTab GT = make_garner();
static_assert(GT.u[0] == 1 && ((long long)GT.u[1] * 255 % 253 + 253) % 253 == 1, "Garner table");
// a digit's sum r_i u_i - sum_{j<i} wu[i][j] v_j is an integer below 2^24
static_assert(NMOD * 127 * 127 < (1 << 24), "Garner sums exact in FP32");
// three symmetric digits fold into an integer below 2^24 (exact in FP32)
static_assert(255LL * 253 * 251 / 2 < (1 << 24), "digit groups exact in FP32");

__device__ __forceinline__ int crt_modulus(int mi) {
    int m = CRT_MOD[0];
#pragma unroll
    for (int i = 1; i < NMOD; ++i)
        if (mi == i) m = CRT_MOD[i];
    return m;
}

// ---------------------------------------------------------------------------
// Residues. One thread per (group of 8 complex rows, column): 16 interleaved
// real values -> b-bit integers -> NMOD residues of 16 int8, written to
// R[i][g][n][0..15].

__global__ void __launch_bounds__(256)
k_residue(SliceSrc src, int K, int n_g, int groups, int b) {
    const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
    const int n = (int)(idx % n_g);
    const int g = (int)(idx / n_g);
    if (g >= groups) return;
    const int sh = b - 1 - col_exp(src.mx, n);
    double x[16];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int k = 8 * g + q;
        double2 v = {0.0, 0.0};
        if (k < K) v = slice_src_row(src, k, n_g, n);
        x[2 * q] = rint(ldexp(v.x, sh));
        x[2 * q + 1] = rint(ldexp(v.y, sh));
    }
    const long long plane = (long long)groups * n_g;   // 16-byte items per modulus
    uint4 *out = reinterpret_cast<uint4 *>(src.S) + (long long)g * n_g + n;
#pragma unroll
    for (int i = 0; i < NMOD; ++i) {
        // x / m is at most 2^28 and at least 1 / (2 m) from a half-integer,
        // so rint of the rounded quotient is exact and so is the remainder
        const double m = CRT_MOD[i], inv = 1.0 / CRT_MOD[i];
        unsigned w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const double r = fma(-m, rint(x[j] * inv), x[j]);
            w[j >> 2] |= ((unsigned)(int)r & 0xffu) << (8 * (j & 3));
        }
        out[i * plane] = uint4{w[0], w[1], w[2], w[3]};
    }
}

// ---------------------------------------------------------------------------
// Products modulo one modulus. One block per (128 x 128 lower-triangle tile,
// segment, modulus): 4 waves of 64 x 64 outputs (4 x 4 MFMA blocks of
// 16 x 16, Re and Im: 128 accumulator registers), two blocks per CU (two
// waves per SIMD). A stage is 64 complex rows: 8 items of 16 bytes per
// column and operand, moved global -> LDS with 16-byte direct loads, two
// 32 KiB buffers (the next stage loads while the current one is
// multiplied). The INT32 sums stay exact for CFOLD stages (checked below);
// longer segments reduce them modulo m every CFOLD stages.
//
// Measured at N_G = 8000 (K = 8100): against 8 waves of 64 x 32 outputs in
// 128-row stages (one block per CU) this shape reads a third less from LDS
// per MFMA and is 9% faster; deeper pipelines (3 to 5 buffers, up to four
// stages in flight) are not faster: the kernel runs INT8 MFMA at a reduced
// clock (about 1.74 GHz by the cycle counters), not waiting on operands.
// Bands of 8 tile columns in the tile order (64 tiles resident per XCD
// share 8 row and 8 column panels) fetch 15% less than bands of 4.

constexpr int CB = 128;                    // tile rows (g') and columns (g)
constexpr int CWM = 2, CWN = 2;            // waves
constexpr int CNT = 64 * CWM * CWN;
constexpr int CTM = CB / CWM / 16, CTN = CB / CWN / 16;   // 16 x 16 blocks per wave
constexpr int CKS = 2;                     // MFMA K steps (32 complex rows) per stage
constexpr int CITEMS = 4 * CKS;            // items per column and stage
constexpr int COP = CITEMS * CB;           // items per operand and stage
constexpr int CBUF = 2 * COP;
constexpr int CFOLD = 1024;                // stages between reductions of the sums
constexpr int CBAND = 8;
constexpr int CFRAG = CWM * CWN * CTM * CTN;   // 16 x 16 blocks per tile (64)
constexpr int CWAVES_EU = 2;               // waves per SIMD (at most 256 registers each)
constexpr int CNBUF = 2;                   // LDS stage buffers: CNBUF - 1 stages in flight
constexpr int CHW = CWM * CWN / 2;         // loader waves per operand
constexpr int CLPW = 2 * CITEMS / CHW;     // direct loads per wave and stage
static_assert((long long)CFOLD * CITEMS * 16 * 127 * 127 + 127 < (1LL << 31), "INT32 sums exact");
static_assert(CFRAG == 64, "the residue layout assumes 64 blocks per tile");

struct CrtArgs {
    const uint4 *P[NSEG], *Q[NSEG];   // residue planes of modulus 0 per segment
    uint2 *out;                        // [NSEG * NMOD][ntri][CFRAG][64 lanes]
    long long plane;                   // items per modulus plane
    int n_g, groups, nt, ntri, ntri8;
};

// symmetric residue of an INT32 sum (exact: the quotient is below 2^24 and at
// least 1 / (2 m) from a half-integer)
__device__ __forceinline__ int sym_res(int x, double m, double inv) {
    const double d = (double)x;
    return (int)fma(-m, rint(d * inv), d);
}

__global__ void __launch_bounds__(CNT) __attribute__((amdgpu_waves_per_eu(CWAVES_EU)))
k_crt_reduce(CrtArgs args) {
    __shared__ uint4 bufs[CNBUF * CBUF];

    const int job = blockIdx.y;
    const int seg = job / NMOD, mi = job - seg * NMOD;
    const int bx = blockIdx.x;
    const int per_xcd = args.ntri8 / 8;
    const int t = (bx % 8) * per_xcd + bx / 8;
    if (t >= args.ntri) return;
    int ti, tj;
    sband_tile(t, args.nt, ti, tj, CBAND);
    if (ti < 0) return;
    const int n_g = args.n_g;
    const int m0 = ti * CB, n0 = tj * CB;
    // the segment's planes, selected with constant indices (a dynamic index
    // into the argument block would copy it to scratch memory)
    const uint4 *P = args.P[0], *Q = args.Q[0];
#pragma unroll
    for (int s = 1; s < NSEG; ++s)
        if (seg == s) {
            P = args.P[s];
            Q = args.Q[s];
        }
    P += mi * args.plane;
    Q += mi * args.plane;
    const double m = crt_modulus(mi);
    const double minv = 1.0 / m;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave % CWM, wn = wave / CWM;

    // loader: the first half of the waves fills P's item rows, the second
    // half Q's; wave w of a half takes rows w, w + CHW, w + 2 CHW, ..., both
    // 64-column halves of each; columns past the edge read the last column
    // (they only feed outputs past N_G, never used)
    static_assert(CB == 128 && CITEMS % CHW == 0, "the loader's split of the stage");
    const int op_w = wave / CHW, row_w = wave % CHW;
    const int cb = (op_w == 0 ? m0 : n0) + lane;
    const unsigned o0 = (unsigned)(cb < n_g ? cb : n_g - 1) * 16u;
    const unsigned o1 = (unsigned)(cb + 64 < n_g ? cb + 64 : n_g - 1) * 16u;
    const uint4 *ldsrc = op_w == 0 ? P : Q;
    auto issue = [&](uint4 *buf, int st) __attribute__((always_inline)) {
        uint4 *dst = buf + op_w * COP + row_w * CB;
        const uint4 *rows = ldsrc + (long long)(st * CITEMS + row_w) * n_g;
#pragma unroll
        for (int i = 0; i < CITEMS / CHW; ++i) {
            const char *r = reinterpret_cast<const char *>(rows + (long long)(CHW * i) * n_g);
            __builtin_amdgcn_global_load_lds(reinterpret_cast<const uint4 *>(r + o0),
                                             dst + CHW * i * CB, 16, 0, 0);
            __builtin_amdgcn_global_load_lds(reinterpret_cast<const uint4 *>(r + o1),
                                             dst + CHW * i * CB + 64, 16, 0, 0);
        }
    };

    i4 accr[CTM][CTN], acci[CTM][CTN];
#pragma unroll
    for (int i = 0; i < CTM; ++i)
#pragma unroll
        for (int j = 0; j < CTN; ++j) {
            accr[i][j] = i4{0, 0, 0, 0};
            acci[i][j] = i4{0, 0, 0, 0};
        }
    const int lg = lane >> 4, lc = lane & 15;
    auto compute = [&](const uint4 *buf) __attribute__((always_inline)) {
        const uint4 *lp = buf;
        const uint4 *lq = buf + COP;
#pragma unroll
        for (int kk = 0; kk < CKS; ++kk) {
            i4 a[CTM];
#pragma unroll
            for (int i = 0; i < CTM; ++i)
                a[i] = __builtin_bit_cast(i4, lp[(kk * 4 + lg) * CB + wm * (CB / CWM) + i * 16 + lc]);
#pragma unroll
            for (int j = 0; j < CTN; ++j) {
                const uint4 u = lq[(kk * 4 + lg) * CB + wn * (CB / CWN) + j * 16 + lc];
                const i4 bq = __builtin_bit_cast(i4, u);
                const i4 bi = i4{(int)im_pairs(u.x), (int)im_pairs(u.y), (int)im_pairs(u.z),
                                 (int)im_pairs(u.w)};
#pragma unroll
                for (int i = 0; i < CTM; ++i) {
                    accr[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[i], bq, accr[i][j], 0, 0, 0);
                    acci[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[i], bi, acci[i][j], 0, 0, 0);
                }
            }
        }
    };
    auto fold = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < CTM; ++i)
#pragma unroll
            for (int j = 0; j < CTN; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    accr[i][j][v] = sym_res(accr[i][j][v], m, minv);
                    acci[i][j][v] = sym_res(acci[i][j][v], m, minv);
                }
    };

    const int nstage = args.groups / CITEMS;
#pragma unroll
    for (int s = 0; s < CNBUF - 1; ++s)
        if (s < nstage) issue(bufs + s * CBUF, s);
    for (int st = 0; st < nstage; ++st) {
        // this wave's loads of stage st are done (those of up to CNBUF - 2
        // later stages may still be in flight); after the barrier every
        // wave's are, and every wave has finished the stage before, whose
        // buffer is refilled next
        if (st + CNBUF - 2 < nstage)
            asm volatile("s_waitcnt vmcnt(%0)" ::"n"((CNBUF - 2) * CLPW) : "memory");
        else
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        // a plain barrier: __syncthreads() would also wait for the later
        // stages' loads (its fence covers every outstanding memory access)
        asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
        // the buffer being computed and the one being loaded are distinct:
        // saying so (restrict) keeps the compiler from waiting for the
        // direct loads before every LDS read of the stage
        auto stage = [&](const uint4 *__restrict__ cur, uint4 *__restrict__ nxt)
                         __attribute__((always_inline)) {
            if (st + CNBUF - 1 < nstage) issue(nxt, st + CNBUF - 1);
            compute(cur);
        };
        stage(bufs + (st % CNBUF) * CBUF, bufs + ((st + CNBUF - 1) % CNBUF) * CBUF);
        if ((st + 1) % CFOLD == 0) fold();
    }
    fold();

    // residues of the 4 rows (4 lg + v) of column lc of every 16 x 16 block:
    // Re in x, Im in y, one byte per row, stored as r + 127 (0 .. 254)
    uint2 *out = args.out + ((long long)job * args.ntri + t) * CFRAG * 64;
#pragma unroll
    for (int i = 0; i < CTM; ++i)
#pragma unroll
        for (int j = 0; j < CTN; ++j) {
            unsigned re = 0u, im = 0u;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                re |= (unsigned)(accr[i][j][v] + 127) << (8 * v);
                im |= (unsigned)(acci[i][j][v] + 127) << (8 * v);
            }
            out[(wave * CTM * CTN + i * CTN + j) * 64 + lane] = uint2{re, im};
        }
}

// ---------------------------------------------------------------------------
// Reconstruction: one thread per (tile, 16 x 16 block, lane) of H or S, i.e.
// 4 outputs (rows 4 lg + v, column lc) as laid out by k_crt_reduce.

struct CrtRecArgs {
    const uint2 *res;
    const unsigned long long *mP[NSEG], *mQ[NSEG];
    double2 *H, *S;
    int n_g, nt, ntri, b;
};

// The integer with residues rb[i] - 127 (rb: the stored bytes). Digit i is
// (r_i u_i - sum_{j<i} (W_j u_i mod m_i) v_j) mod m_i, one reduction per
// digit; digits are folded three at a time in FP32 (exact) and the four
// groups by Horner's rule in FP64.
__device__ __forceinline__ double garner(const float (&rb)[NMOD]) {
    float v[NMOD];
    v[0] = rb[0] - 127.0f;
#pragma unroll
    for (int i = 1; i < NMOD; ++i) {
        const float mf = (float)CRT_MOD[i];
        const float inv = 1.0f / (float)CRT_MOD[i];
        float s = fmaf(rb[i], (float)GT.u[i], -127.0f * (float)GT.u[i]);     // r_i u_i
#pragma unroll
        for (int j = 0; j < i; ++j) s = fmaf(-(float)GT.wu[i][j], v[j], s);  // |s| < 2^24
        v[i] = fmaf(-mf, rintf(s * inv), s);                                  // |v_i| <= 127
    }
    auto fold3 = [&](int i) __attribute__((always_inline)) {   // v_i + m_i (v_i+1 + m_i+1 v_i+2)
        return fmaf((float)CRT_MOD[i], fmaf((float)CRT_MOD[i + 1], v[i + 2], v[i + 1]), v[i]);
    };
    const double g0 = fold3(0), g1 = fold3(3), g2 = fold3(6);
    const double g3 = fmaf((float)CRT_MOD[9], v[10], v[9]);
    constexpr double P3 = (double)CRT_MOD[0] * CRT_MOD[1] * CRT_MOD[2];
    constexpr double P6 = (double)CRT_MOD[3] * CRT_MOD[4] * CRT_MOD[5];
    constexpr double P9 = (double)CRT_MOD[6] * CRT_MOD[7] * CRT_MOD[8];
    static_assert(NMOD == 11, "the digit grouping assumes 11 moduli");
    return fma(fma(fma(g3, P9, g2), P6, g1), P3, g0);
}

__global__ void __launch_bounds__(256)
k_crt_recon(CrtRecArgs a) {
    const long long id = (long long)blockIdx.x * 256 + threadIdx.x;
    const bool isH = blockIdx.y == 0;
    const int lane = (int)(id & 63);
    const int f = (int)((id >> 6) % CFRAG);
    const int t = (int)(id / (64 * CFRAG));
    if (t >= a.ntri) return;
    int ti, tj;
    sband_tile(t, a.nt, ti, tj, CBAND);
    if (ti < 0) return;
    const int wave = f / (CTM * CTN), i = (f % (CTM * CTN)) / CTN, j = f % CTN;
    const int wm = wave % CWM, wn = wave / CWM;
    const int lg = lane >> 4, lc = lane & 15;
    const int n_g = a.n_g;
    const int g = tj * CB + wn * (CB / CWN) + j * 16 + lc;
    const int gp0 = ti * CB + wm * (CB / CWM) + i * 16 + 4 * lg;
    if (g >= n_g || gp0 >= n_g || g > gp0 + 3) return;   // no output of the lower triangle

    double sr[4] = {0.0, 0.0, 0.0, 0.0}, si[4] = {0.0, 0.0, 0.0, 0.0};
    auto segment = [&](int s, const unsigned long long *mP, const unsigned long long *mQ)
                       __attribute__((always_inline)) {
        uint2 w[NMOD];
#pragma unroll
        for (int mi = 0; mi < NMOD; ++mi)
            w[mi] = a.res[(((long long)(s * NMOD + mi) * a.ntri + t) * CFRAG + f) * 64 + lane];
        const int eq = col_exp(mQ, g);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            float rr[NMOD], ri[NMOD];
#pragma unroll
            for (int mi = 0; mi < NMOD; ++mi) {
                rr[mi] = (float)((w[mi].x >> (8 * v)) & 0xffu);
                ri[mi] = (float)((w[mi].y >> (8 * v)) & 0xffu);
            }
            const int gp = gp0 + v < n_g ? gp0 + v : n_g - 1;
            const int sh = col_exp(mP, gp) + eq - 2 * (a.b - 1);
            sr[v] += ldexp(garner(rr), sh);
            si[v] += ldexp(garner(ri), sh);
        }
    };
    if (isH) {
        segment(0, a.mP[0], a.mQ[0]);
        segment(1, a.mP[1], a.mQ[1]);
        segment(2, a.mP[2], a.mQ[2]);
    } else {
        segment(3, a.mP[3], a.mQ[3]);
        segment(4, a.mP[4], a.mQ[4]);
    }
    double2 *out = isH ? a.H : a.S;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int gp = gp0 + v;
        if (gp < n_g && g <= gp) out[(long long)gp * n_g + g] = double2{sr[v], si[v]};
    }
}

int crt_tiles(int n_g, int *nt) {
    *nt = (n_g + CB - 1) / CB;
    return *nt * (*nt + 1) / 2;
}

}  // namespace

int crt_bits(int K) {
    unsigned __int128 M = 1;
    for (int i = 0; i < NMOD; ++i) M *= (unsigned)CRT_MOD[i];
    const unsigned __int128 half = (M - 1) / 2;
    int b = CRT_BMAX;
    while (b > 1 && (unsigned __int128)(2 * (long long)K) << (2 * (b - 1)) > half) --b;
    return b;
}

size_t crt_residue_bytes(int K, int n_g) {
    const long long groups = (long long)((K + CITEMS * 8 - 1) / (CITEMS * 8)) * CITEMS;
    return (size_t)NMOD * groups * n_g * 16;
}

size_t crt_work_bytes(int n_g) {
    int nt;
    const long long ntri = crt_tiles(n_g, &nt);
    return (size_t)NSEG * NMOD * ntri * CFRAG * 64 * sizeof(uint2);
}

hipError_t launch_residue(const SliceSrc &src, int K, int n_g, hipStream_t st) {
    const int groups = (K + CITEMS * 8 - 1) / (CITEMS * 8) * CITEMS;
    hipError_t e = launch_colmax(src, K, n_g, st);
    if (e != hipSuccess) return e;
    const long long items = (long long)groups * n_g;
    hipLaunchKernelGGL(k_residue, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, st, src, K,
                       n_g, groups, crt_bits(K));
    return hipGetLastError();
}

hipError_t launch_crt_reduce(int K, int n_g, const SliceView (&hseg)[3][2],
                             const SliceView (&sseg)[2][2], void *work, double2 *H, double2 *S,
                             hipStream_t st) {
    auto u4 = [](const _Float16 *p) { return reinterpret_cast<const uint4 *>(p); };
    const SliceView *segs[NSEG] = {hseg[0], hseg[1], hseg[2], sseg[0], sseg[1]};
    CrtArgs a;
    CrtRecArgs r;
    for (int s = 0; s < NSEG; ++s) {
        a.P[s] = u4(segs[s][0].S);
        a.Q[s] = u4(segs[s][1].S);
        r.mP[s] = segs[s][0].mx;
        r.mQ[s] = segs[s][1].mx;
    }
    a.out = reinterpret_cast<uint2 *>(work);
    a.n_g = n_g;
    a.groups = (K + CITEMS * 8 - 1) / (CITEMS * 8) * CITEMS;
    a.plane = (long long)a.groups * n_g;
    a.ntri = crt_tiles(n_g, &a.nt);
    a.ntri8 = (a.ntri + 7) / 8 * 8;
    hipLaunchKernelGGL(k_crt_reduce, dim3(a.ntri8, NSEG * NMOD), dim3(CNT), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    r.res = a.out;
    r.H = H;
    r.S = S;
    r.n_g = n_g;
    r.nt = a.nt;
    r.ntri = a.ntri;
    r.b = crt_bits(K);
    const long long threads = (long long)a.ntri * CFRAG * 64;
    hipLaunchKernelGGL(k_crt_recon, dim3((unsigned)((threads + 255) / 256), 2), dim3(256), 0, st, r);
    return hipGetLastError();
}

}  // namespace hs
