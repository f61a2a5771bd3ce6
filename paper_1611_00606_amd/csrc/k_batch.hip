// Batched form of the per-atom stage of Alg. 1 for atoms of mixed N_L: one
// persistent launch runs every atom's preparation (the Cholesky of T^AA_a
// with its failure test, prep_atom.h) and every atom's products
//   Z_a = T_AB,a^H A_a + M2_a^H B_a,   W_a = M1_a^H A_a   (Y_a or X_a)
// with the tile shape of each atom's products chosen per N_L (a table filled
// by the autotuner in hs_tune.hip, or the built-in choice below), on the
// per-atom tile engine of zmfma_atom.h.
//
// Work items, taken in order from one atomic counter by a grid of one
// 8-wave block per CU:
//   [0, N_A)              preparation of atom perm[i] (atoms by N_L, largest
//                         first, so the longest factorizations start first)
//   [N_A, N_A + nz)       Z tiles, atoms in the same order
//   [N_A + nz, N_A + 2nz) W tiles
// A Z tile needs M2_a and a W tile needs M1_a; the preparation item of atom a
// publishes each through a ready flag. An item only ever waits for an item
// with a smaller index, which some running block has already taken, so every
// wait ends; the wait is bounded nevertheless, and a wait that runs out is
// counted and turns every info entry to -1 (checked after the launch).
// With the preparation done elsewhere (the resident context caches it), the
// launch has product items only and nothing waits.
#include "prep_atom.h"
#include "zmfma_atom.h"

namespace hs {

namespace {

constexpr int BT = 512;   // threads of the persistent block (8 waves)

// Candidate tile shapes (BM rows of the atom's N_L x BN columns of N_G):
// 32, 64, 96 or 128 rows by 128 columns, 64 or 96 rows by 192 columns and
// 32 or 64 rows by 256 columns (the wider ones with stages of 8 rows, so
// that two stages fit the LDS). At most nine 16x16 blocks per wave (144
// accumulator registers).
using Cfg0 = AtomCfg<1, 2, 16>;   //  32 x 128
using Cfg1 = AtomCfg<2, 2, 16>;   //  64 x 128
using Cfg2 = AtomCfg<3, 2, 16>;   //  96 x 128
using Cfg3 = AtomCfg<4, 2, 16>;   // 128 x 128
using Cfg4 = AtomCfg<1, 4, 8>;    //  32 x 256
using Cfg5 = AtomCfg<2, 4, 8>;    //  64 x 256
using Cfg6 = AtomCfg<3, 3, 8>;    //  96 x 192
using Cfg7 = AtomCfg<2, 3, 8>;    //  64 x 192
static_assert(Cfg0::NT == BT && Cfg1::NT == BT && Cfg2::NT == BT && Cfg3::NT == BT &&
                  Cfg4::NT == BT && Cfg5::NT == BT && Cfg6::NT == BT && Cfg7::NT == BT,
              "every tile shape runs on the whole persistent block");
static_assert(HS_NUM_TILE_CONFIGS == 8, "tile table and candidate list agree");
static_assert(Cfg0::BM >= ATOM_TILE_MIN_BM && Cfg1::BM >= ATOM_TILE_MIN_BM &&
                  Cfg2::BM >= ATOM_TILE_MIN_BM && Cfg3::BM >= ATOM_TILE_MIN_BM &&
                  Cfg4::BM >= ATOM_TILE_MIN_BM && Cfg5::BM >= ATOM_TILE_MIN_BM &&
                  Cfg6::BM >= ATOM_TILE_MIN_BM && Cfg7::BM >= ATOM_TILE_MIN_BM &&
                  Cfg0::BN >= ATOM_TILE_MIN_BN && Cfg1::BN >= ATOM_TILE_MIN_BN &&
                  Cfg2::BN >= ATOM_TILE_MIN_BN && Cfg3::BN >= ATOM_TILE_MIN_BN &&
                  Cfg4::BN >= ATOM_TILE_MIN_BN && Cfg5::BN >= ATOM_TILE_MIN_BN &&
                  Cfg6::BN >= ATOM_TILE_MIN_BN && Cfg7::BN >= ATOM_TILE_MIN_BN,
              "the tile-position table is sized for these minima");

constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int TILE_LDS = 16 * cmax(cmax(cmax(Cfg0::LDS_ELEMS, Cfg1::LDS_ELEMS),
                                        cmax(Cfg2::LDS_ELEMS, Cfg3::LDS_ELEMS)),
                                   cmax(cmax(Cfg4::LDS_ELEMS, Cfg5::LDS_ELEMS),
                                        cmax(Cfg6::LDS_ELEMS, Cfg7::LDS_ELEMS)));
constexpr int BATCH_LDS = cmax(TILE_LDS, PREP_LDS_BYTES);
static_assert(BATCH_LDS <= 160 * 1024, "LDS of one CU");

constexpr int SPIN_LIMIT = 1 << 22;   // x ~1 us per poll: seconds

struct BatchArgs {
    Atoms at;
    const double2 *T_AA, *T_AB, *T_BB, *U, *A, *B;
    double2 *M1, *M2;
    double *d;
    int *sel, *info;
    double2 *Z, *W;
    const int *perm;   // [N_A] atom at each position
    const int *tiles;  // [2 nz] atom and tile index within the atom of each product tile
    int *ctrl;         // [0] item counter, [1] waits that ran out
    int *flags;        // [2 N_A] M2 ready, M1 ready
    int n_g, nz, do_factor;
    unsigned char cfg[HS_MAX_NL + 1];
};

template <class C>
__device__ __forceinline__ void product_tile(int which, bool failing, int r0, int n, long long t0,
                                             int loc,
                                             int n_g, const double2 *A, const double2 *B,
                                             const double2 *T_AB, const double2 *M1,
                                             const double2 *M2, double2 *Z, double2 *W,
                                             double2 *lds) {
    const int ct = (n_g + C::BN - 1) / C::BN;
    const int m0 = (loc / ct) * C::BM;
    const int n0 = (loc % ct) * C::BN;
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
        const int k0 = w_contraction_start(failing, m0);
        tab.nseg = 1;
        tab.len = n - k0;
        tab.P[0] = M1 + t0 + (long long)k0 * n;
        tab.Q[0] = Aa + (long long)k0 * n_g;
        tab.P[1] = tab.P[0];
        tab.Q[1] = tab.Q[0];
    }
    Acc<C> acc;
    ztile_atom<C, 2>(tab, m0, n, n0, n_g, which == 1 && !failing, acc, lds);

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

// The flag's value once set (nonzero), or 0 if the wait ran out.
__device__ __forceinline__ int wait_flag(const int *f) {
    for (int i = 0; i < SPIN_LIMIT; ++i) {
        if (const int v = __hip_atomic_load(f, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT)) return v;
        __builtin_amdgcn_s_sleep(8);
    }
    return 0;
}

__global__ void __launch_bounds__(BT)
k_batch(BatchArgs args) {
    __shared__ __align__(16) char lds[BATCH_LDS];
    // kind (-1 done, 0 prep, 1 Z, 2 W, 3 skipped), atom, tile, and for
    // tiles the atom's first row, N_L, first element of its blocks, and
    // whether its Cholesky failed
    __shared__ int s_job[7];

    const Atoms at = args.at;
    const int n_atoms = at.n_atoms;
    const int nz = args.nz;
    const int nf = args.do_factor ? n_atoms : 0;
    const int total = nf + 2 * nz;

    // Thread 0 claims and decodes the next item: the counter, then the tile
    // table, then the atom's offsets together with its ready flag (whose
    // value also tells whether the atom's Cholesky failed), so three
    // dependent memory round trips stand between two items.
    for (;;) {
        __syncthreads();   // the previous item is done with LDS and s_job
        if (threadIdx.x == 0) {
            const int it = atomicAdd(args.ctrl, 1);
            int kind = -1, atom = 0, loc = 0, r0 = 0, n = 0, t0 = 0, fail = 0;
            if (it < nf) {
                kind = 0;
                atom = args.perm[it];
            } else if (it < total) {
                int j = it - nf;
                kind = 1;
                if (j >= nz) {
                    kind = 2;
                    j -= nz;
                }
                atom = args.tiles[2 * j];
                loc = args.tiles[2 * j + 1];
                r0 = at.row_off[atom];
                n = at.row_off[atom + 1] - r0;
                t0 = at.t_off[atom];
                if (args.do_factor) {
                    const int f = wait_flag(args.flags + (kind == 1 ? atom : n_atoms + atom));
                    if (!f) {
                        atomicAdd(args.ctrl + 1, 1);
                        kind = 3;   // skipped
                    }
                    fail = f == 2;
                } else if (kind == 2) {
                    // prepared before the launch: the failure test's result is in sel
                    fail = args.sel[2 * at.K + r0] != 0;
                }
            }
            s_job[0] = kind;
            s_job[1] = atom;
            s_job[2] = loc;
            s_job[3] = r0;
            s_job[4] = n;
            s_job[5] = t0;
            s_job[6] = fail;
        }
        __syncthreads();
        const int kind = s_job[0], atom = s_job[1], loc = s_job[2];
        if (kind < 0) break;
        if (kind == 3) continue;
        if (kind == 0) {
            prep_atom<BT>(at, atom, args.T_AA, args.T_BB, args.U, args.M1, args.M2, args.d,
                          args.sel, args.info, lds, args.flags + atom,
                          args.flags + n_atoms + atom);
            continue;
        }
        // What the preparation published is visible to every wave here: thread
        // 0's agent-scope acquire of the ready flag (in wait_flag) is ordered
        // before the barrier above, after which the other waves load (the
        // acquire's cache invalidation acts on the CU's and the XCD's caches,
        // which all waves of the block share). A per-wave acquire of the same
        // flag cost one more memory round trip per item (6% of the stage).
        const int r0 = s_job[3];
        const int n = s_job[4];
        const long long t0 = s_job[5];
        const int which = kind - 1;
        // W tiles of an atom with a Cholesky factor contract a triangle only
        const bool failing = which == 1 && s_job[6] != 0;
        double2 *tl = reinterpret_cast<double2 *>(lds);
        switch (args.cfg[n]) {
            case 0:
                product_tile<Cfg0>(which, failing, r0, n, t0, loc, args.n_g, args.A, args.B, args.T_AB,
                                   args.M1, args.M2, args.Z, args.W, tl);
                break;
            case 1:
                product_tile<Cfg1>(which, failing, r0, n, t0, loc, args.n_g, args.A, args.B, args.T_AB,
                                   args.M1, args.M2, args.Z, args.W, tl);
                break;
            case 2:
                product_tile<Cfg2>(which, failing, r0, n, t0, loc, args.n_g, args.A, args.B, args.T_AB,
                                   args.M1, args.M2, args.Z, args.W, tl);
                break;
            case 3:
                product_tile<Cfg3>(which, failing, r0, n, t0, loc, args.n_g, args.A, args.B, args.T_AB,
                                   args.M1, args.M2, args.Z, args.W, tl);
                break;
            case 4:
                product_tile<Cfg4>(which, failing, r0, n, t0, loc, args.n_g, args.A, args.B, args.T_AB,
                                   args.M1, args.M2, args.Z, args.W, tl);
                break;
            case 5:
                product_tile<Cfg5>(which, failing, r0, n, t0, loc, args.n_g, args.A, args.B, args.T_AB,
                                   args.M1, args.M2, args.Z, args.W, tl);
                break;
            case 6:
                product_tile<Cfg6>(which, failing, r0, n, t0, loc, args.n_g, args.A, args.B, args.T_AB,
                                   args.M1, args.M2, args.Z, args.W, tl);
                break;
            default:
                product_tile<Cfg7>(which, failing, r0, n, t0, loc, args.n_g, args.A, args.B, args.T_AB,
                                   args.M1, args.M2, args.Z, args.W, tl);
                break;
        }
    }
}

// Item tables of one launch, written from kernel arguments (no host copy):
// a chunk of up to BT_CHUNK positions per launch; also clears the counter
// and the ready flags of the chunk's atoms.
constexpr int BT_CHUNK = 256;
struct BatchChunk {
    int perm[BT_CHUNK];
    int zoff[BT_CHUNK];
    int p0, n, last, n_atoms, nz;
};

__global__ void __launch_bounds__(256)
k_batch_tables(BatchChunk c, int *perm, int *zoff, int *ctrl, int *flags) {
    for (int i = threadIdx.x; i < c.n; i += blockDim.x) {
        perm[c.p0 + i] = c.perm[i];
        zoff[c.p0 + i] = c.zoff[i];
        flags[c.perm[i]] = 0;
        flags[c.n_atoms + c.perm[i]] = 0;
    }
    if (threadIdx.x == 0 && c.p0 == 0) {
        ctrl[0] = 0;
        ctrl[1] = 0;
    }
    if (threadIdx.x == 0 && c.last) zoff[c.n_atoms] = c.nz;
}

// Atom and tile index within the atom of every product tile (one block per
// position): the item loop then decodes a tile with one load instead of a
// search over zoff.
__global__ void __launch_bounds__(256) k_batch_tile_index(const int *perm, const int *zoff,
                                                          int *tiles) {
    const int p = blockIdx.x;
    const int atom = perm[p];
    for (int j = zoff[p] + threadIdx.x; j < zoff[p + 1]; j += 256) {
        tiles[2 * j] = atom;
        tiles[2 * j + 1] = j - zoff[p];
    }
}

// After a launch with preparation items: a wait that ran out marks the build.
__global__ void __launch_bounds__(256) k_batch_check(const int *ctrl, int *info, int n_atoms) {
    if (ctrl[1] == 0) return;
    for (int a = blockIdx.x * 256 + threadIdx.x; a < n_atoms; a += gridDim.x * 256) info[a] = -1;
}

}  // namespace

// Compute units of the current device (cached per device).
int num_cus() {
    static int cached[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (!cached[dev]) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            n < 1)
            n = 256;
        cached[dev] = n;
    }
    return cached[dev];
}

int tile_shape(int id, int *bm, int *bn) {
    static const int shapes[HS_NUM_TILE_CONFIGS][2] = {
        {Cfg0::BM, Cfg0::BN}, {Cfg1::BM, Cfg1::BN}, {Cfg2::BM, Cfg2::BN},
        {Cfg3::BM, Cfg3::BN}, {Cfg4::BM, Cfg4::BN}, {Cfg5::BM, Cfg5::BN},
        {Cfg6::BM, Cfg6::BN}, {Cfg7::BM, Cfg7::BN}};
    if (id < 0 || id >= HS_NUM_TILE_CONFIGS) return -1;
    if (bm) *bm = shapes[id][0];
    if (bn) *bn = shapes[id][1];
    return 0;
}

// Built-in choice: the tile with the fewest rows that cover N_L (one row
// tile per atom), 128 columns wide except for 96 rows, where 192 columns
// measured faster (2.40 against 2.50 ms for the stage at N_L = 81,
// N_G = 8000).
int default_tile(int nl) {
    return nl <= 32 ? 0 : nl <= 64 ? 1 : nl <= 96 ? 6 : 3;
}

void BatchPlan::make(const AtomPlan &p, int n_g, const unsigned char *cfg_table) {
    for (int v = 0; v <= HS_MAX_NL; ++v) cfg[v] = cfg_table ? cfg_table[v] : (unsigned char)default_tile(v);
    perm.resize(p.n_atoms);
    for (int a = 0; a < p.n_atoms; ++a) perm[a] = a;
    std::stable_sort(perm.begin(), perm.end(),
                     [&](int x, int y) { return p.nl[x] > p.nl[y]; });
    zoff.assign(p.n_atoms + 1, 0);
    long long acc = 0;
    for (int i = 0; i < p.n_atoms; ++i) {
        zoff[i] = (int)acc;
        const int n = p.nl[perm[i]];
        int bm = 0, bn = 0;
        tile_shape(cfg[n], &bm, &bn);
        acc += (long long)((n + bm - 1) / bm) * ((n_g + bn - 1) / bn);
    }
    zoff[p.n_atoms] = (int)acc;
    nz = acc;
}

bool BatchPlan::valid(const AtomPlan &p, const unsigned char *cfg_table) {
    if (!cfg_table) return true;
    for (int a = 0; a < p.n_atoms; ++a)
        if (cfg_table[p.nl[a]] >= HS_NUM_TILE_CONFIGS) return false;
    return true;
}

hipError_t launch_batch(const AtomPlan &p, const Atoms &at, const BatchPlan &bp, int n_g,
                        bool do_factor, const BatchIO &io, const BatchBufs &bb, hipStream_t st) {
    if (bp.nz > (1LL << 30) || bp.nz > BatchBufs::max_tiles(p.n_atoms, n_g))
        return hipErrorInvalidValue;
    for (int p0 = 0; p0 < p.n_atoms; p0 += BT_CHUNK) {
        BatchChunk c;
        c.p0 = p0;
        c.n = std::min(BT_CHUNK, p.n_atoms - p0);
        for (int i = 0; i < c.n; ++i) {
            c.perm[i] = bp.perm[p0 + i];
            c.zoff[i] = bp.zoff[p0 + i];
        }
        c.last = p0 + c.n == p.n_atoms;
        c.n_atoms = p.n_atoms;
        c.nz = (int)bp.nz;
        hipLaunchKernelGGL(k_batch_tables, dim3(1), dim3(256), 0, st, c, bb.perm, bb.zoff, bb.ctrl,
                           bb.flags);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_batch_tile_index, dim3(p.n_atoms), dim3(256), 0, st, bb.perm, bb.zoff,
                       bb.tiles);
    if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
    BatchArgs a;
    a.at = at;
    a.T_AA = io.T_AA;
    a.T_AB = io.T_AB;
    a.T_BB = io.T_BB;
    a.U = io.U;
    a.A = io.A;
    a.B = io.B;
    a.M1 = io.M1;
    a.M2 = io.M2;
    a.d = io.d;
    a.sel = io.sel;
    a.info = io.info;
    a.Z = io.Z;
    a.W = io.W;
    a.perm = bb.perm;
    a.tiles = bb.tiles;
    a.ctrl = bb.ctrl;
    a.flags = bb.flags;
    a.n_g = n_g;
    a.nz = (int)bp.nz;
    a.do_factor = do_factor ? 1 : 0;
    for (int v = 0; v <= HS_MAX_NL; ++v) a.cfg[v] = bp.cfg[v];
    const long long items = (do_factor ? p.n_atoms : 0) + 2 * bp.nz;
    const int grid = (int)std::min<long long>(num_cus(), items);
    hipLaunchKernelGGL(k_batch, dim3(grid), dim3(BT), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !do_factor) return e;
    hipLaunchKernelGGL(k_batch_check, dim3((p.n_atoms + 255) / 256), dim3(256), 0, st, bb.ctrl,
                       io.info, p.n_atoms);
    return hipGetLastError();
}

}  // namespace hs
