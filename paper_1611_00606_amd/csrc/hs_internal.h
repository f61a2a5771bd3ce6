// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/hs_build.h"

namespace hs {

// Device-side description of the atoms of one build.
struct Atoms {
    const int *row_off;  // [N_A+1] first row of each atom in A, B, U, Z, W
    const int *t_off;    // [N_A+1] first element of each atom's N_L x N_L block
    int n_atoms;
    int max_nl;
    int K;               // total rows
};

// Per-atom preparation (Alg. 1 second loop's factorization, plus the
// operand forms the products need). One block per atom.
//   info[a]   0 or the 1-based failing pivot of T_AA,a's Cholesky
//   M1_a      C_a (lower, zero above) on success, else T_AA,a as a full
//             Hermitian matrix from its lower triangle
//   M2_a      1/2 T_BB,a as a full Hermitian matrix from its lower triangle
//   d[2K]     per contraction row of the S reduction (A rows, then B rows):
//             d[r] = 1, d[K + r] = |U[r]|^2
//   sel[3K]   per contraction row of the H reduction (Z, B, then W rows):
//             sel[r] = sel[K + r] = 0, sel[2K + r] = 1 when row r belongs to
//             an atom on the failure branch (its left operand is then A)
hipError_t launch_prep(const Atoms &at, const double2 *T_AA, const double2 *T_BB,
                       const double2 *U, double2 *M1, double2 *M2, double *d,
                       int *sel, int *info, hipStream_t st);

// Per-atom products (Alg. 1 first loop and second-loop branches):
//   Z_a = T_AB,a^H A_a + M2_a^H B_a      (= T^BA_a A_a + 1/2 T^BB_a B_a)
//   W_a = M1_a^H A_a                     (= Y_a or X_a)
// sel: the preparation's [3K] row selectors (sel[2K + r] != 0 on the rows of
// atoms on the failure branch); on the other atoms M1_a = C_a is lower
// triangular and W_a's rows contract only over l >= their own index.
hipError_t launch_atom(const Atoms &at, int n_g, const double2 *A, const double2 *B,
                       const double2 *T_AB, const double2 *M1, const double2 *M2,
                       const int *sel, double2 *Z, double2 *W, hipStream_t st);

// Start of the contraction of a W_a tile whose output rows begin at m0: with
// C_a lower triangular, conj(C_a[l][m]) is zero for l < m, so rows l < m0
// add nothing to rows m >= m0 (the product is a triangular multiply); the
// failure branch's Hermitian T^AA_a is full.
__device__ __forceinline__ int w_contraction_start(bool failing, int m0) {
    return failing ? 0 : m0;
}

// Large reductions (Alg. 1's zher2k, zherk pair of S, failure-branch zgemm
// and HPD zherk) into the lower triangles of H and S (complex FP64 MFMA;
// g3: 3 real products per complex product instead of 4).
hipError_t launch_reduce(int K, int n_g, const double2 *A, const double2 *B,
                         const double2 *Z, const double2 *W, const int *sel,
                         const double *d, double2 *H, double2 *S, hipStream_t st, bool g3);

// Error bookkeeping shared by the C entry points (thread-local message).
void set_error(int status, const std::string &msg);
const char *message_for(int status);   // the last message if it explains `status`, else NULL
int hip_fail(hipError_t e, const char *where);   // records the message, returns HS_ERR_HIP
int check_device();                              // HS_OK on gfx950, else an error status
int num_cus();                                   // compute units of the current device
inline bool valid_mode(int mode) {   // HS_FP64 .. HS_SPLIT_I8_CRT
    return mode == HS_FP64 || mode == HS_SPLIT_F16 || mode == HS_SPLIT_I8 || mode == HS_FP64_3M ||
           mode == HS_SPLIT_BF16 || mode == HS_SPLIT_I8_CRT;
}
inline bool split_mode(int mode) {   // the operands are sliced (or cut into residues)
    return mode == HS_SPLIT_F16 || mode == HS_SPLIT_I8 || mode == HS_SPLIT_BF16 ||
           mode == HS_SPLIT_I8_CRT;
}

// Split-precision reductions (k_split.hip). A sliced operand: rows of X (or
// of Xalt where sel[k] != 0), optionally scaled by sqrt(rscale[k]); outputs
// the column maxima mx [N_G] (bit patterns of doubles) and the FP16 slices
// S [4][groups][N_G][8], groups = 4 * ceil(K / 16).
struct SliceSrc {
    const double2 *X;
    const double2 *Xalt;
    const int *sel;
    const double *rscale;
    unsigned long long *mx;
    _Float16 *S;
};
struct SliceView {
    const _Float16 *S;
    const unsigned long long *mx;
};
size_t split_slice_bytes(int K, int n_g);
// zero mx, then the column maxima of src into it
hipError_t launch_colmax(const SliceSrc &src, int K, int n_g, hipStream_t st);
// bf16: the same slices held as BF16 and multiplied on BF16 MFMA
hipError_t launch_slice(const SliceSrc &src, int K, int n_g, hipStream_t st, bool bf16);
// H segments (Z,B), (B,Z), (P3,W); S segments (A,A), (Bs,Bs): [segment][P or Q]
hipError_t launch_split_reduce(int K, int n_g, const SliceView (&hseg)[3][2],
                               const SliceView (&sseg)[2][2], double2 *H, double2 *S,
                               hipStream_t st, bool bf16);
// INT8 form: slices S8 [5][groups][N_G][16 int8], groups = 4 * ceil(K / 32);
// same column maxima and segments as the FP16 form.
size_t split8_slice_bytes(int K, int n_g);
hipError_t launch_slice8(const SliceSrc &src, int K, int n_g, hipStream_t st);
hipError_t launch_split8_reduce(int K, int n_g, const SliceView (&hseg)[3][2],
                                const SliceView (&sseg)[2][2], double2 *H, double2 *S,
                                hipStream_t st);
// Modular INT8 form (k_crt.hip): residues R [NMOD][groups][N_G][16 int8],
// groups = 16 * ceil(K / 128), of each operand's b-bit integers; the
// reduction writes each segment's residues into `work` (crt_work_bytes) and
// rebuilds H and S from them.
size_t crt_residue_bytes(int K, int n_g);
size_t crt_work_bytes(int n_g);
int crt_bits(int K);   // integer width b of the operands for contraction length K
hipError_t launch_residue(const SliceSrc &src, int K, int n_g, hipStream_t st);
hipError_t launch_crt_reduce(int K, int n_g, const SliceView (&hseg)[3][2],
                             const SliceView (&sseg)[2][2], void *work, double2 *H, double2 *S,
                             hipStream_t st);
inline size_t slice_bytes(int mode, int K, int n_g) {
    if (mode == HS_SPLIT_I8_CRT) return crt_residue_bytes(K, n_g);
    return mode == HS_SPLIT_I8 ? split8_slice_bytes(K, n_g) : split_slice_bytes(K, n_g);
}
// upper := conj(lower), Im(diag) := 0 for both outputs (launch_mirror1: one matrix)
hipError_t launch_mirror(double2 *H, double2 *S, int n_g, hipStream_t st);
hipError_t launch_mirror1(double2 *M, int n, hipStream_t st);

// Generalized eigenproblem reduction (k_gep.hip): S = L L^H, Ht = L^-1 H L^-H.
// info: device int or NULL (a workspace slot is used then); g3: the large
// products in the 3M form.
size_t gep_workspace_bytes(int N);
hipError_t launch_gep(const double2 *H, const double2 *S, int N, double2 *L, double2 *Ht,
                      int *info, char *ws, hipStream_t st, bool g3);
// Runs launch_gep's orchestration without issuing anything and checks that
// every pair of launches on different streams that touch a common 128 x 128
// cell of a matrix (one writing) is ordered; returns the number of pairs
// that are not (-1 if the orchestration failed), describing a few in report.
int gep_check_schedule(int N, bool g3, int drop_tag, std::string &report);

// ---------------------------------------------------------------------------
// Host-side plan of one atom set and the enqueue steps shared by the one-shot
// build (hs_build_ex) and the resident context (hs_ctx).

// Atom-side sizes and offsets (host copy).
struct AtomPlan {
    int n_atoms = 0, K = 0, max_nl = 0;
    long long t_total = 0;
    std::vector<int> row_off, t_off;      // [N_A+1] each
    std::vector<unsigned char> nl;        // [N_A]
    // Returns 0, or -8 for an invalid N_L (per-atom entries included).
    int make(int N_A, const int32_t *nl_per_atom, int N_L);
    // Device bytes of the k-independent buffers (AtomBufs).
    size_t atom_bytes() const;
    // Device bytes of the per-k-point buffers for N_G (Z, W; plus the
    // sliced operands in the split-precision mode).
    size_t kpoint_bytes(int n_g, int mode = 0) const;
};

// k-independent device buffers of an atom set, carved from one allocation.
struct AtomBufs {
    int *tables;      // row_off [N_A+1], then t_off [N_A+1]
    int *info;        // [N_A]
    int *sel;         // [3K]
    double *d;        // [2K]
    double2 *M1;      // [t_total]
    double2 *M2;      // [t_total]
    void carve(const AtomPlan &p, char *base);
    Atoms atoms(const AtomPlan &p) const;
};

// Batched per-atom stage (k_batch.hip): item tables of one launch.
// Every tile shape has at least ATOM_TILE_MIN_BM rows and ATOM_TILE_MIN_BN
// columns, which bounds the product tiles per atom (and so the tile table).
constexpr int ATOM_TILE_MIN_BM = 32, ATOM_TILE_MIN_BN = 128;
struct BatchBufs {
    int *perm;    // [N_A]
    int *zoff;    // [N_A + 1]
    int *ctrl;    // [2]
    int *flags;   // [2 N_A]
    int *tiles;   // [2 max_tiles(N_A, N_G)] atom, tile within the atom of each product tile
    static long long max_tiles(int n_atoms, int n_g);
    static size_t bytes(int n_atoms, int n_g);
    void carve(int n_atoms, char *base);   // tiles last
};
// Host plan: tile shape per N_L, atom order (N_L descending) and the first
// product tile of each position.
struct BatchPlan {
    unsigned char cfg[HS_MAX_NL + 1];
    std::vector<int> perm, zoff;
    long long nz = 0;   // product tiles per product (Z or W)
    // cfg_table: [HS_MAX_NL + 1] tile id per N_L, or NULL for default_tile
    void make(const AtomPlan &p, int n_g, const unsigned char *cfg_table);
    // every N_L of the plan maps to an existing tile id
    static bool valid(const AtomPlan &p, const unsigned char *cfg_table);
};
struct BatchIO {
    const double2 *T_AA, *T_AB, *T_BB, *U, *A, *B;
    double2 *M1, *M2;
    double *d;
    int *sel, *info;
    double2 *Z, *W;
};
int tile_shape(int id, int *bm, int *bn);   // 0, or -1 for an unknown id
int default_tile(int nl);
// Persistent launch of the per-atom stage (preparation items only when
// do_factor) followed, when do_factor, by the wait check.
hipError_t launch_batch(const AtomPlan &p, const Atoms &at, const BatchPlan &bp, int n_g,
                        bool do_factor, const BatchIO &io, const BatchBufs &bb, hipStream_t st);

// Per-k-point device buffers.
constexpr int NSPLIT = 6;   // sliced operands: A, U B, Z, B, P3 (W or A by row), W
struct KpointBufs {
    double2 *Z, *W;   // [K][N_G] each
    _Float16 *sl[NSPLIT];
    unsigned long long *mx[NSPLIT];
    void *crt;        // segment residues of the modular form (else NULL)
    BatchBufs batch;
    void carve(const AtomPlan &p, int n_g, int mode, char *base);
};

// How the per-atom stage of one build runs: separate preparation and product
// launches (batch = false), or the persistent batched launch with the tile
// table cfg; factor: the batched launch includes the preparation.
struct AtomStage {
    bool batch = false;
    bool factor = false;
    const unsigned char *cfg = nullptr;   // [HS_MAX_NL + 1] or NULL
    const double2 *T_AA = nullptr, *T_BB = nullptr, *U = nullptr;
    int *info = nullptr;
};

// Tables, per-atom Cholesky and operand preparation (k-independent).
// prep = false: tables only (the batched launch prepares the atoms itself).
hipError_t enqueue_atoms(const AtomPlan &p, const AtomBufs &ab, const double2 *T_AA,
                         const double2 *T_BB, const double2 *U, int *info_out, hipStream_t st,
                         bool prep = true);
// Per-atom products and the reductions for one k-point. ev: optional phase
// events [1..4] as in hs_options.phase_events (ev[0] is recorded by the caller).
hipError_t enqueue_kpoint(const AtomPlan &p, const AtomBufs &ab, int n_g, int mode,
                          const double2 *A, const double2 *B, const double2 *T_AB,
                          const KpointBufs &kb, double2 *H, double2 *S, hipStream_t st,
                          const hipEvent_t *ev, const AtomStage &stage = AtomStage());

// Argument checks shared by the one-shot entry points (hs_build's argument
// order; per_atom: N_L comes from a per-atom table and is not checked here).
int check_build_args(const hs_complex *A, const hs_complex *B, const hs_complex *T_AA,
                     const hs_complex *T_AB, const hs_complex *T_BB, const hs_complex *U,
                     int N_A, int N_L, int N_G, const hs_complex *H, const hs_complex *S,
                     bool per_atom);
// One-shot build on stream st with the workspace ws (atom part, then
// k-point part; p.atom_bytes() + p.kpoint_bytes(n_g, mode) bytes). Returns
// HS_OK or a status; enqueues only.
int run_build(const AtomPlan &p, int n_g, int mode, const hs_complex *A, const hs_complex *B,
              const hs_complex *T_AA, const hs_complex *T_AB, const hs_complex *T_BB,
              const hs_complex *U, hs_complex *H, hs_complex *S, char *ws, int32_t *info_user,
              hipStream_t st, void **events, bool batch, const hs_tuning *tuning);

}  // namespace hs
