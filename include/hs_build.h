/*
 * hs_build.h - C ABI of the MI355X (gfx950) Hamiltonian/overlap builder for
 * FLAPW methods (Fabregat-Traver, Davidovic, Hoehnerbach, Di Napoli,
 * "Hybrid CPU-GPU generation of the Hamiltonian and Overlap matrices in
 * FLAPW methods", arXiv:1611.00606).
 *
 * For one k-point it computes (Sec. 2, equations for H and S; index forms in
 * Sec. 1.1)
 *
 *   H = sum_a  A_a^H T^AA_a A_a + A_a^H T^AB_a B_a
 *            + B_a^H T^BA_a A_a + B_a^H T^BB_a B_a,     T^BA_a := (T^AB_a)^H
 *   S = sum_a  A_a^H A_a + B_a^H U_a^H U_a B_a
 *
 * by the route of Alg. 1: per-atom products Z_a = T^BA_a A_a + 1/2 T^BB_a B_a,
 * a per-atom Cholesky T^AA_a = C_a C_a^H with Y_a = C_a^H A_a on success and
 * X_a = T^AA_a A_a on failure, and large stacked Hermitian reductions
 * H = Z^H B + B^H Z + Y_HPD^H Y_HPD + A_notHPD^H X_notHPD,
 * S = A^H A + (U B)^H (U B). All arithmetic is IEEE binary64 (complex double,
 * 8 real flops per complex multiply-add) on the GPU.
 *
 * Conventions shared by every entry point
 *  - complex values are hs_complex = {double re, im} (the layout of
 *    std::complex<double>, C99 double _Complex and torch.complex128);
 *  - every array is C-contiguous (row-major) and lives in DEVICE memory of
 *    the current HIP device, 16-byte aligned (256 recommended), owned by the
 *    caller; the library never frees caller memory and never writes inputs;
 *  - atoms are stacked along rows: K = sum_a N_L(a);
 *      A, B   [K][N_G]          row r of atom a is r - row_offset(a)
 *      T_AA, T_AB, T_BB         per-atom N_L(a) x N_L(a) blocks, row-major,
 *                               concatenated in atom order (for a uniform
 *                               N_L this is [N_A][N_L][N_L])
 *      U      [K]               diagonal of U_a; only |U|^2 enters S
 *      H, S   [N_G][N_G]        outputs, written in full: exactly Hermitian
 *                               (upper = conj(lower)), Im(diagonal) = 0
 *  - index form of the result:
 *      H[g'][g] = sum_a sum_{l',l} conj(A[l'][g']) T_AA[l'][l] A[l][g]
 *               + conj(A[l'][g']) T_AB[l'][l] B[l][g]
 *               + conj(B[l'][g']) conj(T_AB[l][l']) A[l][g]
 *               + conj(B[l'][g']) T_BB[l'][l] B[l][g]
 *      S[g'][g] = sum_a sum_l conj(A[l][g']) A[l][g]
 *               + |U[l]|^2 conj(B[l][g']) B[l][g]
 *    (l, l' run over atom a's rows; T blocks are atom a's).
 *  - T_AA and T_BB are Hermitian; only their LOWER triangles (diagonal
 *    included, imaginary part of the diagonal ignored) are read.
 *
 * Status codes (LAPACK style)
 *    0   success
 *   -i   argument i (1-based, in hs_build's order) is invalid: a NULL
 *        pointer, or a size < 1 (e.g. -7: N_A < 1), or an N_L out of range
 *    1   HIP runtime error (hs_status_string(1) gives the last message)
 *    2   workspace too small (see hs_workspace_bytes)
 *    3   out of device memory (hs_build only: it allocates its workspace)
 *    4   unsupported: N_L > HS_MAX_NL, or the device is not gfx950
 *  A failed per-atom Cholesky is NOT an error: it selects the failure branch
 *  of Alg. 1 for that atom and is reported through info[a] (below). NaN/Inf in
 *  inputs are not checked and propagate; a NaN pivot selects the failure
 *  branch.
 */
#ifndef HS_BUILD_H
#define HS_BUILD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double re, im;
} hs_complex;

#define HS_MAX_NL 128

enum {
    HS_OK = 0,
    HS_ERR_HIP = 1,
    HS_ERR_WORKSPACE = 2,
    HS_ERR_NOMEM = 3,
    HS_ERR_UNSUPPORTED = 4
};

/* Arithmetic of the large reductions (the per-atom Cholesky, the HPD test and
 * the per-atom products are always binary64).
 *   HS_FP64       complex binary64 MFMA.
 *   HS_SPLIT_F16  split precision: each binary64 operand column is scaled by a
 *                 power of two and cut into 4 exact integer slices of 8, 9,
 *                 9, 9 bits held in FP16; the slice products (pairs
 *                 s + t <= 5) run on FP16 MFMA with FP32 accumulation (the two
 *                 leading levels exact, flushed every 64 contraction rows)
 *                 and are recombined in binary64. Error about 2^-35 of the
 *                 operand column maxima per product term (relative Frobenius
 *                 error of H and S 2e-10 .. 4e-10 for Gaussian operands,
 *                 below 1e-9). Inputs must be finite.
 *   HS_SPLIT_I8   split precision on INT8 MFMA: the same column scaling, 5
 *                 integer slices of 7 bits (int8; the first within +-127),
 *                 the 15 pairs s + t <= 6 on INT8 MFMA with exact INT32
 *                 accumulation per level, recombined in binary64 once per
 *                 contraction segment. Error about 2^-35 of the operand
 *                 column maxima per product term (same order as
 *                 HS_SPLIT_F16). Inputs must be finite.
 *   HS_FP64_3M    complex binary64 MFMA with 3 real products per complex
 *                 product instead of 4 (the 3M or Gauss form: for conj(p) q,
 *                 T1 = pr qr, T2 = pi qi, T3 = (pr - pi)(qr + qi) summed
 *                 over the contraction, Re = T1 + T2, Im = T3 - T1 + T2).
 *                 Three quarters of the matrix-core work of HS_FP64; the
 *                 real parts are the same sums, the imaginary parts' error
 *                 bound grows from u (|pr||qi| + |pi||qr|) to
 *                 u (|pr - pi||qr + qi| + |pr||qr| + |pi||qi|) per term
 *                 (u = 2^-53, times the usual contraction-length factor).
 *                 Same workspace as HS_FP64.
 *   HS_SPLIT_BF16 HS_SPLIT_F16 with the slices held as BF16 and multiplied on
 *                 BF16 MFMA. The slices are integers of at most 9 bits
 *                 (magnitude <= 256), exact in BF16 too, and their products
 *                 accumulate exactly in FP32 either way, so H and S are
 *                 bitwise those of HS_SPLIT_F16 (MI355X runs BF16 and FP16
 *                 MFMA at the same dense rate). Workspace as HS_SPLIT_F16.
 *   HS_SPLIT_I8_CRT modular form on INT8 MFMA: each operand column is scaled by
 *                 a power of two and rounded to signed integers of b bits
 *                 (b = 36 for contraction lengths up to about 5e4, one bit
 *                 less per factor of four beyond); the exact integer products
 *                 of each contraction segment are formed modulo 11 pairwise
 *                 coprime moduli <= 255 (symmetric residues in int8, INT32
 *                 sums, one INT8 MFMA product per modulus instead of the 15
 *                 slice pairs of HS_SPLIT_I8) and rebuilt by the Chinese
 *                 remainder theorem (mixed-radix digits) before the binary64
 *                 scaling. The only error is the rounding of the operands,
 *                 2^-36 of their column maxima per element. Workspace: 22
 *                 bytes per operand element and a residue buffer of about
 *                 55 N_G^2 bytes. Inputs must be finite. */
typedef enum {
    HS_FP64 = 0,
    HS_SPLIT_F16 = 1,
    HS_SPLIT_I8 = 2,
    HS_FP64_3M = 3,
    HS_SPLIT_BF16 = 4,
    HS_SPLIT_I8_CRT = 5
} hs_mode;

/* Tile shapes of the batched per-atom stage (see hs_options.batch): shape id
 * -> (BM rows of an atom's N_L, BN columns of N_G) per tile, listed by
 * hs_tile_config. */
#define HS_NUM_TILE_CONFIGS 8

/* Tile shape id for each N_L (entry [N_L], 1 <= N_L <= HS_MAX_NL; entry 0
 * unused), as filled by hs_autotune_atoms. */
typedef struct {
    unsigned char cfg[HS_MAX_NL + 1];
} hs_tuning;

typedef struct {
    /* hipStream_t to enqueue on; NULL = the default (null) stream. */
    void *stream;
    /* device scratch of >= hs_workspace_bytes(...) bytes, 16-byte aligned
       (256 recommended; otherwise hs_build_ex returns -12), owned by the
       caller; contents on entry are ignored. */
    void *workspace;
    size_t workspace_bytes;
    /* device int32 [N_A], or NULL when batch = 0 (required with batch = 1:
       NULL returns -12). On completion info[a] = 0 when T_AA_a had a
       Cholesky factor (atom a took Alg. 1's success branch), else the 1-based
       index j of the first pivot d_j = T_jj - sum_{k<j} |C_jk|^2 that is not
       > 0 or is NaN (LAPACK zpotrf semantics; atom a took the failure
       branch). With batch = 1, info[a] = -1 for EVERY atom means that a
       product tile of the batched launch gave up waiting for its atom's
       preparation (a bounded wait that should never run out): H and S are
       then undefined and the build must be repeated. */
    int32_t *info;
    /* hs_mode */
    int mode;
    /* HOST int32 [N_A] giving N_L of each atom, or NULL when every atom has
       the N_L argument's value. Each entry in [1, HS_MAX_NL]. */
    const int32_t *nl_per_atom;
    /* NULL, or HOST array of HS_NUM_PHASE_EVENTS hipEvent_t (created by the
       caller) that the build records on its stream at the phase boundaries:
       [0] start, [1] after the per-atom Cholesky and operand preparation,
       [2] after the per-atom products (Alg. 1 first loop and second-loop
       branches), [3] after the large lower-triangle reductions of H and S,
       [4] after the conjugate mirroring (end of the build). With batch = 1
       the preparation runs inside the batched launch: [1] is recorded right
       after [0] and [1]..[2] covers preparation and products. */
    void **phase_events;
    /* 0: per-atom preparation and products as separate launches, one tile
       shape for all atoms (the largest N_L decides). 1: batched form - one
       persistent launch runs every atom's Cholesky (with its failure test)
       and every atom's Z_a and W_a tiles, each atom with the tile shape of
       its N_L. Same results up to rounding order. */
    int batch;
    /* HOST hs_tuning or NULL (built-in shapes: 32, 64, 96 or 128 rows, the
       fewest that cover N_L, by 128 columns, 192 for 96 rows). Used when
       batch = 1; every N_L in use must map to an id < HS_NUM_TILE_CONFIGS. */
    const hs_tuning *tuning;
} hs_options;

#define HS_NUM_PHASE_EVENTS 5

/*
 * hs_build - synchronous convenience form.
 * Runs on the default stream with a workspace it allocates and frees itself,
 * and returns after the build has completed (so execution errors are
 * reported). Arguments 1..11 as described above:
 *   1 A, 2 B, 3 T_AA, 4 T_AB, 5 T_BB, 6 U   inputs (device, read-only)
 *   7 N_A >= 1, 8 N_L in [1, HS_MAX_NL], 9 N_G >= 1
 *   10 H, 11 S                              outputs (device, [N_G][N_G])
 */
int hs_build(const hs_complex *A, const hs_complex *B,
             const hs_complex *T_AA, const hs_complex *T_AB,
             const hs_complex *T_BB, const hs_complex *U,
             int N_A, int N_L, int N_G,
             hs_complex *H, hs_complex *S);

/*
 * hs_workspace_bytes - device scratch that hs_build_ex needs for this shape.
 * nl_per_atom: host [N_A] or NULL (uniform N_L). Returns 0 for invalid sizes.
 */
size_t hs_workspace_bytes(int N_A, const int32_t *nl_per_atom, int N_L, int N_G,
                          int mode);

/*
 * hs_build_ex - asynchronous form: enqueues the whole build on opt->stream
 * and returns; the caller synchronizes. Arguments 1..11 as hs_build, 12 opt
 * (required). The return code covers argument checks and launch errors;
 * execution errors surface at the caller's synchronization. The workspace
 * and outputs must not be used by other work until the build completes.
 * Results are deterministic: repeated calls on the same inputs give
 * bitwise-identical H, S and info.
 */
int hs_build_ex(const hs_complex *A, const hs_complex *B,
                const hs_complex *T_AA, const hs_complex *T_AB,
                const hs_complex *T_BB, const hs_complex *U,
                int N_A, int N_L, int N_G,
                hs_complex *H, hs_complex *S,
                const hs_options *opt);

/* Bytes of the device array that hs_build_static uses as its workspace. */
#define HS_STATIC_SCRATCH_BYTES ((size_t)256 << 20)

/*
 * hs_build_static - hs_build_ex for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the build's workspace is a device array inside the
 * library (HS_STATIC_SCRATCH_BYTES per device, held from the first call on
 * that device until the process ends) instead of a caller buffer.
 * Arguments 1..12 as hs_build_ex, except that opt->workspace must be NULL and
 * opt->workspace_bytes 0 (else -12). Enqueues on opt->stream and returns
 * (asynchronous); results are bitwise those of hs_build_ex with the same
 * options. No device memory is allocated or freed: the first call on a
 * device only looks up the array's address there. Returns what hs_build_ex
 * returns, and 2 when hs_workspace_bytes(...) for these sizes and this mode
 * exceeds HS_STATIC_SCRATCH_BYTES (hs_status_string(2) then names both
 * sizes). Every call on one device uses the same array and the kernels
 * clear what they need cleared; calls whose work overlaps on one device
 * (different streams, or different host threads) race on it and give
 * undefined results, so callers serialize them (one stream is enough).
 */
int hs_build_static(const hs_complex *A, const hs_complex *B,
                    const hs_complex *T_AA, const hs_complex *T_AB,
                    const hs_complex *T_BB, const hs_complex *U,
                    int N_A, int N_L, int N_G,
                    hs_complex *H, hs_complex *S,
                    const hs_options *opt);

/* Human-readable text for a status code (thread-local last HIP message for 1). */
const char *hs_status_string(int status);

/*
 * hs_tile_config - shape of batched tile id `id`: *bm rows of an atom's
 * N_L by *bn columns of N_G (either pointer may be NULL). Returns 0, or -1
 * for an id outside [0, HS_NUM_TILE_CONFIGS).
 */
int hs_tile_config(int id, int *bm, int *bn);

/*
 * hs_autotune_atoms - measures every tile shape of the batched per-atom stage
 * on the current device and picks the fastest per N_L.
 * For each of the n_values N_L values (host int32 array, each in
 * [1, HS_MAX_NL]) it builds a synthetic atom set of that N_L (about 2048
 * rows, HPD T^AA blocks) at N_G columns, prepares it once, then times the
 * batched product launch with each shape `reps` times (HIP events on
 * `stream`, NULL = default stream) and keeps the minimum.
 * out (host): entries of the listed N_L values get the fastest id, all
 * other entries the built-in choice. ms (host, optional): [n_values]
 * [HS_NUM_TILE_CONFIGS] minimum times in milliseconds.
 * Allocates and frees its own device memory and synchronizes `stream`: call
 * it at set-up, not inside a build loop.
 * Returns 0, -1 (nl_values NULL), -2 (n_values < 1 or an entry out of
 * range), -3 (N_G < 1), -4 (reps < 1), -6 (out NULL), or a status >= 1.
 */
int hs_autotune_atoms(const int32_t *nl_values, int n_values, int N_G, int reps,
                      void *stream, hs_tuning *out, float *ms);

/* ------------------------------------------------------------------------
 * Reduction of the generalized eigenproblem to standard form, the step that
 * follows the build: per k-point the expansion coefficients c solve
 * H c = lambda S c with S Hermitian and generically positive definite
 * (Sec. 1.1). With
 *     S = L L^H   (Cholesky; L lower with a positive real diagonal)
 *     Ht = L^{-1} H L^{-H}
 * H c = lambda S c holds exactly when Ht y = lambda y with y = L^H c.
 * Right-looking over 128-column panels with an explicit inverse of L; the
 * O(N^3) work runs as products on the complex FP64 MFMA tiles.
 * ---------------------------------------------------------------------- */

/* Device scratch hs_gep_reduce needs for N (0 for N < 1): 5 N^2 complex. */
size_t hs_gep_workspace_bytes(int N);

/*
 * hs_gep_reduce - enqueue the reduction on `stream` (NULL: default stream)
 * and return (asynchronous, like hs_build_ex).
 *   1 H   device [N][N], Hermitian, read in full (an hs_build output)
 *   2 S   device [N][N], Hermitian, only its lower triangle is read
 *   3 N   >= 1
 *   4 L   device [N][N] out: the Cholesky factor, upper triangle zero
 *   5 Ht  device [N][N] out: L^{-1} H L^{-H}, exactly Hermitian with a
 *         real diagonal (its lower triangle mirrored)
 *   6 info  device int32 or NULL: 0, or the 1-based index of the first
 *         pivot of S that is not > 0 or is NaN (LAPACK zpotrf); L and Ht
 *         are undefined then
 *   7 workspace  device, >= hs_gep_workspace_bytes(N) bytes, 16-byte
 *         aligned (256 recommended);  8 workspace_bytes;  9 stream
 * Outputs must not overlap the inputs or each other. Returns 0, -i for an
 * invalid argument i (NULL pointer, N < 1, workspace not 16-byte aligned),
 * 2 (workspace too small), or 1 (HIP error).
 * For N > 384 part of the work runs on up to three library-owned streams of the
 * same device (created on first use, default priority, kept until the process
 * ends), forked from and joined back into `stream` with events: when the call
 * returns, everything it enqueued is ordered before later work on `stream`.
 * Calls that overlap on one device share those streams: each still depends
 * only on its own events (results are unaffected), but their work on the
 * shared streams runs in the order it was enqueued.
 */
int hs_gep_reduce(const hs_complex *H, const hs_complex *S, int N,
                  hs_complex *L, hs_complex *Ht, int32_t *info,
                  void *workspace, size_t workspace_bytes, void *stream);

/*
 * hs_gep_reduce_ex - hs_gep_reduce with the arithmetic of its large products
 * chosen by 10 mode: HS_FP64 (as hs_gep_reduce) or HS_FP64_3M (3 real MFMA
 * products per complex product in every product on the tiles; the 128x128
 * diagonal blocks are still factored and inverted in the 4-product form;
 * error bound of the imaginary parts as described at hs_mode). Any other
 * mode returns -10; arguments 1..9 and the other statuses as hs_gep_reduce.
 */
int hs_gep_reduce_ex(const hs_complex *H, const hs_complex *S, int N,
                     hs_complex *L, hs_complex *Ht, int32_t *info,
                     void *workspace, size_t workspace_bytes, void *stream, int mode);

/*
 * hs_gep_check_schedule - race check of the reduction's stream schedule,
 * host only (no device, no HIP call, nothing allocated on a device). Runs
 * the orchestration of hs_gep_reduce_ex for 1 N and 2 mode (HS_FP64 or
 * HS_FP64_3M) without issuing anything, recording every launch with its
 * stream and the rectangles of each matrix it reads and writes, and every
 * event record and stream wait; then checks with vector clocks that every
 * two launches on different streams that touch a common 128 x 128 cell of a
 * matrix, one of them writing, are ordered by stream order and event waits.
 *   3 drop_wait  0, or a wait site (1..10, in the order the library's
 *         schedule defines them) whose waits are left out: a test hook that
 *         shows the check finds the race a missing wait opens
 *   4 report, 5 report_len  host buffer (or NULL) for a NUL-terminated
 *         description of the first few unordered pairs
 * Returns the number of unordered pairs (0: every conflict is ordered), -1
 * for N < 1, -2 for another mode, -6 if the orchestration reported an
 * error.
 */
int hs_gep_check_schedule(int N, int mode, int drop_wait, char *report, size_t report_len);

/* ------------------------------------------------------------------------
 * Resident context: one atom set, many k-points.
 *
 * T^[..]_a and U_a do not depend on the k-point, while A_a, B_a do: there is
 * one (H, S) pair per independent k-point (Sec. 1.1). The context keeps the
 * atom side on the device and runs the k-independent part of Alg. 1 once:
 * the per-atom Cholesky of T^AA_a with its failure flags (second loop's try
 * step) and the operand forms of the per-atom products. Each k-point then
 * runs only the per-atom products and the large reductions.
 * ---------------------------------------------------------------------- */
typedef struct hs_ctx hs_ctx;

/*
 * hs_ctx_create - copy the atom data into a new context and factorize.
 * Arguments: 1 T_AA, 2 T_AB, 3 T_BB, 4 U (device, layouts as above),
 * 5 N_A >= 1, 6 N_L (uniform N_L, ignored when 7 is given), 7 nl_per_atom
 * (HOST int32 [N_A] or NULL), 8 stream (hipStream_t or NULL), 9 out.
 * Synchronous: returns after the context is ready (inputs may be freed
 * afterwards). The context owns its device memory until hs_ctx_destroy.
 */
int hs_ctx_create(const hs_complex *T_AA, const hs_complex *T_AB, const hs_complex *T_BB,
                  const hs_complex *U, int N_A, int N_L, const int32_t *nl_per_atom,
                  void *stream, hs_ctx **out);

/* Rows K = sum_a N_L(a) of the A, B operands this context expects. */
int hs_ctx_rows(const hs_ctx *ctx);

/* Per-atom failure flags (as hs_options.info) copied to HOST int32 [N_A]. */
int hs_ctx_info(const hs_ctx *ctx, int32_t *info_host);

/* Device scratch that hs_ctx_build needs for N_G (0 for invalid sizes). */
size_t hs_ctx_workspace_bytes(const hs_ctx *ctx, int N_G, int mode);

/* Device bytes one k-point occupies: A, B, H, S and the workspace. This is
 * what the serving loop admits requests by. */
size_t hs_ctx_footprint_bytes(const hs_ctx *ctx, int N_G, int mode);

/*
 * hs_ctx_build - enqueue one k-point on opt->stream (asynchronous, like
 * hs_build_ex). Arguments: 1 ctx, 2 A, 3 B ([K][N_G] device), 4 N_G >= 1,
 * 5 H, 6 S ([N_G][N_G] device), 7 opt (stream, workspace, mode,
 * phase_events, batch and tuning are used; info and nl_per_atom are ignored:
 * the context holds them; with batch = 1 the cached preparation is reused
 * and the batched launch runs the products only). Concurrent calls on
 * different streams with different
 * workspaces and outputs are allowed; results are bitwise identical to a
 * build of the same inputs alone.
 */
int hs_ctx_build(const hs_ctx *ctx, const hs_complex *A, const hs_complex *B, int N_G,
                 hs_complex *H, hs_complex *S, const hs_options *opt);

void hs_ctx_destroy(hs_ctx *ctx);

/* ------------------------------------------------------------------------
 * Serving loop: continuous batching of k-point builds on one context.
 *
 * Requests (one k-point each, any N_G) are queued on submit and admitted as
 * soon as a slot (a HIP stream) is free and their device footprint
 * (hs_ctx_footprint_bytes) fits in the free part of the server's device
 * arena: in arrival order by default, or letting later requests pass one
 * that waits for arena space (hs_server_set_admission). An admitted request
 * copies its A, B from host memory, builds on its slot's stream, and keeps
 * H, S in the arena until released, so work of several requests overlaps on
 * the device. All calls are host-side and non-blocking except
 * hs_server_destroy; one thread drives a server.
 * ---------------------------------------------------------------------- */
typedef struct hs_server hs_server;

typedef struct {
    int64_t id;                 /* caller's tag, unique among live requests */
    int N_G;                    /* >= 1 */
    const hs_complex *A_host;   /* HOST [K][ld] (pinned memory lets the copy overlap) */
    const hs_complex *B_host;   /* HOST [K][ld]; the first N_G columns are used */
    int64_t ld;                 /* row stride of A_host, B_host in elements, >= N_G */
} hs_request;

typedef struct {
    int64_t id;
    int N_G;
    int status;                 /* 0, or the error status of the request */
    hs_complex *H, *S;          /* device [N_G][N_G], valid until hs_server_release */
    double t_submit, t_admit, t_done;   /* seconds on the server clock (hs_server_now) */
} hs_result;

/* Arguments: 1 ctx (must outlive the server), 2 n_slots >= 1,
 * 3 arena_bytes (device memory reserved once, here), 4 mode, 5 out. */
int hs_server_create(hs_ctx *ctx, int n_slots, size_t arena_bytes, int mode, hs_server **out);

/* Admission policies (hs_server_set_admission). */
enum {
    HS_ADMIT_FIFO = 0,    /* arrival order; a request that does not fit the free
                             arena holds back every later one (the default) */
    HS_ADMIT_BYPASS = 1   /* a later request that fits may start while an earlier
                             one waits; a waiting request is passed at most
                             max_bypass times, then nothing behind it starts
                             until it has */
};

/* Arguments: 1 srv, 2 policy (HS_ADMIT_*), 3 max_bypass >= 0 (HS_ADMIT_BYPASS
 * only). Applies from the next hs_server_progress on. Returns 0, -1 (srv
 * NULL), -2 (unknown policy) or -3 (max_bypass < 0). */
int hs_server_set_admission(hs_server *srv, int policy, int max_bypass);

/* Queue a request (host memory must stay valid until its result is popped).
 * Returns HS_ERR_NOMEM (3) when its footprint exceeds the whole arena. */
int hs_server_submit(hs_server *srv, const hs_request *req);

/* Admit and launch what fits, collect completions; returns the number of
 * completed results waiting to be popped, or a negative status on error. */
int hs_server_progress(hs_server *srv);

/* Pop one completed result into *out: returns 1, or 0 when none is ready. */
int hs_server_pop(hs_server *srv, hs_result *out);

/* Free the arena space of a popped result (its H, S become invalid). */
int hs_server_release(hs_server *srv, int64_t id);

/* Requests queued, in flight, or completed but not yet popped. */
int hs_server_pending(const hs_server *srv);

/* Device bytes currently held (admitted or unreleased requests). */
size_t hs_server_used_bytes(const hs_server *srv);

/* Seconds since the server was created (monotonic clock). */
double hs_server_now(const hs_server *srv);

/* Waits for all launched work, then frees the arena and streams. */
void hs_server_destroy(hs_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* HS_BUILD_H */
