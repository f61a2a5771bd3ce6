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

/* Arithmetic of the large reductions. HS_FP64: complex binary64 MFMA. */
typedef enum {
    HS_FP64 = 0
} hs_mode;

typedef struct {
    /* hipStream_t to enqueue on; NULL = the default (null) stream. */
    void *stream;
    /* device scratch of >= hs_workspace_bytes(...) bytes, 256-byte aligned,
       owned by the caller; contents on entry are ignored. */
    void *workspace;
    size_t workspace_bytes;
    /* device int32 [N_A] or NULL. On completion info[a] = 0 when T_AA_a had a
       Cholesky factor (atom a took Alg. 1's success branch), else the 1-based
       index j of the first pivot d_j = T_jj - sum_{k<j} |C_jk|^2 that is not
       > 0 or is NaN (LAPACK zpotrf semantics; atom a took the failure
       branch). */
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
       [4] after the conjugate mirroring (end of the build). */
    void **phase_events;
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

/* Human-readable text for a status code (thread-local last HIP message for 1). */
const char *hs_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* HS_BUILD_H */
