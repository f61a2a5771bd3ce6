// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

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
hipError_t launch_atom(const Atoms &at, int n_g, const double2 *A, const double2 *B,
                       const double2 *T_AB, const double2 *M1, const double2 *M2,
                       double2 *Z, double2 *W, hipStream_t st);

// Large reductions (Alg. 1 l.10, 13-15, 28-29) into the lower triangles of
// H and S, then conjugate mirroring of the upper triangles.
// `mid_event` (optional) is recorded between the reduction and the mirror.
hipError_t launch_reduce(int K, int n_g, const double2 *A, const double2 *B,
                         const double2 *Z, const double2 *W, const int *sel,
                         const double *d, double2 *H, double2 *S, hipStream_t st,
                         hipEvent_t mid_event);

}  // namespace hs
