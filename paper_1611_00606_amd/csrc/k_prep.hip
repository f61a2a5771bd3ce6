// Per-atom preparation, one 512-thread block per atom: the Cholesky of
// T^AA_a with failure detection and the operand forms of the per-atom
// products (the routine itself is in prep_atom.h).
#include "prep_atom.h"

namespace hs {

namespace {

constexpr int PREP_THREADS = 512;

__global__ void __launch_bounds__(PREP_THREADS)
k_prep(Atoms at, const double2 *__restrict__ T_AA, const double2 *__restrict__ T_BB,
       const double2 *__restrict__ U, double2 *__restrict__ M1, double2 *__restrict__ M2,
       double *__restrict__ d, int *__restrict__ sel, int *__restrict__ info_out) {
    __shared__ __align__(16) char lds[PREP_LDS_BYTES];
    prep_atom<PREP_THREADS>(at, blockIdx.x, T_AA, T_BB, U, M1, M2, d, sel, info_out, lds, nullptr,
                            nullptr);
}

}  // namespace

hipError_t launch_prep(const Atoms &at, const double2 *T_AA, const double2 *T_BB,
                       const double2 *U, double2 *M1, double2 *M2, double *d,
                       int *sel, int *info, hipStream_t st) {
    hipLaunchKernelGGL(k_prep, dim3(at.n_atoms), dim3(PREP_THREADS), 0, st, at, T_AA, T_BB, U,
                       M1, M2, d, sel, info);
    return hipGetLastError();
}

}  // namespace hs
