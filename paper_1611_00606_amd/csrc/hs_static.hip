// Allocation-free one-shot build: hs_build_ex with its workspace taken from a
// file-scope device array of fixed size instead of a caller buffer, for
// callers that cannot allocate device memory.
//
// The array lives in the library's code object: each device the library
// runs on holds its own copy (HS_STATIC_SCRATCH_BYTES) from the first use
// until the process ends. Its device address is looked up once per device
// with hipGetSymbolAddress and only that address is handed to the kernels
// (in host code the array's name is not a device address). The build's
// kernels clear everything they need cleared (batch counters and flags,
// column maxima) themselves, so the array's previous contents do not matter.
// Calls that overlap on one device share the array and race.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/hs_build.h"
#include "hs_internal.h"

namespace {

static __device__ __align__(256) unsigned char scratch[HS_STATIC_SCRATCH_BYTES];

// Device address of `scratch` on the current device (looked up on the
// first call per device, with that device current).
int scratch_address(char **out) {
    static std::mutex mu;
    static std::vector<void *> addr;   // per device; nullptr until looked up
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hs::hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(mu);
    if ((int)addr.size() <= dev) addr.resize(dev + 1, nullptr);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hs::hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) {
            hs::set_error(HS_ERR_HIP, "hipGetSymbolAddress(scratch) returned no address");
            return HS_ERR_HIP;
        }
        addr[dev] = p;
    }
    *out = static_cast<char *>(addr[dev]);
    return HS_OK;
}

}  // namespace

extern "C" int hs_build_static(const hs_complex *A, const hs_complex *B, const hs_complex *T_AA,
                               const hs_complex *T_AB, const hs_complex *T_BB,
                               const hs_complex *U, int N_A, int N_L, int N_G, hs_complex *H,
                               hs_complex *S, const hs_options *opt) {
    if (!opt) return -12;
    int rc = hs::check_build_args(A, B, T_AA, T_AB, T_BB, U, N_A, N_L, N_G, H, S,
                                  opt->nl_per_atom != nullptr);
    if (rc != HS_OK) return rc;
    if (!hs::valid_mode(opt->mode) || (opt->batch != 0 && opt->batch != 1)) return -12;
    if (opt->workspace || opt->workspace_bytes) return -12;   // the array is the workspace
    hs::AtomPlan p;
    rc = p.make(N_A, opt->nl_per_atom, N_L);
    if (rc != 0) return rc;
    if (opt->batch && !hs::BatchPlan::valid(p, opt->tuning ? opt->tuning->cfg : nullptr))
        return -12;
    // the batched launch reports a bounded wait that ran out through info
    // (every entry -1), so it needs a caller-visible info array
    if (opt->batch && !opt->info) return -12;
    const size_t need = p.atom_bytes() + p.kpoint_bytes(N_G, opt->mode);
    if (need > (size_t)HS_STATIC_SCRATCH_BYTES) {   // host-side check, before any device call
        hs::set_error(HS_ERR_WORKSPACE, "hs_build_static: the build needs " + std::to_string(need) +
                      " bytes of workspace, the static scratch holds " +
                      std::to_string((size_t)HS_STATIC_SCRATCH_BYTES));
        return HS_ERR_WORKSPACE;
    }
    rc = hs::check_device();
    if (rc != HS_OK) return rc;
    char *ws = nullptr;
    rc = scratch_address(&ws);
    if (rc != HS_OK) return rc;
    return hs::run_build(p, N_G, opt->mode, A, B, T_AA, T_AB, T_BB, U, H, S, ws, opt->info,
                         static_cast<hipStream_t>(opt->stream), opt->phase_events,
                         opt->batch != 0, opt->tuning);
}
