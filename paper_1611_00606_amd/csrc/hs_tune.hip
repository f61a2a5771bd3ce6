// Autotuner of the batched per-atom stage: for each N_L it times every
// candidate tile shape of k_batch on a synthetic atom set of that N_L and
// keeps the fastest (hs_autotune_atoms in hs_build.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <vector>

#include "../../include/hs_build.h"
#include "hs_internal.h"

namespace {

constexpr int TUNE_ROWS = 2048;   // rows of the synthetic atom set per N_L

__device__ __forceinline__ double unit_hash(unsigned long long x) {
    // splitmix64 finalizer -> [-1, 1)
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    x ^= x >> 31;
    return (double)(x >> 11) * 0x1p-52 - 1.0;
}

__global__ void __launch_bounds__(256)
k_fill(double2 *x, long long n, unsigned long long seed) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) x[i] = double2{unit_hash(seed + 2 * i), unit_hash(seed + 2 * i + 1)};
}

// adds `boost` to the diagonal of every n x n block (an HPD T^AA by
// diagonal dominance)
__global__ void __launch_bounds__(256)
k_boost_diag(double2 *t, int n, int n_atoms, double boost) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < (long long)n * n_atoms) {
        const long long a = i / n, r = i % n;
        t[a * n * n + r * n + r].x += boost;
    }
}

hipError_t fill(double2 *x, long long n, unsigned long long seed, hipStream_t st) {
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, n, seed);
    return hipGetLastError();
}

size_t up256(size_t x) { return (x + 255) / 256 * 256; }

// Times every tile shape for one N_L; ms_out[HS_NUM_TILE_CONFIGS].
int tune_one(int nl, int n_g, int reps, hipStream_t st, float *ms_out) {
    const int n_atoms = std::max(4, (TUNE_ROWS + nl - 1) / nl);
    hs::AtomPlan p;
    if (p.make(n_atoms, nullptr, nl) != 0) return HS_ERR_UNSUPPORTED;
    const size_t kn = (size_t)p.K * (size_t)n_g;
    const size_t tb = 16 * (size_t)p.t_total;
    const size_t sizes[] = {16 * kn, 16 * kn, tb, tb, tb, 16 * (size_t)p.K, p.atom_bytes(),
                            p.kpoint_bytes(n_g, HS_FP64)};
    size_t total = 0;
    for (size_t s : sizes) total += up256(s);
    char *mem = nullptr;
    hipError_t e = hipMalloc(&mem, total);
    if (e == hipErrorOutOfMemory) {
        hs::set_error(HS_ERR_NOMEM, "autotune allocation");
        return HS_ERR_NOMEM;
    }
    if (e != hipSuccess) return hs::hip_fail(e, "hipMalloc");
    char *ptr[8];
    size_t o = 0;
    for (int i = 0; i < 8; ++i) {
        ptr[i] = mem + o;
        o += up256(sizes[i]);
    }
    double2 *A = reinterpret_cast<double2 *>(ptr[0]);
    double2 *B = reinterpret_cast<double2 *>(ptr[1]);
    double2 *T_AA = reinterpret_cast<double2 *>(ptr[2]);
    double2 *T_AB = reinterpret_cast<double2 *>(ptr[3]);
    double2 *T_BB = reinterpret_cast<double2 *>(ptr[4]);
    double2 *U = reinterpret_cast<double2 *>(ptr[5]);
    hs::AtomBufs ab;
    ab.carve(p, ptr[6]);
    hs::KpointBufs kb;
    kb.carve(p, n_g, HS_FP64, ptr[7]);

    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    int rc = HS_OK;
    auto check = [&](hipError_t err, const char *where) {
        if (rc == HS_OK && err != hipSuccess) rc = hs::hip_fail(err, where);
        return rc == HS_OK;
    };
    if (check(hipEventCreate(&ev0), "hipEventCreate") && check(hipEventCreate(&ev1), "hipEventCreate")) {
        bool ok = check(fill(A, (long long)kn, 1, st), "fill") &&
                  check(fill(B, (long long)kn, 1ull << 40, st), "fill") &&
                  check(fill(T_AA, p.t_total, 2ull << 40, st), "fill") &&
                  check(fill(T_AB, p.t_total, 3ull << 40, st), "fill") &&
                  check(fill(T_BB, p.t_total, 4ull << 40, st), "fill") &&
                  check(fill(U, p.K, 5ull << 40, st), "fill");
        if (ok) {
            hipLaunchKernelGGL(k_boost_diag, dim3((p.K + 255) / 256), dim3(256), 0, st, T_AA, nl,
                               n_atoms, 2.0 * nl + 2.0);
            ok = check(hipGetLastError(), "boost") &&
                 check(hs::enqueue_atoms(p, ab, T_AA, T_BB, U, nullptr, st, true), "prep");
        }
        const hs::BatchIO io{T_AA, T_AB, T_BB, U, A, B, ab.M1, ab.M2, ab.d, ab.sel, ab.info,
                             kb.Z, kb.W};
        unsigned char table[HS_MAX_NL + 1];
        for (int c = 0; ok && c < HS_NUM_TILE_CONFIGS; ++c) {
            std::fill(table, table + HS_MAX_NL + 1, (unsigned char)c);
            hs::BatchPlan bp;
            bp.make(p, n_g, table);
            ok = check(hs::launch_batch(p, ab.atoms(p), bp, n_g, false, io, kb.batch, st),
                       "autotune launch");
            float best = FLT_MAX;
            for (int r = 0; ok && r < reps; ++r) {
                ok = check(hipEventRecord(ev0, st), "hipEventRecord") &&
                     check(hs::launch_batch(p, ab.atoms(p), bp, n_g, false, io, kb.batch, st),
                           "autotune launch") &&
                     check(hipEventRecord(ev1, st), "hipEventRecord") &&
                     check(hipEventSynchronize(ev1), "autotune run");
                float t = 0.f;
                if (ok) ok = check(hipEventElapsedTime(&t, ev0, ev1), "hipEventElapsedTime");
                if (ok) best = std::min(best, t);
            }
            ms_out[c] = best;
        }
        (void)check(hipStreamSynchronize(st), "autotune run");
    }
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    (void)hipFree(mem);
    return rc;
}

}  // namespace

extern "C" int hs_autotune_atoms(const int32_t *nl_values, int n_values, int N_G, int reps,
                                 void *stream, hs_tuning *out, float *ms) {
    if (!nl_values) return -1;
    if (n_values < 1) return -2;
    for (int i = 0; i < n_values; ++i)
        if (nl_values[i] < 1 || nl_values[i] > HS_MAX_NL) return -2;
    if (N_G < 1) return -3;
    if (reps < 1) return -4;
    if (!out) return -6;
    int rc = hs::check_device();
    if (rc != HS_OK) return rc;
    for (int v = 0; v <= HS_MAX_NL; ++v) out->cfg[v] = (unsigned char)hs::default_tile(v);
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::vector<float> t(HS_NUM_TILE_CONFIGS);
    for (int i = 0; i < n_values; ++i) {
        const int v = nl_values[i];
        int j = 0;
        while (j < i && nl_values[j] != v) ++j;
        if (j < i) {   // repeated value: same measurement
            if (ms)
                std::copy(ms + j * HS_NUM_TILE_CONFIGS, ms + (j + 1) * HS_NUM_TILE_CONFIGS,
                          ms + i * HS_NUM_TILE_CONFIGS);
            continue;
        }
        rc = tune_one(v, N_G, reps, st, t.data());
        if (rc != HS_OK) return rc;
        int best = 0;
        for (int c = 1; c < HS_NUM_TILE_CONFIGS; ++c)
            if (t[c] < t[best]) best = c;
        out->cfg[v] = (unsigned char)best;
        if (ms) std::copy(t.begin(), t.end(), ms + i * HS_NUM_TILE_CONFIGS);
    }
    return HS_OK;
}
