// C ABI of the H/S builder: argument checks, planning (atom tables and the
// workspace carve), and the launch sequence of one build:
//   k_prep    per-atom Cholesky of T^AA with failure flags, operand forms
//   k_atom    per-atom products Z_a, W_a (Y_a or X_a)
//   k_reduce  lower triangles of H and S from the stacked operands
//   k_mirror  conjugate upper triangles
// All work is enqueued on one stream; nothing is synchronized inside
// hs_build_ex.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/hs_build.h"
#include "hs_internal.h"

namespace {

thread_local std::string g_last_error;

int hip_fail(hipError_t e, const char *where) {
    g_last_error = std::string(where) + ": " + hipGetErrorString(e);
    return HS_ERR_HIP;
}

constexpr size_t ALIGN = 256;
size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

// Device check: the kernels are built for gfx950 only.
int check_device() {
    static std::mutex mu;
    static std::vector<int> ok;   // per device: -1 unknown, 0 no, 1 yes
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(mu);
    if ((int)ok.size() <= dev) ok.resize(dev + 1, -1);
    if (ok[dev] < 0) {
        hipDeviceProp_t prop;
        e = hipGetDeviceProperties(&prop, dev);
        if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
        ok[dev] = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : 0;
        if (!ok[dev]) g_last_error = std::string("unsupported device ") + prop.gcnArchName;
    }
    return ok[dev] ? HS_OK : HS_ERR_UNSUPPORTED;
}

// Atom tables (row and T-block offsets) are written on the device by a small
// kernel whose inputs travel as kernel arguments, a chunk of up to
// TABLE_CHUNK atoms per launch. Nothing is copied from host memory, so the
// enqueue is fully asynchronous and needs no host buffer to outlive the call.
constexpr int TABLE_CHUNK = 1024;
struct TableChunk {
    unsigned char nl[TABLE_CHUNK];
    int n;          // atoms in this chunk
    int a0;         // first atom
    int row0;       // row offset of the first atom
    int t0;         // T offset of the first atom
    int last;       // 1 when this chunk ends the atom list (writes the totals)
    int n_atoms;
};

__global__ void __launch_bounds__(256) k_tables(TableChunk c, int *row_off, int *t_off) {
    for (int i = threadIdx.x; i < c.n; i += blockDim.x) {
        int r = c.row0, t = c.t0;
        for (int j = 0; j < i; ++j) {
            r += c.nl[j];
            t += c.nl[j] * c.nl[j];
        }
        row_off[c.a0 + i] = r;
        t_off[c.a0 + i] = t;
        if (c.last && i == c.n - 1) {
            row_off[c.n_atoms] = r + c.nl[i];
            t_off[c.n_atoms] = t + c.nl[i] * c.nl[i];
        }
    }
}

struct Plan {
    int n_atoms = 0, n_g = 0, K = 0, max_nl = 0;
    long long t_total = 0;
    std::vector<int> tables;   // row_off[N_A+1] then t_off[N_A+1] (host copy)
    std::vector<unsigned char> nl; // N_L of each atom
    // workspace carve (byte offsets)
    size_t o_tables, o_info, o_sel, o_d, o_m1, o_m2, o_z, o_w, total;

    // Returns 0, or -8 for an invalid N_L (per-atom entries included).
    int make(int N_A, const int32_t *nl_per_atom, int N_L, int N_G) {
        n_atoms = N_A;
        n_g = N_G;
        tables.assign(2 * (N_A + 1), 0);
        nl.assign(N_A, 0);
        long long rows = 0, tsz = 0;
        for (int a = 0; a < N_A; ++a) {
            const int n = nl_per_atom ? nl_per_atom[a] : N_L;
            if (n < 1 || n > HS_MAX_NL) return -8;
            nl[a] = (unsigned char)n;
            tables[a] = (int)rows;
            tables[N_A + 1 + a] = (int)tsz;
            rows += n;
            tsz += (long long)n * n;
            if (n > max_nl) max_nl = n;
            if (rows > (1LL << 30) || tsz > (1LL << 30)) return -8;
        }
        tables[N_A] = (int)rows;
        tables[2 * N_A + 1] = (int)tsz;
        K = (int)rows;
        t_total = tsz;
        size_t o = 0;
        o_tables = o; o = align_up(o + sizeof(int) * tables.size());
        o_info = o;   o = align_up(o + sizeof(int) * (size_t)N_A);
        o_sel = o;    o = align_up(o + sizeof(int) * 3 * (size_t)K);
        o_d = o;      o = align_up(o + sizeof(double) * 2 * (size_t)K);
        o_m1 = o;     o = align_up(o + 16 * (size_t)t_total);
        o_m2 = o;     o = align_up(o + 16 * (size_t)t_total);
        o_z = o;      o = align_up(o + 16 * (size_t)K * (size_t)N_G);
        o_w = o;      o = align_up(o + 16 * (size_t)K * (size_t)N_G);
        total = o;
        return 0;
    }
};

int check_args(const hs_complex *A, const hs_complex *B, const hs_complex *T_AA,
               const hs_complex *T_AB, const hs_complex *T_BB, const hs_complex *U, int N_A,
               int N_L, int N_G, const hs_complex *H, const hs_complex *S, bool per_atom) {
    if (!A) return -1;
    if (!B) return -2;
    if (!T_AA) return -3;
    if (!T_AB) return -4;
    if (!T_BB) return -5;
    if (!U) return -6;
    if (N_A < 1) return -7;
    if (!per_atom && (N_L < 1 || N_L > HS_MAX_NL)) return -8;
    if (N_G < 1) return -9;
    if (!H) return -10;
    if (!S) return -11;
    return HS_OK;
}

int run(const Plan &p, const hs_complex *A, const hs_complex *B, const hs_complex *T_AA,
        const hs_complex *T_AB, const hs_complex *T_BB, const hs_complex *U, hs_complex *H,
        hs_complex *S, char *ws, int32_t *info_user, hipStream_t st, void **events) {
    hipEvent_t ev[HS_NUM_PHASE_EVENTS] = {};
    if (events)
        for (int i = 0; i < HS_NUM_PHASE_EVENTS; ++i) ev[i] = static_cast<hipEvent_t>(events[i]);
    auto mark = [&](int i) -> hipError_t {
        return ev[i] ? hipEventRecord(ev[i], st) : hipSuccess;
    };
    int *tables = reinterpret_cast<int *>(ws + p.o_tables);
    hipError_t e = mark(0);
    if (e != hipSuccess) return hip_fail(e, "phase event");
    for (int a0 = 0; a0 < p.n_atoms; a0 += TABLE_CHUNK) {
        TableChunk c;
        c.n = std::min(TABLE_CHUNK, p.n_atoms - a0);
        std::memcpy(c.nl, p.nl.data() + a0, c.n);
        c.a0 = a0;
        c.row0 = p.tables[a0];
        c.t0 = p.tables[p.n_atoms + 1 + a0];
        c.last = (a0 + c.n == p.n_atoms);
        c.n_atoms = p.n_atoms;
        hipLaunchKernelGGL(k_tables, dim3(1), dim3(256), 0, st, c, tables, tables + p.n_atoms + 1);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "k_tables launch");
    }

    hs::Atoms at;
    at.row_off = tables;
    at.t_off = tables + p.n_atoms + 1;
    at.n_atoms = p.n_atoms;
    at.max_nl = p.max_nl;
    at.K = p.K;
    int *info = info_user ? info_user : reinterpret_cast<int *>(ws + p.o_info);
    int *sel = reinterpret_cast<int *>(ws + p.o_sel);
    double *d = reinterpret_cast<double *>(ws + p.o_d);
    double2 *M1 = reinterpret_cast<double2 *>(ws + p.o_m1);
    double2 *M2 = reinterpret_cast<double2 *>(ws + p.o_m2);
    double2 *Z = reinterpret_cast<double2 *>(ws + p.o_z);
    double2 *W = reinterpret_cast<double2 *>(ws + p.o_w);
    auto c2 = [](const hs_complex *x) { return reinterpret_cast<const double2 *>(x); };

    e = hs::launch_prep(at, c2(T_AA), c2(T_BB), c2(U), M1, M2, d, sel, info, st);
    if (e != hipSuccess) return hip_fail(e, "k_prep launch");
    if ((e = mark(1)) != hipSuccess) return hip_fail(e, "phase event");
    e = hs::launch_atom(at, p.n_g, c2(A), c2(B), c2(T_AB), M1, M2, Z, W, st);
    if (e != hipSuccess) return hip_fail(e, "k_atom launch");
    if ((e = mark(2)) != hipSuccess) return hip_fail(e, "phase event");
    e = hs::launch_reduce(p.K, p.n_g, c2(A), c2(B), Z, W, sel, d,
                          reinterpret_cast<double2 *>(H), reinterpret_cast<double2 *>(S), st,
                          ev[3]);
    if (e != hipSuccess) return hip_fail(e, "k_reduce launch");
    if ((e = mark(4)) != hipSuccess) return hip_fail(e, "phase event");
    return HS_OK;
}

}  // namespace

extern "C" {

size_t hs_workspace_bytes(int N_A, const int32_t *nl_per_atom, int N_L, int N_G, int mode) {
    if (N_A < 1 || N_G < 1 || mode != HS_FP64) return 0;
    Plan p;
    if (p.make(N_A, nl_per_atom, N_L, N_G) != 0) return 0;
    return p.total;
}

int hs_build_ex(const hs_complex *A, const hs_complex *B, const hs_complex *T_AA,
                const hs_complex *T_AB, const hs_complex *T_BB, const hs_complex *U, int N_A,
                int N_L, int N_G, hs_complex *H, hs_complex *S, const hs_options *opt) {
    if (!opt) return -12;
    int rc = check_args(A, B, T_AA, T_AB, T_BB, U, N_A, N_L, N_G, H, S, opt->nl_per_atom != nullptr);
    if (rc != HS_OK) return rc;
    if (opt->mode != HS_FP64) return -12;
    Plan p;
    rc = p.make(N_A, opt->nl_per_atom, N_L, N_G);
    if (rc != 0) return rc;
    rc = check_device();
    if (rc != HS_OK) return rc;
    if (!opt->workspace || opt->workspace_bytes < p.total) return HS_ERR_WORKSPACE;
    return run(p, A, B, T_AA, T_AB, T_BB, U, H, S, static_cast<char *>(opt->workspace),
               opt->info, static_cast<hipStream_t>(opt->stream), opt->phase_events);
}

int hs_build(const hs_complex *A, const hs_complex *B, const hs_complex *T_AA,
             const hs_complex *T_AB, const hs_complex *T_BB, const hs_complex *U, int N_A,
             int N_L, int N_G, hs_complex *H, hs_complex *S) {
    int rc = check_args(A, B, T_AA, T_AB, T_BB, U, N_A, N_L, N_G, H, S, false);
    if (rc != HS_OK) return rc;
    Plan p;
    rc = p.make(N_A, nullptr, N_L, N_G);
    if (rc != 0) return rc;
    rc = check_device();
    if (rc != HS_OK) return rc;
    void *ws = nullptr;
    hipError_t e = hipMalloc(&ws, p.total);
    if (e == hipErrorOutOfMemory) {
        g_last_error = "workspace allocation";
        return HS_ERR_NOMEM;
    }
    if (e != hipSuccess) return hip_fail(e, "hipMalloc");
    rc = run(p, A, B, T_AA, T_AB, T_BB, U, H, S, static_cast<char *>(ws), nullptr, nullptr,
             nullptr);
    e = hipStreamSynchronize(nullptr);
    if (rc == HS_OK && e != hipSuccess) rc = hip_fail(e, "hs_build execution");
    hipError_t e2 = hipFree(ws);
    if (rc == HS_OK && e2 != hipSuccess) rc = hip_fail(e2, "hipFree");
    return rc;
}

const char *hs_status_string(int status) {
    switch (status) {
        case HS_OK: return "success";
        case HS_ERR_HIP: return g_last_error.empty() ? "HIP runtime error" : g_last_error.c_str();
        case HS_ERR_WORKSPACE: return "workspace too small";
        case HS_ERR_NOMEM: return "out of device memory";
        case HS_ERR_UNSUPPORTED:
            return g_last_error.empty() ? "unsupported size or device" : g_last_error.c_str();
        default:
            if (status < 0) return "invalid argument (-status is its 1-based position)";
            return "unknown status";
    }
}

}  // extern "C"
