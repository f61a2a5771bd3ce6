// C ABI of the H/S builder: argument checks, planning (atom tables and the
// workspace carve), and the launch sequence of one build:
//   k_tables  per-atom row / T-block offsets
//   k_prep    per-atom Cholesky of T^AA with failure flags, operand forms
//   k_atom    per-atom products Z_a, W_a (Y_a or X_a)
//   k_reduce  lower triangles of H and S from the stacked operands
//   k_mirror  conjugate upper triangles
// All work is enqueued on one stream; nothing is synchronized inside
// hs_build_ex. The atom-side steps (k_tables, k_prep) do not depend on the
// k-point and are shared with the resident context (hs_serving.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/hs_build.h"
#include "hs_internal.h"

namespace hs {

namespace {
thread_local std::string g_last_error;
thread_local int g_last_status = HS_OK;   // the status g_last_error explains
constexpr size_t ALIGN = 256;
size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }
}  // namespace

void set_error(int status, const std::string &msg) {
    g_last_error = msg;
    g_last_status = status;
}
const char *message_for(int status) {
    return status == g_last_status && !g_last_error.empty() ? g_last_error.c_str() : nullptr;
}

int hip_fail(hipError_t e, const char *where) {
    set_error(HS_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
    return HS_ERR_HIP;
}

// The kernels are built for gfx950 only.
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
    }
    if (!ok[dev]) {
        set_error(HS_ERR_UNSUPPORTED, "unsupported device (the kernels are built for gfx950)");
        return HS_ERR_UNSUPPORTED;
    }
    return HS_OK;
}

namespace {

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

}  // namespace

int AtomPlan::make(int N_A, const int32_t *nl_per_atom, int N_L) {
    n_atoms = N_A;
    row_off.assign(N_A + 1, 0);
    t_off.assign(N_A + 1, 0);
    nl.assign(N_A, 0);
    max_nl = 0;
    long long rows = 0, tsz = 0;
    for (int a = 0; a < N_A; ++a) {
        const int n = nl_per_atom ? nl_per_atom[a] : N_L;
        if (n < 1 || n > HS_MAX_NL) return -8;
        nl[a] = (unsigned char)n;
        row_off[a] = (int)rows;
        t_off[a] = (int)tsz;
        rows += n;
        tsz += (long long)n * n;
        if (n > max_nl) max_nl = n;
        if (rows > (1LL << 28) || tsz > (1LL << 30)) return -8;
    }
    row_off[N_A] = (int)rows;
    t_off[N_A] = (int)tsz;
    K = (int)rows;
    t_total = tsz;
    return 0;
}

size_t AtomPlan::atom_bytes() const {
    size_t o = 0;
    o = align_up(o + sizeof(int) * 2 * (size_t)(n_atoms + 1));   // tables
    o = align_up(o + sizeof(int) * (size_t)n_atoms);             // info
    o = align_up(o + sizeof(int) * 3 * (size_t)K);               // sel
    o = align_up(o + sizeof(double) * 2 * (size_t)K);            // d
    o = align_up(o + 16 * (size_t)t_total);                      // M1
    o = align_up(o + 16 * (size_t)t_total);                      // M2
    return o;
}

size_t AtomPlan::kpoint_bytes(int n_g, int mode) const {
    size_t b = 2 * align_up(16 * (size_t)K * (size_t)n_g) + BatchBufs::bytes(n_atoms, n_g);
    if (split_mode(mode))
        b += NSPLIT * (align_up(slice_bytes(mode, K, n_g)) + align_up(8 * (size_t)n_g));
    if (mode == HS_SPLIT_I8_CRT) b += align_up(crt_work_bytes(n_g));
    return b;
}

long long BatchBufs::max_tiles(int n_atoms, int n_g) {
    return (long long)n_atoms * ((HS_MAX_NL + ATOM_TILE_MIN_BM - 1) / ATOM_TILE_MIN_BM) *
           ((n_g + ATOM_TILE_MIN_BN - 1) / ATOM_TILE_MIN_BN);
}

size_t BatchBufs::bytes(int n_atoms, int n_g) {
    return align_up(sizeof(int) * (size_t)n_atoms) + align_up(sizeof(int) * (size_t)(n_atoms + 1)) +
           align_up(2 * sizeof(int)) + align_up(2 * sizeof(int) * (size_t)n_atoms) +
           align_up(2 * sizeof(int) * (size_t)max_tiles(n_atoms, n_g));
}

void BatchBufs::carve(int n_atoms, char *base) {
    size_t o = 0;
    perm = reinterpret_cast<int *>(base + o);
    o += align_up(sizeof(int) * (size_t)n_atoms);
    zoff = reinterpret_cast<int *>(base + o);
    o += align_up(sizeof(int) * (size_t)(n_atoms + 1));
    ctrl = reinterpret_cast<int *>(base + o);
    o += align_up(2 * sizeof(int));
    flags = reinterpret_cast<int *>(base + o);
    o += align_up(2 * sizeof(int) * (size_t)n_atoms);
    tiles = reinterpret_cast<int *>(base + o);
}

void AtomBufs::carve(const AtomPlan &p, char *base) {
    size_t o = 0;
    tables = reinterpret_cast<int *>(base + o);
    o = align_up(o + sizeof(int) * 2 * (size_t)(p.n_atoms + 1));
    info = reinterpret_cast<int *>(base + o);
    o = align_up(o + sizeof(int) * (size_t)p.n_atoms);
    sel = reinterpret_cast<int *>(base + o);
    o = align_up(o + sizeof(int) * 3 * (size_t)p.K);
    d = reinterpret_cast<double *>(base + o);
    o = align_up(o + sizeof(double) * 2 * (size_t)p.K);
    M1 = reinterpret_cast<double2 *>(base + o);
    o = align_up(o + 16 * (size_t)p.t_total);
    M2 = reinterpret_cast<double2 *>(base + o);
}

Atoms AtomBufs::atoms(const AtomPlan &p) const {
    Atoms at;
    at.row_off = tables;
    at.t_off = tables + p.n_atoms + 1;
    at.n_atoms = p.n_atoms;
    at.max_nl = p.max_nl;
    at.K = p.K;
    return at;
}

void KpointBufs::carve(const AtomPlan &p, int n_g, int mode, char *base) {
    const size_t half = align_up(16 * (size_t)p.K * (size_t)n_g);
    Z = reinterpret_cast<double2 *>(base);
    W = reinterpret_cast<double2 *>(base + half);
    size_t o = 2 * half;
    batch.carve(p.n_atoms, base + o);
    o += BatchBufs::bytes(p.n_atoms, n_g);
    for (int i = 0; i < NSPLIT; ++i) {
        sl[i] = nullptr;
        mx[i] = nullptr;
        if (!split_mode(mode)) continue;
        sl[i] = reinterpret_cast<_Float16 *>(base + o);
        o += align_up(slice_bytes(mode, p.K, n_g));
        mx[i] = reinterpret_cast<unsigned long long *>(base + o);
        o += align_up(8 * (size_t)n_g);
    }
    crt = mode == HS_SPLIT_I8_CRT ? base + o : nullptr;
}

hipError_t enqueue_atoms(const AtomPlan &p, const AtomBufs &ab, const double2 *T_AA,
                         const double2 *T_BB, const double2 *U, int *info_out, hipStream_t st,
                         bool prep) {
    for (int a0 = 0; a0 < p.n_atoms; a0 += TABLE_CHUNK) {
        TableChunk c;
        c.n = std::min(TABLE_CHUNK, p.n_atoms - a0);
        std::memcpy(c.nl, p.nl.data() + a0, c.n);
        c.a0 = a0;
        c.row0 = p.row_off[a0];
        c.t0 = p.t_off[a0];
        c.last = (a0 + c.n == p.n_atoms);
        c.n_atoms = p.n_atoms;
        hipLaunchKernelGGL(k_tables, dim3(1), dim3(256), 0, st, c, ab.tables,
                           ab.tables + p.n_atoms + 1);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (!prep) return hipSuccess;
    return launch_prep(ab.atoms(p), T_AA, T_BB, U, ab.M1, ab.M2, ab.d, ab.sel,
                       info_out ? info_out : ab.info, st);
}

hipError_t enqueue_kpoint(const AtomPlan &p, const AtomBufs &ab, int n_g, int mode,
                          const double2 *A, const double2 *B, const double2 *T_AB,
                          const KpointBufs &kb, double2 *H, double2 *S, hipStream_t st,
                          const hipEvent_t *ev, const AtomStage &stage) {
    hipError_t e;
    auto mark = [&](int i) -> hipError_t {
        return (ev && ev[i]) ? hipEventRecord(ev[i], st) : hipSuccess;
    };
    if ((e = mark(1)) != hipSuccess) return e;
    if (stage.batch) {
        BatchPlan bp;
        bp.make(p, n_g, stage.cfg);
        const BatchIO io{stage.T_AA, T_AB, stage.T_BB, stage.U, A, B, ab.M1, ab.M2, ab.d,
                         ab.sel, stage.info ? stage.info : ab.info, kb.Z, kb.W};
        e = launch_batch(p, ab.atoms(p), bp, n_g, stage.factor, io, kb.batch, st);
    } else {
        e = launch_atom(ab.atoms(p), n_g, A, B, T_AB, ab.M1, ab.M2, ab.sel, kb.Z, kb.W, st);
    }
    if (e != hipSuccess) return e;
    if ((e = mark(2)) != hipSuccess) return e;
    if (split_mode(mode)) {
        // operands: 0 A, 1 U B, 2 Z, 3 B, 4 P3 (W, or A on failure-branch rows), 5 W
        const int K = p.K;
        const SliceSrc src[NSPLIT] = {
            {A, nullptr, nullptr, nullptr, kb.mx[0], kb.sl[0]},
            {B, nullptr, nullptr, ab.d + K, kb.mx[1], kb.sl[1]},
            {kb.Z, nullptr, nullptr, nullptr, kb.mx[2], kb.sl[2]},
            {B, nullptr, nullptr, nullptr, kb.mx[3], kb.sl[3]},
            {kb.W, A, ab.sel + 2 * (size_t)K, nullptr, kb.mx[4], kb.sl[4]},
            {kb.W, nullptr, nullptr, nullptr, kb.mx[5], kb.sl[5]},
        };
        for (int i = 0; i < NSPLIT; ++i) {
            if (mode == HS_SPLIT_I8_CRT) e = launch_residue(src[i], K, n_g, st);
            else if (mode == HS_SPLIT_I8) e = launch_slice8(src[i], K, n_g, st);
            else e = launch_slice(src[i], K, n_g, st, mode == HS_SPLIT_BF16);
            if (e != hipSuccess) return e;
        }
        SliceView v[NSPLIT];
        for (int i = 0; i < NSPLIT; ++i) v[i] = SliceView{kb.sl[i], kb.mx[i]};
        const SliceView hseg[3][2] = {{v[2], v[3]}, {v[3], v[2]}, {v[4], v[5]}};
        const SliceView sseg[2][2] = {{v[0], v[0]}, {v[1], v[1]}};
        if (mode == HS_SPLIT_I8_CRT)
            e = launch_crt_reduce(K, n_g, hseg, sseg, kb.crt, H, S, st);
        else if (mode == HS_SPLIT_I8)
            e = launch_split8_reduce(K, n_g, hseg, sseg, H, S, st);
        else
            e = launch_split_reduce(K, n_g, hseg, sseg, H, S, st, mode == HS_SPLIT_BF16);
    } else {
        e = launch_reduce(p.K, n_g, A, B, kb.Z, kb.W, ab.sel, ab.d, H, S, st,
                          mode == HS_FP64_3M);
    }
    if (e != hipSuccess) return e;
    if ((e = mark(3)) != hipSuccess) return e;
    if ((e = launch_mirror(H, S, n_g, st)) != hipSuccess) return e;
    return mark(4);
}

int check_build_args(const hs_complex *A, const hs_complex *B, const hs_complex *T_AA,
                     const hs_complex *T_AB, const hs_complex *T_BB, const hs_complex *U,
                     int N_A, int N_L, int N_G, const hs_complex *H, const hs_complex *S,
                     bool per_atom) {
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

namespace {
const double2 *c2(const hs_complex *x) { return reinterpret_cast<const double2 *>(x); }
double2 *c2(hs_complex *x) { return reinterpret_cast<double2 *>(x); }
}  // namespace

// One-shot build: atom part then k-point part of one workspace.
int run_build(const AtomPlan &p, int n_g, int mode, const hs_complex *A, const hs_complex *B,
              const hs_complex *T_AA, const hs_complex *T_AB, const hs_complex *T_BB,
              const hs_complex *U, hs_complex *H, hs_complex *S, char *ws, int32_t *info_user,
              hipStream_t st, void **events, bool batch, const hs_tuning *tuning) {
    hipEvent_t ev[HS_NUM_PHASE_EVENTS] = {};
    if (events)
        for (int i = 0; i < HS_NUM_PHASE_EVENTS; ++i) ev[i] = static_cast<hipEvent_t>(events[i]);
    hipError_t e;
    if (ev[0] && (e = hipEventRecord(ev[0], st)) != hipSuccess) return hs::hip_fail(e, "phase event");
    hs::AtomBufs ab;
    ab.carve(p, ws);
    hs::KpointBufs kb;
    kb.carve(p, n_g, mode, ws + p.atom_bytes());
    e = hs::enqueue_atoms(p, ab, c2(T_AA), c2(T_BB), c2(U), info_user, st, !batch);
    if (e != hipSuccess) return hs::hip_fail(e, "per-atom preparation launch");
    hs::AtomStage stage;
    if (batch) {
        stage.batch = true;
        stage.factor = true;
        stage.cfg = tuning ? tuning->cfg : nullptr;
        stage.T_AA = c2(T_AA);
        stage.T_BB = c2(T_BB);
        stage.U = c2(U);
        stage.info = info_user;
    }
    e = hs::enqueue_kpoint(p, ab, n_g, mode, c2(A), c2(B), c2(T_AB), kb, c2(H), c2(S), st, ev,
                           stage);
    if (e != hipSuccess) return hs::hip_fail(e, "k-point launch");
    return HS_OK;
}

}  // namespace hs

using hs::c2;

extern "C" {

size_t hs_workspace_bytes(int N_A, const int32_t *nl_per_atom, int N_L, int N_G, int mode) {
    if (N_A < 1 || N_G < 1 || !hs::valid_mode(mode)) return 0;
    hs::AtomPlan p;
    if (p.make(N_A, nl_per_atom, N_L) != 0) return 0;
    return p.atom_bytes() + p.kpoint_bytes(N_G, mode);
}

int hs_build_ex(const hs_complex *A, const hs_complex *B, const hs_complex *T_AA,
                const hs_complex *T_AB, const hs_complex *T_BB, const hs_complex *U, int N_A,
                int N_L, int N_G, hs_complex *H, hs_complex *S, const hs_options *opt) {
    if (!opt) return -12;
    int rc = hs::check_build_args(A, B, T_AA, T_AB, T_BB, U, N_A, N_L, N_G, H, S,
                                  opt->nl_per_atom != nullptr);
    if (rc != HS_OK) return rc;
    if (!hs::valid_mode(opt->mode) || (opt->batch != 0 && opt->batch != 1)) return -12;
    hs::AtomPlan p;
    rc = p.make(N_A, opt->nl_per_atom, N_L);
    if (rc != 0) return rc;
    if (opt->batch && !hs::BatchPlan::valid(p, opt->tuning ? opt->tuning->cfg : nullptr))
        return -12;
    // the batched launch reports a bounded wait that ran out through info
    // (every entry -1), so it needs a caller-visible info array
    if (opt->batch && !opt->info) return -12;
    if (reinterpret_cast<uintptr_t>(opt->workspace) % 16) return -12;   // 16-byte loads
    rc = hs::check_device();
    if (rc != HS_OK) return rc;
    const size_t need = p.atom_bytes() + p.kpoint_bytes(N_G, opt->mode);
    if (!opt->workspace || opt->workspace_bytes < need) {
        hs::set_error(HS_ERR_WORKSPACE, "workspace too small: the build needs " + std::to_string(need) +
                      " bytes, " + std::to_string(opt->workspace ? opt->workspace_bytes : 0) +
                      " given");
        return HS_ERR_WORKSPACE;
    }
    return hs::run_build(p, N_G, opt->mode, A, B, T_AA, T_AB, T_BB, U, H, S,
                         static_cast<char *>(opt->workspace),
               opt->info, static_cast<hipStream_t>(opt->stream), opt->phase_events,
               opt->batch != 0, opt->tuning);
}

int hs_build(const hs_complex *A, const hs_complex *B, const hs_complex *T_AA,
             const hs_complex *T_AB, const hs_complex *T_BB, const hs_complex *U, int N_A,
             int N_L, int N_G, hs_complex *H, hs_complex *S) {
    int rc = hs::check_build_args(A, B, T_AA, T_AB, T_BB, U, N_A, N_L, N_G, H, S, false);
    if (rc != HS_OK) return rc;
    hs::AtomPlan p;
    rc = p.make(N_A, nullptr, N_L);
    if (rc != 0) return rc;
    rc = hs::check_device();
    if (rc != HS_OK) return rc;
    void *ws = nullptr;
    hipError_t e = hipMalloc(&ws, p.atom_bytes() + p.kpoint_bytes(N_G));
    if (e == hipErrorOutOfMemory) {
        hs::set_error(HS_ERR_NOMEM, "workspace allocation");
        return HS_ERR_NOMEM;
    }
    if (e != hipSuccess) return hs::hip_fail(e, "hipMalloc");
    rc = hs::run_build(p, N_G, HS_FP64, A, B, T_AA, T_AB, T_BB, U, H, S, static_cast<char *>(ws),
                       nullptr, nullptr, nullptr, false, nullptr);
    e = hipStreamSynchronize(nullptr);
    if (rc == HS_OK && e != hipSuccess) rc = hs::hip_fail(e, "hs_build execution");
    hipError_t e2 = hipFree(ws);
    if (rc == HS_OK && e2 != hipSuccess) rc = hs::hip_fail(e2, "hipFree");
    return rc;
}

int hs_tile_config(int id, int *bm, int *bn) { return hs::tile_shape(id, bm, bn); }

size_t hs_gep_workspace_bytes(int N) { return N < 1 ? 0 : hs::gep_workspace_bytes(N); }

int hs_gep_reduce(const hs_complex *H, const hs_complex *S, int N, hs_complex *L, hs_complex *Ht,
                  int32_t *info, void *workspace, size_t workspace_bytes, void *stream) {
    return hs_gep_reduce_ex(H, S, N, L, Ht, info, workspace, workspace_bytes, stream, HS_FP64);
}

int hs_gep_reduce_ex(const hs_complex *H, const hs_complex *S, int N, hs_complex *L,
                     hs_complex *Ht, int32_t *info, void *workspace, size_t workspace_bytes,
                     void *stream, int mode) {
    if (!H) return -1;
    if (!S) return -2;
    if (N < 1) return -3;
    if (!L) return -4;
    if (!Ht) return -5;
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % 16) return -7;
    if (mode != HS_FP64 && mode != HS_FP64_3M) return -10;
    int rc = hs::check_device();
    if (rc != HS_OK) return rc;
    if (workspace_bytes < hs::gep_workspace_bytes(N)) {
        hs::set_error(HS_ERR_WORKSPACE, "workspace too small: the reduction needs " +
                      std::to_string(hs::gep_workspace_bytes(N)) + " bytes, " +
                      std::to_string(workspace_bytes) + " given");
        return HS_ERR_WORKSPACE;
    }
    hipError_t e = hs::launch_gep(c2(H), c2(S), N, c2(L), c2(Ht), info,
                                  static_cast<char *>(workspace), static_cast<hipStream_t>(stream),
                                  mode == HS_FP64_3M);
    return e == hipSuccess ? HS_OK : hs::hip_fail(e, "hs_gep_reduce launch");
}

int hs_gep_check_schedule(int N, int mode, int drop_wait, char *report, size_t report_len) {
    if (N < 1) return -1;
    if (mode != HS_FP64 && mode != HS_FP64_3M) return -2;
    std::string rep;
    const int n = hs::gep_check_schedule(N, mode == HS_FP64_3M, drop_wait, rep);
    if (report && report_len) {
        const size_t k = std::min(rep.size(), report_len - 1);
        std::memcpy(report, rep.data(), k);
        report[k] = '\0';
    }
    return n < 0 ? -6 : n;
}

const char *hs_status_string(int status) {
    const char *m = hs::message_for(status);
    switch (status) {
        case HS_OK: return "success";
        case HS_ERR_HIP: return m ? m : "HIP runtime error";
        case HS_ERR_WORKSPACE: return m ? m : "workspace too small";
        case HS_ERR_NOMEM: return m ? m : "out of device memory";
        case HS_ERR_UNSUPPORTED: return m ? m : "unsupported size or device";
        default:
            if (status < 0) return "invalid argument (-status is its 1-based position)";
            return "unknown status";
    }
}

}  // extern "C"
