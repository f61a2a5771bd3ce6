#!/usr/bin/env python3
"""Benchmark of one H/S build on one MI355X.

A step is one pass of the whole build (per-atom Cholesky and operand
preparation, per-atom products, the large lower-triangle reductions of H and
S, conjugate mirroring) over one synthetic k-point with inputs resident in
HBM. The default workload is the N_G = 8000 case (N_A = 100 atoms, N_L = 81,
complex FP64).

Prints one JSON line with the FP64-equivalent TFLOP/s of the build
(algorithmic flops / measured time), the roofline of the dominant kernel
(the reduction, timed live with HIP events on the stream it runs on), and
the CPU oracle timed on a bounded sample of the same workload.
"""

from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_MFMA_PEAK_TFLOPS = 78.6   # MI355X dense FP64 matrix peak
FP16_MFMA_PEAK_TFLOPS = 2500.0  # MI355X dense FP16 matrix peak
HBM_PEAK_GBS = 8000.0
# FP16 MFMA flops the split form issues per FP64 flop of the reductions: per
# complex multiply-add (8 FP64 flops) 10 slice pairs x 2 MFMAs (Re, Im) x 2
# interleaved real products x 2 flops = 80.
SPLIT_F16_PER_FP64 = 10.0
INT8_MFMA_PEAK_TOPS = 5000.0    # MI355X dense INT8 matrix peak
# INT8 MFMA ops per FP64 flop: 15 slice pairs x 2 MFMAs x 2 interleaved
# products x 2 ops = 120 per complex multiply-add (8 FP64 flops).
SPLIT_I8_PER_FP64 = 15.0
# FP64 MFMA flops the 3M form issues per FP64 flop of the reductions: 3 real
# products per complex multiply-add instead of 4.
FP64_3M_PER_FP64 = 0.75
# INT8 MFMA ops of the modular form per FP64 flop: 11 moduli x 2 MFMAs x 2
# interleaved products x 2 ops = 88 per complex multiply-add.
CRT_I8_PER_FP64 = 11.0


# HBM traffic records: rocprofv3 counter summaries under profiles/, each
# tagged with a digest of the kernel's sources (so a record of older code is
# never reported) and the bytes one launch moved on the N_G = 8000 workload.
SPLIT_SOURCES = ["paper_1611_00606_amd/csrc/k_split.hip", "paper_1611_00606_amd/csrc/split_common.h"]
TRAFFIC_RECORDS = {
    "k_reduce": ("k_reduce_precision_ng8000.md",
                 ["paper_1611_00606_amd/csrc/zmfma_tile.h", "paper_1611_00606_amd/csrc/zmfma_direct.h",
                  "paper_1611_00606_amd/csrc/k_reduce.hip"]),
    "k_reduce_3m": ("k_reduce_3m_precision_ng8000.md",
                    ["paper_1611_00606_amd/csrc/zmfma_tile.h", "paper_1611_00606_amd/csrc/zmfma_direct.h",
                     "paper_1611_00606_amd/csrc/k_reduce.hip"]),
    "k_split_reduce": ("k_split_reduces_precision_ng8000.md", SPLIT_SOURCES),
    "k_split8_reduce": ("k_split_reduces_precision_ng8000.md", SPLIT_SOURCES),
    "k_split_reduce_bf16": ("k_split_reduces_precision_ng8000.md", SPLIT_SOURCES),
    "k_crt_reduce": ("k_crt_reduce_precision_ng8000.md",
                     ["paper_1611_00606_amd/csrc/k_crt.hip", "paper_1611_00606_amd/csrc/split_common.h"]),
}
TRAFFIC_UNIT = ("HBM bytes per launch: rocprofv3 TCC_EA0 read requests by size (32, 64, 128 B) "
                "and write requests by size (32, 64 B), one launch on this workload")


def measured_traffic(config: str, kernel: str = "k_reduce"):
    """HBM bytes per launch of `kernel` from its committed rocprofv3 counter
    record, or None when the record is for another workload or the kernel's
    sources have changed since the counters were taken."""
    if config != "precision" or kernel not in TRAFFIC_RECORDS:
        return None
    name, sources = TRAFFIC_RECORDS[kernel]
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            rec[k.strip()] = v.strip()
    if rec.get(f"{kernel} source_sha256") != kernel_source_digest(sources):
        return None
    v = rec.get(f"{kernel} traffic_bytes")
    return float(v) if v else None


def kernel_source_digest(sources) -> str:
    """SHA-256 of a kernel's sources with comments and whitespace removed, so
    that a change of the code (not of its comments) invalidates the record."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in sources:
        text = open(os.path.join(ROOT, f)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        h.update(re.sub(r"\s+", "", text).encode())
    return h.hexdigest()


def reduction_bytes(K: int, n_g: int, slice_bytes_per_elem: float = 16.0, operands: int = 4) -> float:
    """Algorithmic HBM bytes of one reduction launch: every operand read once
    (operands x K x N_G elements of slice_bytes_per_elem bytes) and the two
    lower triangles written (2 x N_G^2 / 2 complex values)."""
    return float(operands) * slice_bytes_per_elem * K * n_g + 16.0 * float(n_g) ** 2


class HipEvents:
    """Raw hipEvent_t handles from the HIP runtime torch has loaded."""

    def __init__(self):
        import torch  # noqa: F401  (binds the runtime torch ships)
        self.rt = ctypes.CDLL("libamdhip64.so.7")
        self.rt.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.rt.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                                ctypes.c_void_p]
        self.rt.hipEventSynchronize.argtypes = [ctypes.c_void_p]
        self.rt.hipEventDestroy.argtypes = [ctypes.c_void_p]

    def create(self, n):
        out = []
        for _ in range(n):
            e = ctypes.c_void_p()
            assert self.rt.hipEventCreate(ctypes.byref(e)) == 0
            out.append(e.value)
        return out

    def elapsed_ms(self, a, b):
        assert self.rt.hipEventSynchronize(ctypes.c_void_p(b)) == 0
        ms = ctypes.c_float()
        assert self.rt.hipEventElapsedTime(ctypes.byref(ms), ctypes.c_void_p(a), ctypes.c_void_p(b)) == 0
        return float(ms.value)

    def destroy(self, evs):
        for e in evs:
            self.rt.hipEventDestroy(ctypes.c_void_p(e))


def _blas_threads() -> int:
    try:
        from threadpoolctl import threadpool_info
        return int(max([i.get("num_threads", 1) for i in threadpool_info()
                        if i.get("user_api") == "blas"] or [1]))
    except Exception:
        return len(os.sched_getaffinity(0))


def cpu_baseline(p, alg1_seconds: float):
    """Time the CPU oracle on the whole workload; Alg. 1 through host
    BLAS/LAPACK (the paper's own CPU method) on the first atoms, sized to
    about alg1_seconds."""
    import oracle
    from paper_1611_00606_amd.flops import algorithmic_flops
    threads = _blas_threads()
    t0 = time.perf_counter()
    oracle.hamiltonian(p.A, p.B, p.T_AA, p.T_AB, p.T_BB, p.nl)
    oracle.overlap(p.A, p.B, p.U, p.nl)
    dt = time.perf_counter() - t0
    info = np.zeros(p.N_A, np.int32)
    info[list(p.failing)] = 1
    f = algorithmic_flops(p.nl, p.N_G, info)

    def alg1(n):
        k = int(p.nl[:n].sum())
        t = int((p.nl[:n].astype(np.int64) ** 2).sum())
        t1 = time.perf_counter()
        oracle.algorithm1(p.A[:k], p.B[:k], p.T_AA[:t], p.T_AB[:t], p.T_BB[:t], p.U[:k], p.nl[:n])
        return time.perf_counter() - t1

    n = int(max(1, min(p.N_A, round(alg1_seconds / max(alg1(1), 1e-3)))))
    dt_alg1 = alg1(n)
    f1 = algorithmic_flops(p.nl[:n], p.N_G, info[:n])
    return {
        "value": f / dt / 1e12,
        "unit": "TFLOP/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": f"direct-sum oracle (NumPy complex128) on the whole workload ({p.N_A} atoms, "
                  f"N_G={p.N_G}): {dt:.2f} s for {f:.3e} algorithmic flops",
        "cpu_model": _cpu_model(),
        "blas": _blas_vendor(),
        "alg1_host_tflops": round(f1 / dt_alg1 / 1e12, 4),
        "alg1_host_sample": f"Alg. 1 through SciPy BLAS/LAPACK (zher2k, zherk, zpotrf, ztrmm, ...) "
                            f"on atoms 0..{n - 1} at full N_G: {dt_alg1:.2f} s",
    }


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _blas_vendor() -> str:
    try:
        from threadpoolctl import threadpool_info
        libs = [f"{i.get('internal_api')} {i.get('version')}" for i in threadpool_info()
                if i.get("user_api") == "blas"]
        return ", ".join(sorted(set(libs))) or "unknown"
    except Exception:
        return "unknown"


def atom_stage_rates(p, info, ms: float):
    """Per-atom stage (Cholesky, T.A / T.B products): FP64 rate and HBM rate
    against the minimum traffic (read A, B and the T blocks, write Z, W)."""
    from paper_1611_00606_amd.flops import paper_step_flops
    f = paper_step_flops(p.nl, p.N_G, info)
    flops = sum(f[k] for k in ("loop1_zgemm_TBA_A", "loop1_zhemm_TBB_B", "loop2_zpotrf",
                               "loop2_ztrmm_Y", "loop2_zhemm_X"))
    nbytes = 16.0 * (4 * float(p.K) * p.N_G + 3 * float((p.nl.astype(np.int64) ** 2).sum()))
    return {"ms": round(ms, 4), "tflops": round(flops / (ms * 1e-3) / 1e12, 3),
            "frac_fp64_peak": round(flops / (ms * 1e-3) / 1e12 / FP64_MFMA_PEAK_TFLOPS, 4),
            "hbm_gbs": round(nbytes / (ms * 1e-3) / 1e9, 1),
            "frac_hbm_peak": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def sync_build_wall_ms(p, reps: int = 3):
    """Host wall time of the synchronous hs_build (allocates and frees its
    workspace, returns after completion); uniform N_L only."""
    import torch
    from paper_1611_00606_amd import hs_build
    if not np.all(p.nl == p.nl[0]):
        return None
    dev = torch.device("cuda:0")
    up = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)  # noqa: E731
    A, B, taa, tab, tbb, U = (up(x) for x in (p.A, p.B, p.T_AA, p.T_AB, p.T_BB, p.U))
    H = torch.empty((p.N_G, p.N_G), dtype=torch.complex128, device=dev)
    S = torch.empty_like(H)
    hs_build(A, B, taa, tab, tbb, U, p.N_A, int(p.nl[0]), p.N_G, H, S)
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        hs_build(A, B, taa, tab, tbb, U, p.N_A, int(p.nl[0]), p.N_G, H, S)
        ts.append(time.perf_counter() - t0)
    del A, B, taa, tab, tbb, U, H, S
    torch.cuda.empty_cache()
    return round(1e3 * float(np.median(ts)), 3)


def timed_builds(run, steps: int, warmup: int, hip):
    """Mean per-phase and whole-build milliseconds of `steps` builds."""
    import torch
    from paper_1611_00606_amd import HS_NUM_PHASE_EVENTS
    for _ in range(warmup):
        run.run()
    torch.cuda.synchronize()
    evs = [hip.create(HS_NUM_PHASE_EVENTS) for _ in range(steps)]
    for k in range(steps):
        run.run(phase_events=evs[k])
    torch.cuda.synchronize()
    ph = np.array([[hip.elapsed_ms(e[i], e[i + 1]) for i in range(HS_NUM_PHASE_EVENTS - 1)]
                   for e in evs]).mean(axis=0)
    total = float(np.mean([hip.elapsed_ms(e[0], e[-1]) for e in evs]))
    hip.destroy([e for es in evs for e in es])
    return ph, total


SPLIT_MODES = {
    1: dict(name="split_f16", traffic_kernel="k_split_reduce", slice_bytes=16.0,
            mode="split_f16 (slices of 8+9+9+9 bits in FP16, 10 slice pairs on FP16 MFMA, FP32 "
                 "accumulation flushed every 64 rows, FP64 recombination)",
            per_fp64=SPLIT_F16_PER_FP64, peak=FP16_MFMA_PEAK_TFLOPS,
            unit="TFLOP/s (FP16 MFMA flops issued)",
            kernel="slicing + split reduction (phase 2..3)", phase="slice_and_reduce_HS"),
    2: dict(name="split_i8", traffic_kernel="k_split8_reduce", slice_bytes=10.0,
            mode="split_i8 (five 7-bit int8 slices, 15 slice pairs on INT8 MFMA, exact INT32 "
                 "accumulation per level, FP64 recombination per segment)",
            per_fp64=SPLIT_I8_PER_FP64, peak=INT8_MFMA_PEAK_TOPS,
            unit="TOP/s (INT8 MFMA ops issued)",
            kernel="slicing + split reduction (phase 2..3)", phase="slice_and_reduce_HS"),
    4: dict(name="split_bf16", traffic_kernel="k_split_reduce_bf16", slice_bytes=16.0,
            mode="split_bf16 (the FP16 form's slices held as BF16 on BF16 MFMA: the same "
                 "integers, exact in both formats, so the same H and S)",
            per_fp64=SPLIT_F16_PER_FP64, peak=FP16_MFMA_PEAK_TFLOPS,
            unit="TFLOP/s (BF16 MFMA flops issued)",
            kernel="slicing + split reduction (phase 2..3)", phase="slice_and_reduce_HS"),
    5: dict(name="split_i8_crt", traffic_kernel="k_crt_reduce", slice_bytes=22.0,
            mode="split_i8_crt (36-bit integers per operand column, exact products modulo 11 "
                 "coprime moduli <= 255 on INT8 MFMA, Chinese-remainder reconstruction, FP64 "
                 "scaling per segment)",
            per_fp64=CRT_I8_PER_FP64, peak=INT8_MFMA_PEAK_TOPS,
            unit="TOP/s (INT8 MFMA ops issued)",
            kernel="residues + modular reduction + reconstruction (phase 2..3)",
            phase="slice_and_reduce_HS"),
    3: dict(name="fp64_3m", traffic_kernel="k_reduce_3m", slice_bytes=16.0,
            mode="fp64_3m (complex FP64 with 3 real MFMA products per complex product: "
                 "T1 = pr qr, T2 = pi qi, T3 = (pr - pi)(qr + qi); Re = T1 + T2, Im = T3 - T1 + T2)",
            per_fp64=FP64_3M_PER_FP64, peak=FP64_MFMA_PEAK_TFLOPS,
            unit="TFLOP/s (FP64 MFMA flops issued)",
            kernel="k_reduce, 3M form", phase="reduce_HS"),
}


def split_bench(p, steps: int, warmup: int, fp64_ms: float, hip, mode: int, n_cols: int = 12,
                atom_kw=None):
    """Split-precision (or 3M) form on the same workload: time and speedup
    over the FP64 path. Returns (result, sample): the sample holds seeded
    columns of its H and S, which the CPU-baseline leg compares with the
    oracle (cpu_baseline_errors)."""
    import torch
    from paper_1611_00606_amd import DeviceBuild
    from paper_1611_00606_amd.flops import algorithmic_flops, reduction_flops

    m = SPLIT_MODES[mode]
    run = DeviceBuild.from_problem(p, device="cuda:0", mode=mode, **(atom_kw or {}))
    ph, total = timed_builds(run, steps, warmup, hip)
    info = run.info.cpu().numpy()
    rng = np.random.default_rng(1234)
    cols = np.sort(rng.choice(p.N_G, size=min(n_cols, p.N_G), replace=False))
    idx = torch.as_tensor(cols, device=run.H.device)
    Hc = run.H.index_select(1, idx).cpu().numpy()
    Sc = run.S.index_select(1, idx).cpu().numpy()
    del run
    torch.cuda.empty_cache()
    f = algorithmic_flops(p.nl, p.N_G, info)
    issued = m["per_fp64"] * reduction_flops(p.nl, p.N_G) / (ph[2] * 1e-3) / 1e12
    # split forms read six sliced operands (16 B per complex element for the
    # FP16 slices, 10 B for the INT8 ones); the 3M form the four FP64 ones
    alg_bytes = reduction_bytes(p.K, p.N_G, m["slice_bytes"], 6 if mode in (1, 2, 4, 5) else 4)
    if mode == 5:
        # the modular reduction writes each segment's residues (5 segments x
        # 11 moduli x 2 bytes per lower-triangle element) instead of H and S
        alg_bytes += (55.0 - 16.0) * float(p.N_G) ** 2
    traffic = measured_traffic(p.name, m["traffic_kernel"])
    return {
        "mode": m["mode"],
        "ms_per_step": round(total, 3),
        "value": round(f / (total * 1e-3) / 1e12, 3),
        "unit": "TFLOP/s (FP64-equivalent)",
        "speedup_vs_fp64": round(fp64_ms / total, 3),
        "phases_ms": {"prep_cholesky": round(float(ph[0]), 4), "atom_products": round(float(ph[1]), 4),
                      m["phase"]: round(float(ph[2]), 4), "mirror": round(float(ph[3]), 4)},
        "roofline": {
            "kernel": m["kernel"],
            "bound": "mfma",
            "achieved": round(issued, 2),
            "peak": m["peak"],
            "unit": m["unit"],
            "frac": round(issued / m["peak"], 4),
            "traffic": traffic,
            "traffic_unit": TRAFFIC_UNIT + f" ({m['traffic_kernel']})",
            "algorithmic_bytes": alg_bytes,
            "traffic_ratio": round(traffic / alg_bytes, 2) if traffic is not None else None,
        },
        "rel_err_H": None,
        "rel_err_S": None,
        "err_sample": f"{len(cols)} seeded columns of H and S vs the CPU oracle "
                      "(evaluated in the CPU-baseline leg; null with --no-cpu-baseline)",
    }, (cols, Hc, Sc)


def cpu_baseline_errors(p, samples):
    """CPU-baseline leg: the oracle's columns of H and S for the columns each
    GPU form sampled, and each form's relative Frobenius error on them."""
    import oracle
    cache, out = {}, {}
    for name, (cols, Hc, Sc) in samples.items():
        key = tuple(int(c) for c in cols)
        if key not in cache:
            cache[key] = (oracle.hamiltonian_columns(p.A, p.B, p.T_AA, p.T_AB, p.T_BB, p.nl, cols),
                          oracle.overlap_columns(p.A, p.B, p.U, p.nl, cols))
        Hr, Sr = cache[key]
        out[name] = (float(np.linalg.norm(Hc - Hr) / np.linalg.norm(Hr)),
                     float(np.linalg.norm(Sc - Sr) / np.linalg.norm(Sr)))
    return out


def batching_bench(seed: int, steps: int, hip):
    """Batched form on the mixed-N_L workload (128 atoms, N_L 16/49/81/121 x 32,
    N_G = 6000, 6 failing atoms): per-atom stage (preparation + products) and
    whole build with separate launches, with the batched launch on the
    built-in tile shapes, and with the shapes the autotuner picks."""
    import torch
    from hs_inputs import make_config
    from paper_1611_00606_amd import DeviceBuild
    from paper_1611_00606_amd.flops import paper_step_flops
    from paper_1611_00606_amd.tuning import autotune

    p = make_config("batching", seed=seed)
    t0 = time.perf_counter()
    tuning, report = autotune(sorted(set(p.nl.tolist())), p.N_G, reps=3)
    tune_s = time.perf_counter() - t0
    res, info = {}, None
    for name, kw in (("separate", {}), ("batched_default", {"batch": 1}),
                     ("batched_tuned", {"batch": 1, "tuning": tuning})):
        run = DeviceBuild.from_problem(p, device="cuda:0", **kw)
        ph, total = timed_builds(run, steps, 1, hip)
        info = run.info.cpu().numpy()
        res[name] = (float(ph[0] + ph[1]), total)
        del run
        torch.cuda.empty_cache()
    f = paper_step_flops(p.nl, p.N_G, info)
    f_atoms = sum(f[k] for k in ("loop1_zgemm_TBA_A", "loop1_zhemm_TBB_B", "loop2_zpotrf",
                                 "loop2_ztrmm_Y", "loop2_zhemm_X"))
    return {
        "workload": f"batching: N_A={p.N_A}, N_L 16/49/81/121 x 32, N_G={p.N_G}, "
                    f"{int((info != 0).sum())} failing atoms",
        "atom_stage_ms": {k: round(v[0], 4) for k, v in res.items()},
        "build_ms": {k: round(v[1], 3) for k, v in res.items()},
        "atom_stage_tflops": {k: round(f_atoms / (v[0] * 1e-3) / 1e12, 3) for k, v in res.items()},
        "speedup_atom_stage_tuned_vs_separate": round(res["separate"][0] / res["batched_tuned"][0], 3),
        "atom_stage_frac_of_fp64_peak": round(f_atoms / (res["batched_tuned"][0] * 1e-3) / 1e12
                                              / FP64_MFMA_PEAK_TFLOPS, 4),
        "autotune": {str(v): {"bm_bn": list(r["bm_bn"]), "ms_per_shape": r["ms"]}
                     for v, r in report.items()},
        "autotune_s": round(tune_s, 2),
        "atom_stage_flops": f_atoms,
    }


def serving_inputs(seed: int, K: int, threads: int = 16):
    """The serving stream's requests: N_G of each (integer-uniform in
    [1500, 9000]) and its own seeded A, B, drawn once (in parallel) into
    pinned host memory and shared by every mode's run."""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    from hs_inputs import serving_request_ab, serving_requests
    sizes = [int(x) for x in serving_requests(seed)]

    def one(r):
        A, B = serving_request_ab(seed, r, sizes[r], K)
        pa = torch.empty(A.shape, dtype=torch.complex128, pin_memory=True)
        pb = torch.empty(B.shape, dtype=torch.complex128, pin_memory=True)
        pa.numpy()[...] = A
        pb.numpy()[...] = B
        return pa, pb

    with ThreadPoolExecutor(min(threads, len(sizes))) as ex:
        data = list(ex.map(one, range(len(sizes))))
    return sizes, data


def serving_bench(seed: int, sizes, data, n_slots: int = 4, arena_gb: float = 24.0,
                  load: float = 0.8, streams: int = 5, mode: int = 0, n_check: int = 8,
                  admission: int = 0, max_bypass: int = 0):
    """Serving form: 64 k-point requests on one resident atom set (64 atoms,
    N_L = 64), N_G integer-uniform in [1500, 9000], each with its own seeded
    A, B in pinned host memory (serving_inputs), Poisson arrivals at `load` /
    (mean latency of a request served alone), continuous batching on
    `n_slots` streams with admission by device footprint into an arena of
    `arena_gb` GB (admission policy `admission`: 0 arrival order, 1 later
    requests may pass one waiting for space, at most `max_bypass` times); a
    request's host->device copy of A, B is part of its service. The same 64 requests are served under `streams` independently
    seeded arrival sequences; latency percentiles pool all of them. Then an
    untimed pass serves `n_check` of the requests (the smallest and largest
    N_G among them) in one burst and keeps seeded columns of each result,
    which the CPU-baseline leg compares with the oracle. Returns (summary,
    samples)."""
    from hs_inputs import serving_arrivals, serving_atoms
    from paper_1611_00606_amd.flops import algorithmic_flops
    from paper_1611_00606_amd.serving import (Context, ServingLoop, device_columns_to_host,
                                              percentile, summarize)

    atoms = serving_atoms(seed)
    ctx = Context(atoms.T_AA, atoms.T_AB, atoms.T_BB, atoms.U, atoms.nl)
    info = ctx.info()
    reqs = [{"id": r, "N_G": n, "A_ptr": data[r][0].data_ptr(), "B_ptr": data[r][1].data_ptr(),
             "ld": n} for r, n in enumerate(sizes)]
    arena = int(arena_gb * 1e9)
    loop = ServingLoop(ctx, n_slots, arena, mode=mode, admission=admission, max_bypass=max_bypass)
    # calibration: a spread of requests served one at a time
    cal_ids = [int(i) for i in np.argsort(sizes)[np.linspace(0, len(sizes) - 1, 8).astype(int)]]
    alone = []
    for i in cal_ids:
        rec = loop.run([dict(reqs[i], id=1000 + i)], [0.0])
        alone.append(rec[0]["latency"])
    mean_alone = float(np.mean(alone))
    rate = load / mean_alone
    runs, offered, peak = [], [], 0
    for j in range(streams):
        arrivals = serving_arrivals(seed + j, len(reqs), rate)
        arrivals = arrivals - arrivals[0]
        offered.append((len(reqs) - 1) / arrivals[-1])
        runs.append(loop.run([dict(r, id=r["id"] + 10000 * j) for r in reqs], arrivals))
        peak = max(peak, loop.peak_bytes)
    # capacity: all requests at once (the stream is no longer rate-limited
    # by its arrivals; builds/s is what the slots and the arena sustain)
    sat = loop.run([dict(r, id=r["id"] + 30000) for r in reqs], [0.0] * len(reqs))
    sat_span = max(r["done"] for r in sat) - min(r["arrival"] for r in sat)
    # untimed check pass: n_check requests in one burst, seeded columns kept
    order = np.argsort(sizes)
    chk = [int(order[0]), int(order[-1])]
    for x in np.random.default_rng(seed + 77).permutation(len(sizes)):
        if len(chk) < n_check and int(x) not in chk:
            chk.append(int(x))
    samples = {}

    def keep(res):
        rid = int(res["id"]) - 20000
        n = int(res["N_G"])
        cols = np.sort(np.random.default_rng(rid).choice(n, size=4, replace=False))
        samples[rid] = (cols, device_columns_to_host(res["H"], n, cols),
                        device_columns_to_host(res["S"], n, cols))

    loop.run([dict(reqs[i], id=20000 + i) for i in chk], [0.0] * len(chk), on_result=keep)
    loop.close()
    ctx.close()
    flops_of = lambda n: algorithmic_flops(atoms.nl, n, info)  # noqa: E731
    per_stream = [summarize(r, flops_of) for r in runs]
    out = summarize([x for r in runs for x in r], flops_of)
    out["builds_per_s"] = float(np.mean([q["builds_per_s"] for q in per_stream]))
    out["tflops_fp64_equiv"] = float(np.mean([q["tflops_fp64_equiv"] for q in per_stream]))
    out["span_s"] = float(np.mean([q["span_s"] for q in per_stream]))
    out["requests"] = len(reqs)
    out["streams"] = streams
    out["latency_samples"] = len(reqs) * streams
    out["offered_rate_per_s"] = [round(x, 3) for x in offered]
    out.update({
        "mode": {0: "fp64", 1: "split_f16", 2: "split_i8", 3: "fp64_3m", 4: "split_bf16",
                 5: "split_i8_crt"}[mode],
        "workload": "64 requests, N_A=64 atoms, N_L=64, N_G uniform in [1500, 9000], each with "
                    "its own seeded A, B in pinned host memory, Poisson arrivals",
        "arrival_rate_per_s": rate,   # nominal Poisson rate; offered_rate_per_s is realized
        "load": load,
        "alone_mean_latency_ms": 1e3 * mean_alone,
        "alone_p99_latency_ms": 1e3 * percentile(alone, 99),
        "n_slots": n_slots,
        "admission": ("arrival order" if admission == 0 else
                      f"bypass (a waiting request is passed at most {max_bypass} times)"),
        "arena_gb": arena_gb,
        "peak_arena_gb": peak / 1e9,
        "saturated_builds_per_s": len(sat) / sat_span,
        "saturated_tflops_fp64_equiv": sum(flops_of(r["N_G"]) for r in sat) / sat_span / 1e12,
        "checked_requests": chk,
        "max_rel_err_H": None,
        "max_rel_err_S": None,
        "err_sample": f"4 seeded columns of H and S of each of {len(chk)} requests served "
                      "together in an untimed burst, vs the CPU oracle (evaluated in the "
                      "CPU-baseline leg; null with --no-cpu-baseline)",
    })
    return {k: (round(v, 4) if isinstance(v, float) else v) for k, v in out.items()}, samples


def serving_errors(seed: int, sizes, data, samples):
    """CPU-baseline leg: the oracle's columns for each checked served request;
    the largest relative column error of H and of S."""
    import oracle
    from hs_inputs import serving_atoms
    atoms = serving_atoms(seed)
    eh = es = 0.0
    for rid, (cols, Hc, Sc) in samples.items():
        A, B = data[rid][0].numpy(), data[rid][1].numpy()
        Hr = oracle.hamiltonian_columns(A, B, atoms.T_AA, atoms.T_AB, atoms.T_BB, atoms.nl, cols)
        Sr = oracle.overlap_columns(A, B, atoms.U, atoms.nl, cols)
        eh = max(eh, float(np.max(np.linalg.norm(Hc - Hr, axis=0) / np.linalg.norm(Hr, axis=0))))
        es = max(es, float(np.max(np.linalg.norm(Sc - Sr, axis=0) / np.linalg.norm(Sr, axis=0))))
    return eh, es


def failure_branch_bench(p, steps: int, hip, atom_kw, counts=(0, 3, 32), seed: int = 0):
    """The paper's failure branch (Sec. 2: T^AA_a without a Cholesky factor)
    inside the reduction: the same workload with 0, 3 and 32 atoms whose
    T^AA_a is shifted by -2 lambda_max (negative definite), timed the same
    way. Their rows contribute A_a^H X_a to H's lower triangle in the same
    K-loop as the HPD rows' Y_a^H Y_a, so the reduction's time should not
    depend on how many atoms fail."""
    from paper_1611_00606_amd import DeviceBuild
    from paper_1611_00606_amd.flops import reduction_flops
    import torch
    rng = np.random.default_rng(seed)
    order = rng.permutation(p.N_A)
    out = {"workload": f"N_A={p.N_A}, N_L={int(p.nl[0])}, N_G={p.N_G}, K={p.K}; failing atoms "
                       "get T^AA - 2 lambda_max I", "reduce_ms": {}, "build_ms": {},
           "reduce_tflops": {}, "info_nonzero": {}}
    for n_fail in counts:
        q = p.copy() if n_fail else p
        for a in sorted(int(x) for x in order[:n_fail]):
            t = q.t_block("T_AA", a).copy()
            lam = float(np.linalg.eigvalsh(t).max())
            t[np.diag_indices(t.shape[0])] -= 2.0 * lam
            q.set_t_block("T_AA", a, t)
        run = DeviceBuild.from_problem(q, device="cuda:0", **(atom_kw or {}))
        ph, total = timed_builds(run, steps, 1, hip)
        out["info_nonzero"][str(n_fail)] = int((run.info.cpu().numpy() != 0).sum())
        out["reduce_ms"][str(n_fail)] = round(float(ph[2]), 3)
        out["build_ms"][str(n_fail)] = round(total, 3)
        out["reduce_tflops"][str(n_fail)] = round(
            reduction_flops(q.nl, q.N_G) / (float(ph[2]) * 1e-3) / 1e12, 3)
        del run, q
        torch.cuda.empty_cache()
    r = out["reduce_ms"]
    out["max_rel_diff_reduce_ms"] = round(
        (max(r.values()) - min(r.values())) / min(r.values()), 4)
    return out


# Tab. 6 of the paper (NaCl, K_max = 4.0, two K20Xm through cuBLAS-XT): rates
# of the five large products, GFLOP/s; and the end-to-end times of Tabs. 2
# and 3 (K_max = 4.0, 16 cores + 2 GPUs), seconds. Context only: other
# hardware, and this library fuses the five products into two reductions.
PAPER_TAB6_GFLOPS = {"S1_zherk_A": 1974.63, "S2_zherk_UB": 1956.72, "H1_zher2k": 1818.57,
                     "H2_zgemm_failing": 1859.72, "H3_zherk_Y": 1816.66}
PAPER_KMAX4_SECONDS = {"nacl_kmax4": 46.97, "auag_kmax4": 43.54}


def paper_shape_bench(name: str, seed: int, steps: int, hip):
    """One build at the shape of one of the paper's systems at K_max = 4.0
    (Tab. 1), synthetic values, in the timed configuration (batched per-atom
    stage, autotuned tile shapes)."""
    import torch
    from hs_inputs import make_config
    from paper_1611_00606_amd import DeviceBuild
    from paper_1611_00606_amd.flops import algorithmic_flops, reduction_flops
    from paper_1611_00606_amd.tuning import autotune
    p = make_config(name, seed=seed)
    tuning, _ = autotune(sorted(set(p.nl.tolist())), p.N_G, reps=3)
    run = DeviceBuild.from_problem(p, device="cuda:0", batch=1, tuning=tuning)
    ph, total = timed_builds(run, steps, 1, hip)
    info = run.info.cpu().numpy()
    del run
    torch.cuda.empty_cache()
    f = algorithmic_flops(p.nl, p.N_G, info)
    f_red = reduction_flops(p.nl, p.N_G)
    return {
        "workload": f"{name}: N_A={p.N_A}, N_L={int(p.nl[0])}, N_G={p.N_G}, K={p.K} "
                    "(the paper's system shape at K_max = 4.0, synthetic values)",
        "ms_per_build": round(total, 3),
        "tflops": round(f / (total * 1e-3) / 1e12, 3),
        "pct_of_fp64_mfma_peak": round(100 * f / (total * 1e-3) / 1e12 / FP64_MFMA_PEAK_TFLOPS, 2),
        "phases_ms": {"atom_stage": round(float(ph[0] + ph[1]), 3),
                      "reduce_HS": round(float(ph[2]), 3), "mirror": round(float(ph[3]), 3)},
        "reduce_gflops": round(f_red / (float(ph[2]) * 1e-3) / 1e9, 1),
        "paper_context": {
            "tab6_gflops_nacl_kmax4_2xK20Xm": PAPER_TAB6_GFLOPS,
            "end_to_end_s_16cores_2xK20Xm": PAPER_KMAX4_SECONDS[name],
            "note": "the paper's five products run separately; here S1+S2 and H1+H2+H3 are two "
                    "fused lower-triangle reductions in one launch, reduce_gflops is their "
                    "combined rate",
        },
        "failing_atoms": int((info != 0).sum()),
    }


def gep_bench(run, steps: int, hip):
    """Reduction of the generalized eigenproblem (S = L L^H, Ht = L^-1 H L^-H)
    applied to the H and S the timed build produced, timed with HIP events on the
    launch stream; then the same with the products in the 3M form."""
    import torch
    from paper_1611_00606_amd import HS_FP64, HS_FP64_3M, hs_gep_reduce, hs_gep_workspace_bytes
    N = int(run.H.shape[0])
    dev = run.H.device
    L = torch.empty_like(run.H)
    Ht = torch.empty_like(run.H)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    ws = torch.empty(hs_gep_workspace_bytes(N), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    rt = hip.rt
    rt.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]

    def timed(mode):
        hs_gep_reduce(run.H, run.S, L, Ht, info=info, workspace=ws, stream=stream, mode=mode)
        torch.cuda.synchronize()
        ms = []
        for _ in range(steps):
            e0, e1 = hip.create(2)
            assert rt.hipEventRecord(ctypes.c_void_p(e0), ctypes.c_void_p(stream.cuda_stream)) == 0
            hs_gep_reduce(run.H, run.S, L, Ht, info=info, workspace=ws, stream=stream, mode=mode)
            assert rt.hipEventRecord(ctypes.c_void_p(e1), ctypes.c_void_p(stream.cuda_stream)) == 0
            torch.cuda.synchronize()
            ms.append(hip.elapsed_ms(e0, e1))
            hip.destroy([e0, e1])
        res = float(torch.linalg.matrix_norm(L @ L.conj().T - run.S) / torch.linalg.matrix_norm(run.S))
        return ms, res

    ms, res = timed(HS_FP64)
    med = float(np.median(ms))
    # the minimal count of the standard route: zpotrf (4/3 N^3) + zhegst (4 N^3)
    f_min = 16.0 / 3.0 * N ** 3
    # executed: factor and inverse 8/3 N^3, then V = H L^-H and Ht (16/3 N^3), or from
    # N = 4096 on WH = (L^-1 lower(H))^H and the two-term Ht (4 N^3)
    f_exec = (20.0 / 3.0 if N >= 4096 else 8.0) * N ** 3
    out = {
        "N": N, "info": int(info.item()),
        "ms_median": round(med, 3), "ms_min": round(float(min(ms)), 3),
        "tflops": round(f_min / (med * 1e-3) / 1e12, 2),
        "pct_of_fp64_mfma_peak": round(100 * f_min / (med * 1e-3) / 1e12
                                       / FP64_MFMA_PEAK_TFLOPS, 1),
        "tflops_executed": round(f_exec / (med * 1e-3) / 1e12, 2),
        "pct_of_fp64_mfma_peak_executed": round(100 * f_exec / (med * 1e-3) / 1e12
                                                / FP64_MFMA_PEAK_TFLOPS, 1),
        "residual_S_LLH": res,
        "flop_counts": "tflops: 16/3 N^3, the zpotrf (4/3 N^3) + zhegst (4 N^3) count of the "
                       "standard reduction; executed: 20/3 N^3 from N = 4096 (8 N^3 below), the "
                       "explicit-inverse route this library takes",
    }
    ms3, res3 = timed(HS_FP64_3M)
    med3 = float(np.median(ms3))
    out["fp64_3m"] = {
        "mode": "products on the tiles in the 3M form (3 real MFMA products per complex product)",
        "info": int(info.item()),
        "ms_median": round(med3, 3), "ms_min": round(float(min(ms3)), 3),
        "tflops_fp64_equiv": round(f_min / (med3 * 1e-3) / 1e12, 2),
        "speedup_vs_fp64": round(med / med3, 3),
        "residual_S_LLH": res3,
    }
    del L, Ht, ws
    torch.cuda.empty_cache()
    return out


def cpu_baseline_gep(n_full: int, n: int = 2000):
    """The oracle's reduction (column Cholesky + scipy triangular solves) on a
    bounded sample, N = n, and that time scaled by (n_full / n)^3."""
    import oracle as O
    rng = np.random.default_rng(0)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    S = A @ A.conj().T + n * np.eye(n)
    H = A + A.conj().T
    t0 = time.perf_counter()
    O.gep_reduce(H, S)
    t = time.perf_counter() - t0
    return {"kind": "oracle", "sample": f"random Hermitian pair, N = {n}",
            "ms": round(1e3 * t, 1), "ms_scaled_to_full_N": round(1e3 * t * (n_full / n) ** 3, 1),
            "cores": _blas_threads()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="precision")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="host time for the Alg. 1 sample of the CPU baseline (the oracle "
                         "always runs on the whole workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the serving-form measurement (k-point builds/s, p50/p99)")
    ap.add_argument("--no-split", action="store_true",
                    help="skip the split-precision and 3M measurements")
    ap.add_argument("--split-modes", default="1,2,3,4,5",
                    help="alternative reduction modes to measure (1 = HS_SPLIT_F16, "
                         "2 = HS_SPLIT_I8, 3 = HS_FP64_3M, 4 = HS_SPLIT_BF16, "
                         "5 = HS_SPLIT_I8_CRT)")
    ap.add_argument("--per-atom", choices=["batched", "separate"], default="batched",
                    help="per-atom stage of the timed builds: the batched persistent launch with "
                         "autotuned tile shapes, or separate preparation and product launches")
    ap.add_argument("--no-batching", action="store_true",
                    help="skip the batched per-atom stage measurement")
    ap.add_argument("--no-gep", action="store_true",
                    help="skip the generalized eigenproblem reduction of the built H and S")
    ap.add_argument("--no-failure-branch", action="store_true",
                    help="skip the reduction timed with 0, 3 and 32 failing atoms")
    ap.add_argument("--no-paper-shapes", action="store_true",
                    help="skip the builds at the paper's NaCl and AuAg shapes (K_max = 4.0)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run one plain device copy of MIB MiB (to scale HBM byte "
                         "counters against a kernel of known traffic) and exit")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the H/S build here is a single-GPU path "
              "(a sharding over GPUs is designed but not built). Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from hs_inputs import make_config
    from paper_1611_00606_amd import DeviceBuild, HS_NUM_PHASE_EVENTS
    from paper_1611_00606_amd.flops import algorithmic_flops, reduction_flops

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        n = args.copy_calibration << 20
        src = torch.ones(n // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": n, "bytes_written": n}), flush=True)
        return
    p = make_config(args.config, seed=args.seed)
    print(f"bench: config {args.config} N_A={p.N_A} N_G={p.N_G} K={p.K}", file=sys.stderr, flush=True)
    atom_kw = {}
    if args.per_atom == "batched":
        # set-up, outside the timed region: tile shapes per N_L for this N_G
        from paper_1611_00606_amd.tuning import autotune
        tuning, _ = autotune(sorted(set(p.nl.tolist())), p.N_G, reps=3)
        atom_kw = {"batch": 1, "tuning": tuning}
    run = DeviceBuild.from_problem(p, device="cuda:0", **atom_kw)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        run.run(stream=stream)
    torch.cuda.synchronize()
    info = run.info.cpu().numpy()

    hip = HipEvents()
    evs = [hip.create(HS_NUM_PHASE_EVENTS) for _ in range(args.steps)]
    t_start, t_end = hip.create(2)
    torch.cuda.synchronize()
    rt = hip.rt
    rt.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    assert rt.hipEventRecord(ctypes.c_void_p(t_start), ctypes.c_void_p(stream.cuda_stream)) == 0
    w0 = time.perf_counter()
    for k in range(args.steps):
        run.run(stream=stream, phase_events=evs[k])
    assert rt.hipEventRecord(ctypes.c_void_p(t_end), ctypes.c_void_p(stream.cuda_stream)) == 0
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    total_ms = hip.elapsed_ms(t_start, t_end)
    ms_step = total_ms / args.steps
    phases = np.array([[hip.elapsed_ms(e[i], e[i + 1]) for i in range(HS_NUM_PHASE_EVENTS - 1)]
                       for e in evs])
    ph_mean = phases.mean(axis=0)
    per_build = phases.sum(axis=1)
    hip.destroy([e for es in evs for e in es] + [t_start, t_end])

    f_alg = algorithmic_flops(p.nl, p.N_G, info)
    value = f_alg / (ms_step * 1e-3) / 1e12
    f_red = reduction_flops(p.nl, p.N_G)
    red_ms = float(ph_mean[2])
    achieved = f_red / (red_ms * 1e-3) / 1e12

    traffic = measured_traffic(args.config)
    out = {
        "metric": "H+S build FP64-equiv TFLOP/s (% MFMA peak); k-point builds/s + p99 latency",
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128 (f64)",
        "data": "synthetic",
        "pct_of_fp64_mfma_peak": round(100 * value / FP64_MFMA_PEAK_TFLOPS, 2),
        "config": {
            "workload": f"{args.config}: one k-point H+S build, N_A={p.N_A}, "
                        f"N_L={sorted(set(p.nl.tolist()))}, N_G={p.N_G}, plain FP64 path",
            "N_A": p.N_A, "N_L": sorted(set(p.nl.tolist())), "N_G": p.N_G, "K": p.K,
            "failing_atoms": int((info != 0).sum()), "seed": args.seed,
            "algorithmic_flops": f_alg,
        },
        "per_atom_stage": ("batched: per-atom Cholesky and products in one persistent launch, "
                           "autotuned tile shapes (phase 'atom_products' covers both)")
                          if args.per_atom == "batched" else "separate launches",
        "phases_ms": {
            "prep_cholesky": round(float(ph_mean[0]), 4),
            "atom_products": round(float(ph_mean[1]), 4),
            "reduce_HS": round(float(ph_mean[2]), 4),
            "mirror": round(float(ph_mean[3]), 4),
        },
        "atom_stage": atom_stage_rates(p, info, float(ph_mean[0] + ph_mean[1])),
        "build_ms_stats": {"median": round(float(np.median(per_build)), 3),
                           "min": round(float(np.min(per_build)), 3),
                           "p90": round(float(np.percentile(per_build, 90)), 3)},
        "wall_s_timed_region": round(wall, 3),
        "roofline": {
            "kernel": "k_reduce",
            "bound": "mfma",
            "achieved": round(achieved, 3),
            "peak": FP64_MFMA_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved / FP64_MFMA_PEAK_TFLOPS, 4),
            "traffic": traffic,
            "traffic_unit": TRAFFIC_UNIT,
            "algorithmic_bytes": reduction_bytes(p.K, p.N_G),
            "traffic_ratio": (round(traffic / reduction_bytes(p.K, p.N_G), 2)
                              if traffic is not None else None),
            "algorithmic_bytes_def": "16 (4 K N_G + N_G^2): A, B, Z, W read once, two lower "
                                     "triangles written",
        },
        "cpu_baseline": None,
    }
    if not args.no_gep:
        print("bench: generalized eigenproblem reduction", file=sys.stderr, flush=True)
        out["gep"] = gep_bench(run, max(3, args.steps // 2), HipEvents())
    del run
    torch.cuda.empty_cache()
    out["hs_build_sync_wall_ms"] = sync_build_wall_ms(p)
    samples = {}   # GPU columns of the alternative forms, checked in the CPU-baseline leg
    if not args.no_split:
        print("bench: split precision and 3M", file=sys.stderr, flush=True)
        hip = HipEvents()
        for mode in [int(m) for m in args.split_modes.split(",") if m]:
            name = SPLIT_MODES[mode]["name"]
            out[name], samples[name] = split_bench(p, max(3, args.steps // 2), 1, ms_step, hip,
                                                   mode, atom_kw=atom_kw)
    if not args.no_failure_branch:
        print("bench: failure branch (0, 3, 32 failing atoms)", file=sys.stderr, flush=True)
        out["failure_branch"] = failure_branch_bench(p, max(3, args.steps // 2), HipEvents(),
                                                     atom_kw, seed=args.seed)
    if not args.no_batching:
        print("bench: batched per-atom stage", file=sys.stderr, flush=True)
        out["batching"] = batching_bench(args.seed, max(3, args.steps // 2), HipEvents())
    serving_samples = {}
    if not args.no_serving:
        print("bench: serving stream inputs (64 requests, pinned host memory)", file=sys.stderr,
              flush=True)
        from hs_inputs import SERVING
        sizes, sdata = serving_inputs(args.seed, SERVING["N_A"] * SERVING["N_L"])
        modes = [0] + ([1, 2, 3, 5] if not args.no_split else [])
        for mode in modes:
            key = {0: "serving", 1: "serving_split_f16", 2: "serving_split_i8",
                   3: "serving_fp64_3m", 5: "serving_split_i8_crt"}[mode]
            print(f"bench: serving stream, {key}", file=sys.stderr, flush=True)
            out[key], serving_samples[key] = serving_bench(args.seed, sizes, sdata, mode=mode)
        print("bench: serving stream, bypass admission", file=sys.stderr, flush=True)
        out["serving_bypass"], serving_samples["serving_bypass"] = serving_bench(
            args.seed, sizes, sdata, mode=0, admission=1, max_bypass=4)
        out["kpoint_builds_per_s"] = out["serving"]["builds_per_s"]
        out["p99_latency_ms"] = out["serving"]["p99_latency_ms"]
    if not args.no_paper_shapes:
        out["paper_shapes"] = {}
        for name in ("nacl_kmax4", "auag_kmax4"):
            print(f"bench: paper shape {name}", file=sys.stderr, flush=True)
            out["paper_shapes"][name] = paper_shape_bench(name, args.seed, 3, HipEvents())
    if not args.no_cpu_baseline:
        print("bench: CPU baseline (oracle on the whole workload)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(p, args.cpu_seconds)
        for name, (eh, es) in cpu_baseline_errors(p, samples).items():
            out[name]["rel_err_H"], out[name]["rel_err_S"] = eh, es
        for key, smp in serving_samples.items():
            out[key]["max_rel_err_H"], out[key]["max_rel_err_S"] = serving_errors(
                args.seed, sizes, sdata, smp)
        if "gep" in out:
            out["gep"]["cpu_baseline"] = cpu_baseline_gep(out["gep"]["N"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
