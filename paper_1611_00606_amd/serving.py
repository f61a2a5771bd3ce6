"""Serving form: a stream of k-point builds on one resident atom set.

`Context` owns an hs_ctx (atom data resident on the device, Cholesky factors
and failure flags cached: they do not depend on the k-point). `ServingLoop`
drives an hs_server: requests arrive on a schedule, are submitted when they
arrive, and the native server admits them as slots and arena memory free up
(continuous batching), copies their inputs, builds them on separate HIP
streams and reports completion times. This module is the host control loop
only; admission, memory management, copies and builds are in the library.
"""

from __future__ import annotations

import ctypes
import time
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np

from . import _binding as B


class Context:
    """Resident atom data (T^AA, T^AB, T^BB, U) on one device."""

    def __init__(self, T_AA, T_AB, T_BB, U, nl, device="cuda:0", stream=None):
        import torch
        nl = np.asarray(nl, dtype=np.int32)
        self.N_A = int(nl.shape[0])
        self.uniform = bool(np.all(nl == nl[0]))
        self.nl = nl
        dev = torch.device(device)

        def up(x):
            return torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex128)).to(dev)

        t = [up(x) for x in (T_AA, T_AB, T_BB, U)]
        self.handle = B.hs_ctx_create(*t, self.N_A, int(nl[0]) if self.uniform else 0,
                                      None if self.uniform else nl, stream=stream)
        self.K = B.hs_ctx_rows(self.handle)
        self.device = dev

    def info(self) -> np.ndarray:
        return B.hs_ctx_info(self.handle, self.N_A)

    def footprint_bytes(self, n_g: int, mode: int = B.HS_FP64) -> int:
        return B.hs_ctx_footprint_bytes(self.handle, n_g, mode)

    def workspace_bytes(self, n_g: int, mode: int = B.HS_FP64) -> int:
        return B.hs_ctx_workspace_bytes(self.handle, n_g, mode)

    def build(self, A, Bm, n_g, H, S, workspace, stream=None, phase_events=None,
              mode: int = B.HS_FP64, batch: int = 0, tuning=None):
        return B.hs_ctx_build(self.handle, A, Bm, n_g, H, S, workspace=workspace, stream=stream,
                              phase_events=phase_events, mode=mode, batch=batch, tuning=tuning)

    def close(self):
        if self.handle:
            B.hs_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _hip():
    import torch  # noqa: F401  (the HIP runtime torch ships)
    rt = ctypes.CDLL("libamdhip64.so.7")
    rt.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    rt.hipMemcpy.restype = ctypes.c_int
    sz = ctypes.c_size_t
    rt.hipMemcpy2D.argtypes = [ctypes.c_void_p, sz, ctypes.c_void_p, sz, sz, sz, ctypes.c_int]
    rt.hipMemcpy2D.restype = ctypes.c_int
    return rt


def device_matrix_to_host(ptr: int, n: int) -> np.ndarray:
    """Copy an [n][n] complex128 device matrix (a served result) to the host."""
    out = np.empty((n, n), np.complex128)
    rc = _hip().hipMemcpy(out.ctypes.data, ptr, out.nbytes, 2)  # device to host
    if rc != 0:
        raise RuntimeError(f"hipMemcpy failed ({rc})")
    return out


def device_columns_to_host(ptr: int, n: int, cols: Sequence[int]) -> np.ndarray:
    """Columns `cols` of an [n][n] complex128 device matrix, as an [n][len(cols)]
    host array (one strided copy per column)."""
    out = np.empty((len(cols), n), np.complex128)
    rt = _hip()
    for j, g in enumerate(cols):
        rc = rt.hipMemcpy2D(out[j].ctypes.data, 16, ptr + 16 * int(g), 16 * n, 16, n, 2)
        if rc != 0:
            raise RuntimeError(f"hipMemcpy2D failed ({rc})")
    return out.T.copy()


def percentile(x: Sequence[float], q: float) -> float:
    """Nearest-rank percentile."""
    s = sorted(x)
    if not s:
        return float("nan")
    k = max(1, int(np.ceil(q / 100.0 * len(s))))
    return float(s[k - 1])


class ServingLoop:
    """One hs_server over a Context: n_slots streams and a device arena."""

    def __init__(self, ctx: Context, n_slots: int, arena_bytes: int, mode: int = B.HS_FP64,
                 admission: int = B.HS_ADMIT_FIFO, max_bypass: int = 0):
        self.ctx = ctx
        self.mode = int(mode)
        self.handle = B.hs_server_create(ctx.handle, n_slots, arena_bytes, mode)
        B.hs_server_set_admission(self.handle, admission, max_bypass)
        self.arena_bytes = int(arena_bytes)
        self.n_slots = int(n_slots)

    def run(self, requests: List[Dict], arrivals: Sequence[float],
            on_result: Optional[Callable[[Dict], None]] = None,
            poll_sleep: float = 2e-4) -> List[Dict]:
        """Serve `requests` (dicts with id, N_G, A_ptr, B_ptr, ld: host
        pointers to [K][ld] complex128 rows) arriving at `arrivals` seconds
        after the start. Each completed result is passed to on_result (device
        H, S valid during the call) and then released. Returns one record per
        request with its arrival, admit and completion times (server clock)
        and its latency = completion - arrival."""
        srv = self.handle
        order = np.argsort(np.asarray(arrivals), kind="stable")
        t0 = B.hs_server_now(srv)
        sched = {requests[i]["id"]: t0 + float(arrivals[i]) for i in range(len(requests))}
        recs: Dict[int, Dict] = {}
        peak = 0
        nxt = 0
        n = len(requests)
        while len(recs) < n:
            now = B.hs_server_now(srv)
            while nxt < n and t0 + float(arrivals[order[nxt]]) <= now:
                r = requests[order[nxt]]
                B.hs_server_submit(srv, r["id"], r["N_G"], r["A_ptr"], r["B_ptr"], r["ld"])
                nxt += 1
            ready = B.hs_server_progress(srv)
            peak = max(peak, B.hs_server_used_bytes(srv))
            got = False
            for _ in range(ready):
                res = B.hs_server_pop(srv)
                if res is None:
                    break
                got = True
                if res["status"] != 0:
                    raise B.HSError(res["status"], f"request {res['id']} failed")
                if on_result is not None:
                    on_result(res)
                B.hs_server_release(srv, res["id"])
                arr = sched[res["id"]]
                recs[res["id"]] = {"id": res["id"], "N_G": res["N_G"], "arrival": arr,
                                   "submit": res["t_submit"], "admit": res["t_admit"],
                                   "done": res["t_done"], "latency": res["t_done"] - arr}
            if not got:
                time.sleep(poll_sleep)
        self.peak_bytes = peak
        return [recs[r["id"]] for r in requests]

    def close(self):
        if self.handle:
            B.hs_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def summarize(recs: List[Dict], flops_of: Callable[[int], float]) -> Dict:
    """builds/s, p50/p99 latency and FP64-equivalent TFLOP/s of a served stream."""
    lat = [r["latency"] for r in recs]
    t_first = min(r["arrival"] for r in recs)
    t_last = max(r["done"] for r in recs)
    span = t_last - t_first
    flops = sum(flops_of(r["N_G"]) for r in recs)
    return {
        "requests": len(recs),
        "builds_per_s": len(recs) / span,
        "p50_latency_ms": 1e3 * percentile(lat, 50),
        "p99_latency_ms": 1e3 * percentile(lat, 99),
        "mean_latency_ms": 1e3 * float(np.mean(lat)),
        "tflops_fp64_equiv": flops / span / 1e12,
        "span_s": span,
    }
