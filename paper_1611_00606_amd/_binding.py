"""ctypes binding of libhsbuild.so: argument marshalling only.

Every function here has the name of the C entry point it calls (declared in
include/hs_build.h) and forwards device pointers of torch tensors, sizes and
the current HIP stream. No arithmetic of the build happens in Python, and
there is no fallback: if the HIP library is not built or cannot be loaded,
every call raises.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhsbuild.so")

HS_OK = 0
HS_ERR_HIP = 1
HS_ERR_WORKSPACE = 2
HS_ERR_NOMEM = 3
HS_ERR_UNSUPPORTED = 4
HS_FP64 = 0
HS_SPLIT_F16 = 1
HS_SPLIT_I8 = 2
HS_FP64_3M = 3
HS_SPLIT_BF16 = 4
HS_SPLIT_I8_CRT = 5
HS_MAX_NL = 128
HS_NUM_PHASE_EVENTS = 5
HS_NUM_TILE_CONFIGS = 8
HS_STATIC_SCRATCH_BYTES = 256 << 20
HS_ADMIT_FIFO = 0
HS_ADMIT_BYPASS = 1


class HSError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"hs_build status {status}: {message}")
        self.status = status


class hs_tuning(ctypes.Structure):
    _fields_ = [("cfg", ctypes.c_ubyte * (HS_MAX_NL + 1))]


class hs_options(ctypes.Structure):
    _fields_ = [
        ("stream", ctypes.c_void_p),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
        ("info", ctypes.c_void_p),
        ("mode", ctypes.c_int),
        ("nl_per_atom", ctypes.POINTER(ctypes.c_int32)),
        ("phase_events", ctypes.POINTER(ctypes.c_void_p)),
        ("batch", ctypes.c_int),
        ("tuning", ctypes.POINTER(hs_tuning)),
    ]


class hs_request(ctypes.Structure):
    _fields_ = [
        ("id", ctypes.c_int64),
        ("N_G", ctypes.c_int),
        ("A_host", ctypes.c_void_p),
        ("B_host", ctypes.c_void_p),
        ("ld", ctypes.c_int64),
    ]


class hs_result(ctypes.Structure):
    _fields_ = [
        ("id", ctypes.c_int64),
        ("N_G", ctypes.c_int),
        ("status", ctypes.c_int),
        ("H", ctypes.c_void_p),
        ("S", ctypes.c_void_p),
        ("t_submit", ctypes.c_double),
        ("t_admit", ctypes.c_double),
        ("t_done", ctypes.c_double),
    ]


_lib = None


def load_library() -> ctypes.CDLL:
    """Load libhsbuild.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    # torch ships its own HIP runtime (SONAME libamdhip64.so.7). Loading it
    # first makes this library bind to that same runtime instead of a second
    # copy, so torch's streams and device pointers are valid here.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
            "(hipcc, gfx950). There is no non-HIP fallback.")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32 = ctypes.c_void_p, ctypes.c_int
    lib.hs_build.argtypes = [vp] * 6 + [i32, i32, i32, vp, vp]
    lib.hs_build.restype = i32
    lib.hs_build_ex.argtypes = [vp] * 6 + [i32, i32, i32, vp, vp, ctypes.POINTER(hs_options)]
    lib.hs_build_ex.restype = i32
    lib.hs_build_static.argtypes = [vp] * 6 + [i32, i32, i32, vp, vp, ctypes.POINTER(hs_options)]
    lib.hs_build_static.restype = i32
    lib.hs_workspace_bytes.argtypes = [i32, ctypes.POINTER(ctypes.c_int32), i32, i32, i32]
    lib.hs_workspace_bytes.restype = ctypes.c_size_t
    lib.hs_status_string.argtypes = [i32]
    lib.hs_status_string.restype = ctypes.c_char_p
    sz = ctypes.c_size_t
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.hs_ctx_create.argtypes = [vp] * 4 + [i32, i32, i32p, vp, ctypes.POINTER(vp)]
    lib.hs_ctx_create.restype = i32
    lib.hs_ctx_rows.argtypes = [vp]
    lib.hs_ctx_rows.restype = i32
    lib.hs_ctx_info.argtypes = [vp, i32p]
    lib.hs_ctx_info.restype = i32
    lib.hs_ctx_workspace_bytes.argtypes = [vp, i32, i32]
    lib.hs_ctx_workspace_bytes.restype = sz
    lib.hs_ctx_footprint_bytes.argtypes = [vp, i32, i32]
    lib.hs_ctx_footprint_bytes.restype = sz
    lib.hs_ctx_build.argtypes = [vp, vp, vp, i32, vp, vp, ctypes.POINTER(hs_options)]
    lib.hs_ctx_build.restype = i32
    lib.hs_ctx_destroy.argtypes = [vp]
    lib.hs_ctx_destroy.restype = None
    lib.hs_server_create.argtypes = [vp, i32, sz, i32, ctypes.POINTER(vp)]
    lib.hs_server_create.restype = i32
    lib.hs_server_submit.argtypes = [vp, ctypes.POINTER(hs_request)]
    lib.hs_server_submit.restype = i32
    lib.hs_server_set_admission.argtypes = [vp, i32, i32]
    lib.hs_server_set_admission.restype = i32
    lib.hs_server_progress.argtypes = [vp]
    lib.hs_server_progress.restype = i32
    lib.hs_server_pop.argtypes = [vp, ctypes.POINTER(hs_result)]
    lib.hs_server_pop.restype = i32
    lib.hs_server_release.argtypes = [vp, ctypes.c_int64]
    lib.hs_server_release.restype = i32
    lib.hs_server_pending.argtypes = [vp]
    lib.hs_server_pending.restype = i32
    lib.hs_server_used_bytes.argtypes = [vp]
    lib.hs_server_used_bytes.restype = sz
    lib.hs_server_now.argtypes = [vp]
    lib.hs_server_now.restype = ctypes.c_double
    lib.hs_server_destroy.argtypes = [vp]
    lib.hs_server_destroy.restype = None
    ip = ctypes.POINTER(ctypes.c_int)
    lib.hs_tile_config.argtypes = [i32, ip, ip]
    lib.hs_tile_config.restype = i32
    lib.hs_autotune_atoms.argtypes = [i32p, i32, i32, i32, vp, ctypes.POINTER(hs_tuning),
                                      ctypes.POINTER(ctypes.c_float)]
    lib.hs_autotune_atoms.restype = i32
    lib.hs_gep_workspace_bytes.argtypes = [i32]
    lib.hs_gep_workspace_bytes.restype = sz
    lib.hs_gep_reduce.argtypes = [vp, vp, i32, vp, vp, vp, vp, sz, vp]
    lib.hs_gep_reduce.restype = i32
    lib.hs_gep_reduce_ex.argtypes = [vp, vp, i32, vp, vp, vp, vp, sz, vp, i32]
    lib.hs_gep_reduce_ex.restype = i32
    lib.hs_gep_check_schedule.argtypes = [i32, i32, i32, ctypes.c_char_p, sz]
    lib.hs_gep_check_schedule.restype = i32
    _lib = lib
    return lib


def _ptr(t) -> Optional[int]:
    """Device pointer of a tensor (None passes NULL)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if not t.is_cuda:
        raise ValueError("hs_build operands must be device tensors")
    if not t.is_contiguous():
        raise ValueError("hs_build operands must be contiguous")
    return t.data_ptr()


def _check_c128(*ts):
    import torch
    for t in ts:
        if t is not None and not isinstance(t, int) and t.dtype != torch.complex128:
            raise ValueError("hs_build operands must be complex128")


def _nl_array(nl_per_atom: Optional[Sequence[int]]):
    if nl_per_atom is None:
        return None, None
    arr = np.ascontiguousarray(np.asarray(nl_per_atom, dtype=np.int32))
    return arr, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def hs_status_string(status: int) -> str:
    return load_library().hs_status_string(int(status)).decode()


def _raise(status: int, check: bool) -> int:
    if status != HS_OK and check:
        raise HSError(status, hs_status_string(status))
    return status


def hs_workspace_bytes(N_A: int, nl_per_atom, N_L: int, N_G: int, mode: int = HS_FP64) -> int:
    arr, p = _nl_array(nl_per_atom)
    return int(load_library().hs_workspace_bytes(int(N_A), p, int(N_L), int(N_G), int(mode)))


def hs_build(A, B, T_AA, T_AB, T_BB, U, N_A, N_L, N_G, H, S, check: bool = True) -> int:
    """Synchronous build (default stream, library-allocated workspace)."""
    _check_c128(A, B, T_AA, T_AB, T_BB, U, H, S)
    rc = load_library().hs_build(_ptr(A), _ptr(B), _ptr(T_AA), _ptr(T_AB), _ptr(T_BB), _ptr(U),
                                 int(N_A), int(N_L), int(N_G), _ptr(H), _ptr(S))
    return _raise(rc, check)


def _tuning_ptr(tuning):
    if tuning is None:
        return None
    if not isinstance(tuning, hs_tuning):
        raise TypeError("tuning must be an hs_tuning")
    return ctypes.pointer(tuning)


def _options(workspace, info, stream, mode, nl_per_atom, phase_events, batch, tuning):
    """hs_options for the one-shot builds; returns (opt, objects to keep alive)."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    elif not isinstance(stream, int):
        stream = stream.cuda_stream
    if info is not None and info.dtype != torch.int32:
        raise ValueError("info must be int32")
    arr, p = _nl_array(nl_per_atom)
    opt = hs_options()
    opt.stream = stream
    opt.workspace = _ptr(workspace)
    opt.workspace_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
    opt.info = _ptr(info)
    opt.mode = int(mode)
    opt.nl_per_atom = p
    opt.batch = int(batch)
    tp = _tuning_ptr(tuning)
    if tp is not None:
        opt.tuning = tp
    ev = None
    if phase_events is not None:
        if len(phase_events) != HS_NUM_PHASE_EVENTS:
            raise ValueError("phase_events needs HS_NUM_PHASE_EVENTS handles")
        ev = (ctypes.c_void_p * HS_NUM_PHASE_EVENTS)(*phase_events)
        opt.phase_events = ctypes.cast(ev, ctypes.POINTER(ctypes.c_void_p))
    return opt, (arr, tp, ev)


def hs_build_ex(A, B, T_AA, T_AB, T_BB, U, N_A, N_L, N_G, H, S, *, workspace,
                info=None, stream=None, mode: int = HS_FP64, nl_per_atom=None,
                phase_events=None, batch: int = 0, tuning=None, check: bool = True) -> int:
    """Asynchronous build on `stream` (default: torch's current stream).

    workspace: uint8 device tensor of >= hs_workspace_bytes(...) bytes.
    info: int32 device tensor [N_A] or None.
    nl_per_atom: host sequence of N_A ints, or None for a uniform N_L.
    phase_events: None or a sequence of HS_NUM_PHASE_EVENTS raw hipEvent_t handles.
    batch: 1 runs the per-atom stage as the batched persistent launch.
    tuning: None or an hs_tuning (tile shape per N_L) for the batched launch.
    """
    _check_c128(A, B, T_AA, T_AB, T_BB, U, H, S)
    opt, keep = _options(workspace, info, stream, mode, nl_per_atom, phase_events, batch, tuning)
    rc = load_library().hs_build_ex(_ptr(A), _ptr(B), _ptr(T_AA), _ptr(T_AB), _ptr(T_BB), _ptr(U),
                                    int(N_A), int(N_L), int(N_G), _ptr(H), _ptr(S),
                                    ctypes.byref(opt))
    del keep
    return _raise(rc, check)


def hs_build_static(A, B, T_AA, T_AB, T_BB, U, N_A, N_L, N_G, H, S, *, info=None,
                    stream=None, mode: int = HS_FP64, nl_per_atom=None, phase_events=None,
                    batch: int = 0, tuning=None, check: bool = True) -> int:
    """hs_build_ex without a workspace: the library's fixed device array of
    HS_STATIC_SCRATCH_BYTES serves as one (no device allocation). Calls
    that overlap on one device race on that array."""
    _check_c128(A, B, T_AA, T_AB, T_BB, U, H, S)
    opt, keep = _options(None, info, stream, mode, nl_per_atom, phase_events, batch, tuning)
    rc = load_library().hs_build_static(_ptr(A), _ptr(B), _ptr(T_AA), _ptr(T_AB), _ptr(T_BB),
                                        _ptr(U), int(N_A), int(N_L), int(N_G), _ptr(H), _ptr(S),
                                        ctypes.byref(opt))
    del keep
    return _raise(rc, check)


# ---------------------------------------------------------------------------
# Resident context and serving loop


def _stream_handle(stream):
    import torch
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return stream if isinstance(stream, int) else stream.cuda_stream


def hs_ctx_create(T_AA, T_AB, T_BB, U, N_A, N_L, nl_per_atom=None, stream=None) -> int:
    """Create a resident context; returns its handle (synchronous)."""
    _check_c128(T_AA, T_AB, T_BB, U)
    arr, p = _nl_array(nl_per_atom)
    out = ctypes.c_void_p()
    rc = load_library().hs_ctx_create(_ptr(T_AA), _ptr(T_AB), _ptr(T_BB), _ptr(U), int(N_A),
                                      int(N_L), p, _stream_handle(stream), ctypes.byref(out))
    del arr
    _raise(rc, True)
    return out.value


def hs_ctx_rows(ctx) -> int:
    return int(load_library().hs_ctx_rows(ctx))


def hs_ctx_info(ctx, N_A) -> np.ndarray:
    info = np.zeros(int(N_A), np.int32)
    rc = load_library().hs_ctx_info(ctx, info.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    _raise(rc, True)
    return info


def hs_ctx_workspace_bytes(ctx, N_G, mode=HS_FP64) -> int:
    return int(load_library().hs_ctx_workspace_bytes(ctx, int(N_G), int(mode)))


def hs_ctx_footprint_bytes(ctx, N_G, mode=HS_FP64) -> int:
    return int(load_library().hs_ctx_footprint_bytes(ctx, int(N_G), int(mode)))


def hs_ctx_build(ctx, A, B, N_G, H, S, *, workspace, stream=None, mode=HS_FP64,
                 phase_events=None, batch: int = 0, tuning=None, check=True) -> int:
    _check_c128(A, B, H, S)
    opt = hs_options()
    opt.stream = _stream_handle(stream)
    opt.workspace = _ptr(workspace)
    opt.workspace_bytes = workspace.numel() * workspace.element_size()
    opt.mode = int(mode)
    opt.batch = int(batch)
    tp = _tuning_ptr(tuning)
    if tp is not None:
        opt.tuning = tp
    ev = None
    if phase_events is not None:
        ev = (ctypes.c_void_p * HS_NUM_PHASE_EVENTS)(*phase_events)
        opt.phase_events = ctypes.cast(ev, ctypes.POINTER(ctypes.c_void_p))
    rc = load_library().hs_ctx_build(ctx, _ptr(A), _ptr(B), int(N_G), _ptr(H), _ptr(S),
                                     ctypes.byref(opt))
    return _raise(rc, check)


def hs_ctx_destroy(ctx) -> None:
    load_library().hs_ctx_destroy(ctx)


def hs_server_create(ctx, n_slots, arena_bytes, mode=HS_FP64) -> int:
    out = ctypes.c_void_p()
    rc = load_library().hs_server_create(ctx, int(n_slots), int(arena_bytes), int(mode),
                                         ctypes.byref(out))
    _raise(rc, True)
    return out.value


def hs_server_submit(srv, rid, N_G, A_host_ptr, B_host_ptr, ld, check=True) -> int:
    req = hs_request(int(rid), int(N_G), A_host_ptr, B_host_ptr, int(ld))
    return _raise(load_library().hs_server_submit(srv, ctypes.byref(req)), check)


def hs_server_set_admission(srv, policy: int, max_bypass: int = 0, check=True) -> int:
    return _raise(load_library().hs_server_set_admission(srv, int(policy), int(max_bypass)), check)


def hs_server_progress(srv) -> int:
    n = load_library().hs_server_progress(srv)
    if n < 0:
        raise HSError(n, hs_status_string(n))
    return n


def hs_server_pop(srv):
    """The next completed result as a dict, or None."""
    r = hs_result()
    if load_library().hs_server_pop(srv, ctypes.byref(r)) != 1:
        return None
    return {"id": r.id, "N_G": r.N_G, "status": r.status, "H": r.H, "S": r.S,
            "t_submit": r.t_submit, "t_admit": r.t_admit, "t_done": r.t_done}


def hs_server_release(srv, rid) -> int:
    return _raise(load_library().hs_server_release(srv, int(rid)), True)


def hs_server_pending(srv) -> int:
    return int(load_library().hs_server_pending(srv))


def hs_server_used_bytes(srv) -> int:
    return int(load_library().hs_server_used_bytes(srv))


def hs_server_now(srv) -> float:
    return float(load_library().hs_server_now(srv))


def hs_server_destroy(srv) -> None:
    load_library().hs_server_destroy(srv)


# ---------------------------------------------------------------------------
# Batched per-atom stage: tile shapes and the autotuner


def hs_tile_config(cfg_id: int):
    """(BM, BN) of batched tile shape `cfg_id`, or None for an unknown id."""
    bm, bn = ctypes.c_int(), ctypes.c_int()
    rc = load_library().hs_tile_config(int(cfg_id), ctypes.byref(bm), ctypes.byref(bn))
    return None if rc != 0 else (bm.value, bn.value)


def hs_autotune_atoms(nl_values, N_G, reps=3, stream=None):
    """Fastest batched tile shape per N_L on the current device.

    Returns (hs_tuning, ms) with ms[i][c] the minimum time in milliseconds of
    shape c for nl_values[i]."""
    vals = np.ascontiguousarray(np.asarray(nl_values, dtype=np.int32).reshape(-1))
    out = hs_tuning()
    ms = np.zeros((max(1, vals.size), HS_NUM_TILE_CONFIGS), np.float32)
    rc = load_library().hs_autotune_atoms(
        vals.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if vals.size else None,
        int(vals.size), int(N_G), int(reps), _stream_handle(stream), ctypes.byref(out),
        ms.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
    _raise(rc, True)
    return out, ms[: vals.size]


# ---------------------------------------------------------------------------
# Generalized eigenproblem reduction


def hs_gep_workspace_bytes(N) -> int:
    return int(load_library().hs_gep_workspace_bytes(int(N)))


def hs_gep_check_schedule(N: int, mode: int = HS_FP64, drop_wait: int = 0):
    """(count, report): race check of the reduction's stream schedule for N
    (host only, nothing is launched). count is the number of pairs of
    launches on different streams that touch a common 128 x 128 cell, one
    writing, with no ordering between them; negative for invalid arguments.
    drop_wait leaves out one wait site (a test hook)."""
    buf = ctypes.create_string_buffer(4096)
    n = load_library().hs_gep_check_schedule(int(N), int(mode), int(drop_wait), buf, len(buf))
    return int(n), buf.value.decode()


def hs_gep_reduce(H, S, L, Ht, *, info=None, workspace=None, stream=None, check=True,
                  mode: int = HS_FP64) -> int:
    """S = L L^H, Ht = L^-1 H L^-H on `stream` (asynchronous). H, S, L, Ht:
    complex128 device tensors [N][N]; info: int32 device tensor [1] or None;
    workspace: uint8 device tensor (allocated here when None); mode: HS_FP64
    (hs_gep_reduce) or HS_FP64_3M (hs_gep_reduce_ex)."""
    import torch
    _check_c128(H, S, L, Ht)
    N = int(H.shape[0])
    for t in (H, S, L, Ht):
        if tuple(t.shape) != (N, N) or not t.is_contiguous() or t.device != H.device:
            raise ValueError("H, S, L, Ht must be contiguous [N][N] tensors on one device")
    if workspace is None:
        workspace = torch.empty(hs_gep_workspace_bytes(N), dtype=torch.uint8, device=H.device)
    if info is not None and info.dtype != torch.int32:
        raise ValueError("info must be int32")
    lib = load_library()
    args = (_ptr(H), _ptr(S), N, _ptr(L), _ptr(Ht), _ptr(info), _ptr(workspace),
            workspace.numel(), _stream_handle(stream))
    if mode == HS_FP64:
        rc = lib.hs_gep_reduce(*args)
    else:
        rc = lib.hs_gep_reduce_ex(*args, int(mode))
    return _raise(rc, check)
