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
HS_MAX_NL = 128
HS_NUM_PHASE_EVENTS = 5


class HSError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"hs_build status {status}: {message}")
        self.status = status


class hs_options(ctypes.Structure):
    _fields_ = [
        ("stream", ctypes.c_void_p),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
        ("info", ctypes.c_void_p),
        ("mode", ctypes.c_int),
        ("nl_per_atom", ctypes.POINTER(ctypes.c_int32)),
        ("phase_events", ctypes.POINTER(ctypes.c_void_p)),
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
    lib.hs_workspace_bytes.argtypes = [i32, ctypes.POINTER(ctypes.c_int32), i32, i32, i32]
    lib.hs_workspace_bytes.restype = ctypes.c_size_t
    lib.hs_status_string.argtypes = [i32]
    lib.hs_status_string.restype = ctypes.c_char_p
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


def hs_build_ex(A, B, T_AA, T_AB, T_BB, U, N_A, N_L, N_G, H, S, *, workspace,
                info=None, stream=None, mode: int = HS_FP64, nl_per_atom=None,
                phase_events=None, check: bool = True) -> int:
    """Asynchronous build on `stream` (default: torch's current stream).

    workspace: uint8 device tensor of >= hs_workspace_bytes(...) bytes.
    info: int32 device tensor [N_A] or None.
    nl_per_atom: host sequence of N_A ints, or None for a uniform N_L.
    phase_events: None or a sequence of HS_NUM_PHASE_EVENTS raw hipEvent_t handles.
    """
    import torch
    _check_c128(A, B, T_AA, T_AB, T_BB, U, H, S)
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
    ev = None
    if phase_events is not None:
        if len(phase_events) != HS_NUM_PHASE_EVENTS:
            raise ValueError("phase_events needs HS_NUM_PHASE_EVENTS handles")
        ev = (ctypes.c_void_p * HS_NUM_PHASE_EVENTS)(*phase_events)
        opt.phase_events = ctypes.cast(ev, ctypes.POINTER(ctypes.c_void_p))
    rc = load_library().hs_build_ex(_ptr(A), _ptr(B), _ptr(T_AA), _ptr(T_AB), _ptr(T_BB), _ptr(U),
                                    int(N_A), int(N_L), int(N_G), _ptr(H), _ptr(S),
                                    ctypes.byref(opt))
    del arr
    return _raise(rc, check)
