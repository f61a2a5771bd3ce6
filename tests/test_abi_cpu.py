"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point the header declares, sizes its workspace, and rejects bad
arguments with LAPACK-style codes before touching the device."""

import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import paper_1611_00606_amd as P
from paper_1611_00606_amd import _binding as Bd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))
           if f.endswith(".h")]


def _declared():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(hs_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_entry_points():
    names = _declared()
    for want in ("hs_build", "hs_build_ex", "hs_workspace_bytes", "hs_status_string",
                 "hs_gep_reduce", "hs_gep_reduce_ex", "hs_gep_workspace_bytes",
                 "hs_gep_check_schedule"):
        assert want in names


def test_library_exports_every_declared_symbol():
    lib = P.load_library()
    for name in _declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", P.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if l.strip()}
    for name in _declared():
        assert name in exported, name


def test_workspace_bytes():
    K, ng = 100 * 81, 8000
    ws = P.hs_workspace_bytes(100, None, 81, ng)
    assert ws >= 2 * 16 * K * ng            # Z and W stacks
    assert ws < 2 * 16 * K * ng + (64 << 20)
    nl = [16, 49, 81, 121]
    ws_mixed = P.hs_workspace_bytes(4, nl, 0, 6000)
    assert ws_mixed >= 2 * 16 * sum(nl) * 6000
    assert P.hs_workspace_bytes(0, None, 16, 100) == 0
    assert P.hs_workspace_bytes(1, None, 129, 100) == 0
    assert P.hs_workspace_bytes(2, [16, 0], 16, 100) == 0
    assert P.hs_workspace_bytes(1, None, 16, 0) == 0
    assert P.hs_workspace_bytes(1, None, 16, 10, 7) == 0


FAKE = 0x1000  # never dereferenced: argument checks return first


def _hs_build(*args):
    lib = P.load_library()
    return lib.hs_build(*args)


@pytest.mark.parametrize("pos", range(6))
def test_null_input_pointer(pos):
    ptrs = [FAKE] * 6
    ptrs[pos] = None
    assert _hs_build(*ptrs, 2, 4, 8, FAKE, FAKE) == -(pos + 1)


@pytest.mark.parametrize("n_a,n_l,n_g,code", [(0, 4, 8, -7), (-3, 4, 8, -7), (2, 0, 8, -8),
                                              (2, 129, 8, -8), (2, 4, 0, -9)])
def test_bad_sizes(n_a, n_l, n_g, code):
    assert _hs_build(*[FAKE] * 6, n_a, n_l, n_g, FAKE, FAKE) == code


def test_null_outputs():
    assert _hs_build(*[FAKE] * 6, 2, 4, 8, None, FAKE) == -10
    assert _hs_build(*[FAKE] * 6, 2, 4, 8, FAKE, None) == -11


def test_build_ex_option_checks():
    lib = P.load_library()
    assert lib.hs_build_ex(*[FAKE] * 6, 2, 4, 8, FAKE, FAKE, None) == -12
    for bad in (6, -1):
        opt = Bd.hs_options()
        opt.mode = bad
        assert lib.hs_build_ex(*[FAKE] * 6, 2, 4, 8, FAKE, FAKE, ctypes.byref(opt)) == -12
    nl = np.array([4, 200], np.int32)
    opt = Bd.hs_options()
    opt.nl_per_atom = nl.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    assert lib.hs_build_ex(*[FAKE] * 6, 2, 0, 8, FAKE, FAKE, ctypes.byref(opt)) == -8
    opt = Bd.hs_options()
    opt.workspace = FAKE + 8   # not 16-byte aligned
    opt.workspace_bytes = 1 << 40
    assert lib.hs_build_ex(*[FAKE] * 6, 2, 4, 8, FAKE, FAKE, ctypes.byref(opt)) == -12


def test_status_strings():
    assert P.hs_status_string(0) == "success"
    assert "workspace" in P.hs_status_string(2)
    assert "argument" in P.hs_status_string(-3)


def test_binding_rejects_host_tensors():
    import torch
    t = torch.zeros(4, dtype=torch.complex128)
    with pytest.raises(ValueError):
        P.hs_build(t, t, t, t, t, t, 1, 2, 2, t, t)


def test_context_and_server_argument_checks():
    lib = P.load_library()
    out = ctypes.c_void_p()
    assert lib.hs_ctx_create(None, FAKE, FAKE, FAKE, 2, 4, None, None, ctypes.byref(out)) == -1
    assert lib.hs_ctx_create(FAKE, FAKE, FAKE, None, 2, 4, None, None, ctypes.byref(out)) == -4
    assert lib.hs_ctx_create(FAKE, FAKE, FAKE, FAKE, 0, 4, None, None, ctypes.byref(out)) == -5
    assert lib.hs_ctx_create(FAKE, FAKE, FAKE, FAKE, 2, 200, None, None, ctypes.byref(out)) == -6
    nl = np.array([4, 0], np.int32)
    assert lib.hs_ctx_create(FAKE, FAKE, FAKE, FAKE, 2, 0,
                             nl.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), None,
                             ctypes.byref(out)) == -7
    assert lib.hs_ctx_create(FAKE, FAKE, FAKE, FAKE, 2, 4, None, None, None) == -9
    assert lib.hs_ctx_rows(None) == 0
    assert lib.hs_ctx_workspace_bytes(None, 10, 0) == 0
    assert lib.hs_ctx_footprint_bytes(None, 10, 0) == 0
    opt = Bd.hs_options()
    assert lib.hs_ctx_build(None, FAKE, FAKE, 8, FAKE, FAKE, ctypes.byref(opt)) == -1
    assert lib.hs_server_create(None, 2, 1 << 20, 0, ctypes.byref(out)) == -1
    assert lib.hs_server_create(FAKE, 0, 1 << 20, 0, ctypes.byref(out)) == -2
    assert lib.hs_server_create(FAKE, 2, 0, 0, ctypes.byref(out)) == -3
    assert lib.hs_server_create(FAKE, 2, 1 << 20, 9, ctypes.byref(out)) == -4
    assert lib.hs_server_submit(None, None) == -1
    assert lib.hs_server_progress(None) == -1
    assert lib.hs_server_pop(None, None) == -1
    assert lib.hs_server_release(None, 3) == -1
    assert lib.hs_server_pending(None) == 0
    assert lib.hs_server_used_bytes(None) == 0
    assert lib.hs_server_now(None) == 0.0


def test_split_mode_workspace():
    fp64 = P.hs_workspace_bytes(10, None, 49, 1000, P.HS_FP64)
    split = P.hs_workspace_bytes(10, None, 49, 1000, P.HS_SPLIT_F16)
    K = 490
    groups = (K + 15) // 16 * 4
    assert split >= fp64 + 6 * 4 * groups * 1000 * 16
    i8 = P.hs_workspace_bytes(10, None, 49, 1000, P.HS_SPLIT_I8)
    groups8 = (K + 31) // 32 * 4
    assert i8 >= fp64 + 6 * 5 * groups8 * 1000 * 16
    assert i8 < split   # 5 bytes per real value against 8
    # the 3M form changes only the arithmetic of the reductions
    assert P.hs_workspace_bytes(10, None, 49, 1000, P.HS_FP64_3M) == fp64
    # BF16 slices take the FP16 slices' room; an unknown mode none
    assert P.hs_workspace_bytes(10, None, 49, 1000, P.HS_SPLIT_BF16) == split
    # modular form: 11 residues of 2 bytes per complex element and operand
    # (contraction padded to 128 rows), plus the segments' residues of the
    # 128 x 128 lower-triangle tiles (5 segments x 11 moduli x 2 bytes)
    crt = P.hs_workspace_bytes(10, None, 49, 1000, P.HS_SPLIT_I8_CRT)
    groups_c = (K + 127) // 128 * 16
    nt = (1000 + 127) // 128
    crt_res = 5 * 11 * (nt * (nt + 1) // 2) * 128 * 128 * 2
    assert crt >= fp64 + 6 * 11 * groups_c * 1000 * 16 + crt_res
    assert crt < fp64 + 6 * 11 * groups_c * 1000 * 16 + crt_res + 6 * (1000 * 8 + 4096) + 8192
    assert P.hs_workspace_bytes(10, None, 49, 1000, 6) == 0
    assert P.hs_workspace_bytes(10, None, 49, 1000, -1) == 0


def test_tile_configs():
    shapes = [P.hs_tile_config(c) for c in range(P.HS_NUM_TILE_CONFIGS)]
    assert all(s is not None for s in shapes)
    assert len(set(shapes)) == len(shapes)
    for bm, bn in shapes:
        assert bm % 32 == 0 and bm <= 128 and bn in (128, 192, 256)
    # the built-in choice: the fewest rows that cover N_L, 192 columns for 96
    # rows, else 128
    from paper_1611_00606_amd.tuning import default_shape as ds
    for v in range(1, 129):
        bm, bn = shapes[ds(v)]
        assert bm >= v and bm - 32 < v and bn == (192 if bm == 96 else 128)
    assert P.hs_tile_config(-1) is None and P.hs_tile_config(P.HS_NUM_TILE_CONFIGS) is None
    from paper_1611_00606_amd.tuning import default_shape, tuning_from_table
    assert all(0 <= default_shape(v) < P.HS_NUM_TILE_CONFIGS for v in range(1, 129))
    t = tuning_from_table({16: 0, 121: 5})
    assert t.cfg[16] == 0 and t.cfg[121] == 5 and t.cfg[49] == default_shape(49)
    with pytest.raises(ValueError):
        tuning_from_table({16: P.HS_NUM_TILE_CONFIGS})
    with pytest.raises(ValueError):
        tuning_from_table({0: 1})


def test_batch_option_checks():
    lib = P.load_library()
    opt = Bd.hs_options()
    opt.batch = 2
    assert lib.hs_build_ex(*[FAKE] * 6, 2, 4, 8, FAKE, FAKE, ctypes.byref(opt)) == -12
    opt = Bd.hs_options()
    opt.batch = 1
    t = Bd.hs_tuning()
    for v in range(len(t.cfg)):
        t.cfg[v] = 1
    t.cfg[4] = 6   # the N_L in use maps to an unknown shape
    opt.tuning = ctypes.pointer(t)
    assert lib.hs_build_ex(*[FAKE] * 6, 2, 4, 8, FAKE, FAKE, ctypes.byref(opt)) == -12
    opt = Bd.hs_options()
    opt.batch = 1   # batched launch without an info array to report a timed-out wait
    assert lib.hs_build_ex(*[FAKE] * 6, 2, 4, 8, FAKE, FAKE, ctypes.byref(opt)) == -12
    assert lib.hs_build_static(*[FAKE] * 6, 2, 4, 8, FAKE, FAKE, ctypes.byref(opt)) == -12
    opt = Bd.hs_options()
    opt.batch = 2
    assert lib.hs_ctx_build(FAKE, FAKE, FAKE, 8, FAKE, FAKE, ctypes.byref(opt)) == -7


def test_autotune_argument_checks():
    lib = P.load_library()
    t = Bd.hs_tuning()
    vals = np.array([16, 49], np.int32)
    vp = vals.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    assert lib.hs_autotune_atoms(None, 2, 100, 1, None, ctypes.byref(t), None) == -1
    assert lib.hs_autotune_atoms(vp, 0, 100, 1, None, ctypes.byref(t), None) == -2
    bad = np.array([16, 129], np.int32)
    assert lib.hs_autotune_atoms(bad.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), 2, 100, 1,
                                 None, ctypes.byref(t), None) == -2
    assert lib.hs_autotune_atoms(vp, 2, 0, 1, None, ctypes.byref(t), None) == -3
    assert lib.hs_autotune_atoms(vp, 2, 100, 0, None, ctypes.byref(t), None) == -4
    assert lib.hs_autotune_atoms(vp, 2, 100, 1, None, None, None) == -6


def test_gep_argument_checks():
    lib = P.load_library()
    assert P.hs_gep_workspace_bytes(0) == 0
    assert P.hs_gep_workspace_bytes(100) >= 2 * 16 * 100 * 100
    args = [FAKE, FAKE, 8, FAKE, FAKE, None, FAKE, 1 << 20, None]
    for pos, bad in ((0, None), (1, None), (2, 0), (3, None), (4, None), (6, None),
                     (6, FAKE + 8)):
        a = list(args)
        a[pos] = bad
        assert lib.hs_gep_reduce(*a) == -(pos + 1)
        assert lib.hs_gep_reduce_ex(*a, P.HS_FP64_3M) == -(pos + 1)
    for bad_mode in (P.HS_SPLIT_F16, P.HS_SPLIT_I8, P.HS_SPLIT_BF16, P.HS_SPLIT_I8_CRT, -1):
        assert lib.hs_gep_reduce_ex(*args, bad_mode) == -10


def test_build_static_host_checks():
    """hs_build_static: option checks, and builds larger than its device
    array rejected on the host before any device call."""
    lib = P.load_library()
    assert lib.hs_build_static(*[FAKE] * 6, 2, 4, 8, FAKE, FAKE, None) == -12
    opt = Bd.hs_options()
    opt.workspace = FAKE
    opt.workspace_bytes = 1 << 30
    assert lib.hs_build_static(*[FAKE] * 6, 2, 4, 8, FAKE, FAKE, ctypes.byref(opt)) == -12
    opt = Bd.hs_options()
    assert lib.hs_build_static(None, *[FAKE] * 5, 2, 4, 8, FAKE, FAKE, ctypes.byref(opt)) == -1
    assert lib.hs_build_static(*[FAKE] * 6, 2, 4, 0, FAKE, FAKE, ctypes.byref(opt)) == -9
    opt.mode = 9
    assert lib.hs_build_static(*[FAKE] * 6, 2, 4, 8, FAKE, FAKE, ctypes.byref(opt)) == -12
    text = open(os.path.join(ROOT, "include", "hs_build.h")).read()
    m = re.search(r"#define HS_STATIC_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == P.HS_STATIC_SCRATCH_BYTES
    for mode, (n_a, n_l, n_g) in ((0, (100, 81, 8000)), (1, (10, 100, 2500))):
        need = P.hs_workspace_bytes(n_a, None, n_l, n_g, mode)
        assert need > P.HS_STATIC_SCRATCH_BYTES
        opt = Bd.hs_options()
        opt.mode = mode
        assert lib.hs_build_static(*[FAKE] * 6, n_a, n_l, n_g, FAKE, FAKE,
                                   ctypes.byref(opt)) == P.HS_ERR_WORKSPACE
        msg = P.hs_status_string(P.HS_ERR_WORKSPACE)
        assert str(need) in msg and str(P.HS_STATIC_SCRATCH_BYTES) in msg
    # the largest plain-FP64 builds it takes: the 32-atom N_L = 49 case at N_G = 2000
    assert P.hs_workspace_bytes(32, None, 49, 2000, 0) <= P.HS_STATIC_SCRATCH_BYTES
