"""MI355X-native generation of the FLAPW Hamiltonian and overlap matrices.

The build runs in libhsbuild.so (hand-written HIP for gfx950; C ABI in
include/hs_build.h). This package is its Python binding: marshalling of
torch device tensors and streams into the C entry points, which keep their
C names here.
"""

from ._binding import (  # noqa: F401
    HS_OK,
    HS_ERR_HIP,
    HS_ERR_WORKSPACE,
    HS_ERR_NOMEM,
    HS_ERR_UNSUPPORTED,
    HS_FP64,
    HS_SPLIT_F16,
    HS_SPLIT_I8,
    HS_FP64_3M,
    HS_SPLIT_BF16,
    HS_SPLIT_I8_CRT,
    HS_MAX_NL,
    HS_NUM_PHASE_EVENTS,
    HS_NUM_TILE_CONFIGS,
    HS_STATIC_SCRATCH_BYTES,
    HS_ADMIT_FIFO,
    HS_ADMIT_BYPASS,
    HSError,
    hs_tuning,
    LIB_PATH,
    load_library,
    hs_build,
    hs_build_ex,
    hs_build_static,
    hs_workspace_bytes,
    hs_status_string,
)
from ._binding import (  # noqa: F401,E402
    hs_ctx_create,
    hs_ctx_rows,
    hs_ctx_info,
    hs_ctx_workspace_bytes,
    hs_ctx_footprint_bytes,
    hs_ctx_build,
    hs_ctx_destroy,
    hs_server_create,
    hs_server_submit,
    hs_server_set_admission,
    hs_server_progress,
    hs_server_pop,
    hs_server_release,
    hs_server_pending,
    hs_server_used_bytes,
    hs_server_now,
    hs_server_destroy,
    hs_tile_config,
    hs_autotune_atoms,
    hs_gep_workspace_bytes,
    hs_gep_reduce,
    hs_gep_check_schedule,
)
from .runner import DeviceBuild  # noqa: F401,E402
