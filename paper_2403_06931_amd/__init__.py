"""MI355X-native subsequence dynamic time warping (sDTW).

The hot path -- the DP fill of a batch of queries against one long reference,
its last-row reduction to (cost, end position), the batched persistent form,
the checkpointed walk-back gradient and the batch z-normaliser that prepares
the inputs -- runs in hand-written HIP kernels for gfx950 behind the C ABI in
include/sdtw.h (libsdtw.so).  This package is the thin Python binding over
that library.
"""
from .api import (SDTW_COST_ABSOLUTE, SDTW_COST_SQUARED, SDTW_F_CHECKPOINT,  # noqa: F401
                  SDTW_F_PERSISTENT, SDTW_F_WAVES_PER_SIMD, SDTW_ROW_CKPT_EVERY, SdtwError, sdtw_align, sdtw_align_workspace_bytes,
                  sdtw_backward, sdtw_backward_workspace_bytes,
                  sdtw_checkpoint_floats, sdtw_default_variant, sdtw_forward,
                  sdtw_forward_f16, sdtw_forward_f16_workspace_bytes, sdtw_forward_noalloc,
                  sdtw_forward_pruned,
                  sdtw_forward_u8, sdtw_forward_u8_workspace_bytes,
                  sdtw_forward_workspace_bytes, sdtw_variant_count, sdtw_variant_info,
                  sdtw_workspace_bytes, sdtw_znorm, sdtw_znorm_workspace_bytes, workspace)
from .graph import ForwardGraph  # noqa: F401,E402
from .autograd import SDTWFunction, sdtw  # noqa: F401,E402
from . import autotune  # noqa: F401,E402
