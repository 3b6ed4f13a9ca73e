"""ctypes binding of libsdtw.so (the C ABI in include/sdtw.h).

Argument marshalling only: every step of the sDTW path runs in the HIP
kernels of the library.  Importing this module fails loudly when the library
has not been built; there is no fallback.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# SDTW_LIBRARY may name another build of the same library (for example one
# whose host code is built with sanitizers)
LIB_PATH = os.environ.get("SDTW_LIBRARY") or os.path.join(_HERE, "libsdtw.so")

SDTW_COST_SQUARED = 0
SDTW_COST_ABSOLUTE = 1
SDTW_OK = 0
SDTW_ERR_INVALID_ARG = -1
SDTW_ERR_WORKSPACE = -2
SDTW_ERR_UNSUPPORTED = -3
SDTW_ERR_HIP = -4
SDTW_F_CHECKPOINT = 1
SDTW_F_PERSISTENT = 2
SDTW_F_WAVES_SHIFT = 8


def SDTW_F_WAVES_PER_SIMD(n: int) -> int:
    """Flags bits asking the persistent grid for n resident wavefronts per SIMD."""
    return int(n) << SDTW_F_WAVES_SHIFT


SDTW_MAX_REF_LEN = 1 << 30
SDTW_NOALLOC_SCRATCH_BYTES = 16 << 20
SDTW_ROW_CKPT_EVERY = 256

_c_i32p = ctypes.POINTER(ctypes.c_int32)
_vp = ctypes.c_void_p


class SdtwError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} (status {status})")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"libsdtw.so is not built ({LIB_PATH}); run __graft_entry__.build() "
            "or python paper_2403_06931_amd/csrc/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    lib.sdtw_status_string.argtypes = [ctypes.c_int]
    lib.sdtw_status_string.restype = ctypes.c_char_p
    lib.sdtw_variant_count.argtypes = []
    lib.sdtw_variant_count.restype = ctypes.c_int32
    lib.sdtw_variant_info.argtypes = [ctypes.c_int32, _c_i32p, _c_i32p, _c_i32p, _c_i32p,
                                      _c_i32p]
    lib.sdtw_variant_info.restype = ctypes.c_int
    lib.sdtw_default_variant.argtypes = [_vp, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32]
    lib.sdtw_default_variant.restype = ctypes.c_int32
    lib.sdtw_forward_workspace_bytes.argtypes = [_vp, ctypes.c_int32, ctypes.c_int64,
                                                 ctypes.c_int32, ctypes.c_int32]
    lib.sdtw_forward_workspace_bytes.restype = ctypes.c_size_t
    lib.sdtw_workspace_bytes.argtypes = [_vp, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
                                         ctypes.c_int32]
    lib.sdtw_workspace_bytes.restype = ctypes.c_size_t
    lib.sdtw_checkpoint_floats.argtypes = [_vp, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32]
    lib.sdtw_checkpoint_floats.restype = ctypes.c_size_t
    lib.sdtw_forward.argtypes = [_vp, _vp, _vp, ctypes.c_int32, _vp, ctypes.c_int64,
                                 ctypes.c_int32, _vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32,
                                 ctypes.c_int32, _vp, ctypes.c_size_t, _vp]
    lib.sdtw_forward.restype = ctypes.c_int
    lib.sdtw_forward_noalloc.argtypes = [_vp, _vp, _vp, ctypes.c_int32, _vp, ctypes.c_int64,
                                         ctypes.c_int32, _vp, _vp, _vp, ctypes.c_int32,
                                         ctypes.c_int32, ctypes.c_int32, _vp]
    lib.sdtw_forward_noalloc.restype = ctypes.c_int
    lib.sdtw_forward_pruned.argtypes = [_vp, _vp, _vp, ctypes.c_int32, _vp, ctypes.c_int64,
                                        ctypes.c_float, _vp, _vp, ctypes.c_int32, ctypes.c_int32,
                                        _vp, ctypes.c_size_t, _vp]
    lib.sdtw_forward_pruned.restype = ctypes.c_int
    lib.sdtw_forward_u8_workspace_bytes.argtypes = [_vp, ctypes.c_int32, ctypes.c_int64]
    lib.sdtw_forward_u8_workspace_bytes.restype = ctypes.c_size_t
    lib.sdtw_forward_u8.argtypes = [_vp, _vp, _vp, ctypes.c_int32, _vp, ctypes.c_int64, _vp,
                                    _vp, _vp, ctypes.c_int32, _vp, ctypes.c_size_t, _vp]
    lib.sdtw_forward_u8.restype = ctypes.c_int
    lib.sdtw_backward_workspace_bytes.argtypes = [_vp, ctypes.c_int32, ctypes.c_int64,
                                                  ctypes.c_int32]
    lib.sdtw_backward_workspace_bytes.restype = ctypes.c_size_t
    lib.sdtw_backward.argtypes = [_vp, _vp, _vp, ctypes.c_int32, _vp, ctypes.c_int64,
                                  ctypes.c_int32, _vp, _vp, _vp, _vp, ctypes.c_int32, _vp, _vp,
                                  _vp, ctypes.c_size_t, _vp]
    lib.sdtw_backward.restype = ctypes.c_int
    lib.sdtw_forward_f16_workspace_bytes.argtypes = [_vp, ctypes.c_int32, ctypes.c_int64]
    lib.sdtw_forward_f16_workspace_bytes.restype = ctypes.c_size_t
    lib.sdtw_forward_f16.argtypes = [_vp, _vp, _vp, ctypes.c_int32, _vp, ctypes.c_int64,
                                     ctypes.c_int32, _vp, _vp, ctypes.c_int32, _vp,
                                     ctypes.c_size_t, _vp]
    lib.sdtw_forward_f16.restype = ctypes.c_int
    lib.sdtw_align_workspace_bytes.argtypes = [_vp, ctypes.c_int32, ctypes.c_int64,
                                               ctypes.c_int32]
    lib.sdtw_align_workspace_bytes.restype = ctypes.c_size_t
    lib.sdtw_align.argtypes = [_vp, _vp, _vp, ctypes.c_int32, _vp, ctypes.c_int64,
                               ctypes.c_int32, _vp, _vp, _vp, ctypes.c_int32, _vp, _vp, _vp,
                               _vp, ctypes.c_size_t, _vp]
    lib.sdtw_align.restype = ctypes.c_int
    lib.sdtw_znorm_workspace_bytes.argtypes = [_vp, ctypes.c_int32]
    lib.sdtw_znorm_workspace_bytes.restype = ctypes.c_size_t
    lib.sdtw_znorm.argtypes = [_vp, _vp, _vp, ctypes.c_int32, _vp, _vp, ctypes.c_size_t, _vp]
    lib.sdtw_znorm.restype = ctypes.c_int
    return lib


lib = _load()


def status_string(status: int) -> str:
    return lib.sdtw_status_string(int(status)).decode()


def check(status: int, where: str) -> None:
    if status != SDTW_OK:
        raise SdtwError(status, where)
