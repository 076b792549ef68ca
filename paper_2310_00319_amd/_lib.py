"""ctypes declarations for libtvolap.so (the C ABI in include/tvolap.h).

The library links against libamdhip64.so.7. PyTorch's ROCm build ships a HIP
runtime with the same soname; importing torch first makes the dynamic loader
bind the library to that one runtime, so device pointers and streams created by
torch are valid inside the library. ``load()`` checks that exactly one HIP
runtime is mapped into the process and fails loudly otherwise, and fails
loudly when the library has not been built. There is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (must be loaded before the library, see above)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtvolap.so")

TVOLAP_OK = 0
TVOLAP_EINVAL = -1
TVOLAP_ENOMEM = -2
TVOLAP_EDEVICE = -3
TVOLAP_ESTATE = -4

DTYPES = {"f32": 0, "bf16": 1, "f16": 2}

EXPORTED = (
    "tvolap_create", "tvolap_destroy", "tvolap_set_ir", "tvolap_set_irs", "tvolap_select_ir",
    "tvolap_process_block", "tvolap_process_blocks", "tvolap_reset", "tvolap_get_info", "tvolap_get_partitions",
    "tvolap_set_timing", "tvolap_get_timing", "tvolap_last_error", "tvolap_version",
    "tvolap_configure", "tvolap_autotune", "tvolap_configure_batch", "tvolap_autotune_batch",
    "tvolap_capture_begin", "tvolap_capture_end",
    "tvolap_graph_launch", "tvolap_offline_workspace_bytes", "tvolap_offline_ir_spectra",
    "tvolap_offline_forward", "tvolap_offline_backward", "tvolap_offline_last_error",
    "tvolap_offline_forward_noalloc", "tvolap_cmp_blocks", "tvolap_cmp_workspace_bytes", "tvolap_cmp_forward",
    "tvolap_cftdc_forward", "tvolap_cmp_last_error",
    "tvolap_nup_create", "tvolap_nup_destroy", "tvolap_nup_set_ir", "tvolap_nup_select_ir",
    "tvolap_nup_process_block", "tvolap_nup_reset", "tvolap_nup_autotune", "tvolap_nup_period",
    "tvolap_nup_capture_begin", "tvolap_nup_capture_end", "tvolap_nup_graph_launch", "tvolap_nup_last_error",
)


class TvolapOfflineShape(ctypes.Structure):
    _fields_ = [
        ("hop", ctypes.c_int32),
        ("n_channels", ctypes.c_int32),
        ("n_partitions", ctypes.c_int32),
        ("n_slots", ctypes.c_int32),
        ("n_samples", ctypes.c_int64),
    ]


class TvolapCmpShape(ctypes.Structure):
    _fields_ = [
        ("method", ctypes.c_int32),
        ("block", ctypes.c_int32),
        ("n_channels", ctypes.c_int32),
        ("n_slots", ctypes.c_int32),
        ("n_samples", ctypes.c_int64),
        ("n_taps", ctypes.c_int32),
        ("analysis", ctypes.c_int32),
        ("synthesis", ctypes.c_int32),
    ]


class TvolapConfig(ctypes.Structure):
    _fields_ = [
        ("hop", ctypes.c_int32),
        ("n_channels", ctypes.c_int32),
        ("n_inputs", ctypes.c_int32),
        ("input_of_channel", ctypes.POINTER(ctypes.c_int32)),
        ("max_taps", ctypes.c_int32),
        ("taps_of_channel", ctypes.POINTER(ctypes.c_int32)),
        ("n_slots", ctypes.c_int32),
        ("spectra_dtype", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
        ("max_batch", ctypes.c_int32),
        ("n_outputs", ctypes.c_int32),
        ("output_of_channel", ctypes.POINTER(ctypes.c_int32)),
    ]


class TvolapNupConfig(ctypes.Structure):
    _fields_ = [
        ("base", TvolapConfig),
        ("tail_ratio", ctypes.c_int32),
        ("head_partitions", ctypes.c_int32),
    ]


class TvolapInfo(ctypes.Structure):
    _fields_ = [
        ("hop", ctypes.c_int32), ("n_channels", ctypes.c_int32), ("n_inputs", ctypes.c_int32),
        ("n_slots", ctypes.c_int32), ("spectra_dtype", ctypes.c_int32),
        ("bins", ctypes.c_int32),
        ("sum_partitions", ctypes.c_int64),
        ("sum_input_partitions", ctypes.c_int64),
        ("mac_bytes_per_block", ctypes.c_int64),
        ("block_bytes", ctypes.c_int64),
        ("bank_bytes", ctypes.c_int64),
        ("delay_line_bytes", ctypes.c_int64),
        ("workspace_bytes", ctypes.c_int64),
        ("n_work_items", ctypes.c_int32),
        ("mac_chunk", ctypes.c_int32),
        ("mac_waves", ctypes.c_int32),
        ("mac_grid", ctypes.c_int32),
        ("fused", ctypes.c_int32),
        ("n_cu", ctypes.c_int32),
        ("batch_chunk", ctypes.c_int32),
        ("batch_vec", ctypes.c_int32),
        ("batch_waves", ctypes.c_int32),
        ("batch_tile_width", ctypes.c_int32),
        ("batch_work_items", ctypes.c_int32),
        ("batch_rows", ctypes.c_int32),
        ("batch_time_block", ctypes.c_int32),
        ("batch_group", ctypes.c_int32),
        ("batch_engine", ctypes.c_int32),
        ("n_outputs", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class TvolapError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"tvolap error {code}: {msg}")
        self.code = code


_lib = None


def _hip_runtimes_mapped() -> list:
    paths = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                parts = line.split()
                if len(parts) >= 6 and "libamdhip64.so" in parts[-1]:
                    paths.add(os.path.realpath(parts[-1]))
    except OSError:
        pass
    return sorted(paths)


def _declare(lib):
    c_int, c_i32, c_i64, c_vp = ctypes.c_int, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    lib.tvolap_create.argtypes = [ctypes.POINTER(TvolapConfig), ctypes.POINTER(c_vp)]
    lib.tvolap_destroy.argtypes = [c_vp]
    lib.tvolap_set_ir.argtypes = [c_vp, c_i32, c_i32, c_vp, c_i32, c_i32]
    lib.tvolap_set_irs.argtypes = [c_vp, c_i32, c_vp, c_i64]
    lib.tvolap_select_ir.argtypes = [c_vp, c_vp]
    lib.tvolap_process_block.argtypes = [c_vp, c_vp, c_i64, c_vp, c_i64, c_vp]
    lib.tvolap_process_blocks.argtypes = [c_vp, c_vp, c_i64, c_i32, c_vp, c_i64, c_vp, c_i64]
    lib.tvolap_reset.argtypes = [c_vp]
    lib.tvolap_get_info.argtypes = [c_vp, ctypes.POINTER(TvolapInfo)]
    lib.tvolap_get_partitions.argtypes = [c_vp, c_vp]
    lib.tvolap_set_timing.argtypes = [c_vp, c_i32]
    lib.tvolap_get_timing.argtypes = [c_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_double), ctypes.POINTER(c_i64)]
    lib.tvolap_last_error.argtypes = [c_vp]
    lib.tvolap_last_error.restype = ctypes.c_char_p
    lib.tvolap_configure.argtypes = [c_vp, c_i32, c_i32, c_i32, c_i32]
    lib.tvolap_autotune.argtypes = [c_vp, c_i32, ctypes.POINTER(ctypes.c_float)]
    lib.tvolap_configure_batch.argtypes = [c_vp, c_i32, c_i32, c_i32, c_i32, c_i32, c_i32]
    lib.tvolap_autotune_batch.argtypes = [c_vp, c_i32, ctypes.POINTER(ctypes.c_float)]
    lib.tvolap_capture_begin.argtypes = [c_vp]
    lib.tvolap_capture_end.argtypes = [c_vp]
    lib.tvolap_graph_launch.argtypes = [c_vp]
    lib.tvolap_version.argtypes = []
    lib.tvolap_version.restype = ctypes.c_char_p
    shp = ctypes.POINTER(TvolapOfflineShape)
    lib.tvolap_offline_workspace_bytes.argtypes = [shp]
    lib.tvolap_offline_workspace_bytes.restype = c_i64
    lib.tvolap_offline_ir_spectra.argtypes = [shp, c_vp, c_i32, c_vp, c_vp]
    lib.tvolap_offline_forward.argtypes = [shp, c_vp, c_vp, c_vp, c_vp, c_vp, c_i64, c_vp]
    lib.tvolap_offline_backward.argtypes = [shp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_i64, c_vp]
    lib.tvolap_offline_forward_noalloc.argtypes = [shp, c_vp, c_vp, c_vp, c_vp, c_vp]
    cshp = ctypes.POINTER(TvolapCmpShape)
    lib.tvolap_cmp_blocks.argtypes = [cshp]
    lib.tvolap_cmp_blocks.restype = c_i64
    lib.tvolap_cmp_workspace_bytes.argtypes = [cshp]
    lib.tvolap_cmp_workspace_bytes.restype = c_i64
    lib.tvolap_cmp_forward.argtypes = [cshp, c_vp, c_vp, c_vp, c_vp, c_vp, c_i64, c_vp]
    lib.tvolap_cftdc_forward.argtypes = [c_i32, c_i32, c_i32, c_i64, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp]
    lib.tvolap_nup_create.argtypes = [ctypes.POINTER(TvolapNupConfig), ctypes.POINTER(c_vp)]
    lib.tvolap_nup_destroy.argtypes = [c_vp]
    lib.tvolap_nup_set_ir.argtypes = [c_vp, c_i32, c_i32, c_vp, c_i32, c_i32]
    lib.tvolap_nup_select_ir.argtypes = [c_vp, c_vp]
    lib.tvolap_nup_process_block.argtypes = [c_vp, c_vp, c_i64, c_vp, c_i64, c_vp]
    lib.tvolap_nup_reset.argtypes = [c_vp]
    lib.tvolap_nup_autotune.argtypes = [c_vp, c_i32]
    lib.tvolap_nup_period.argtypes = [c_vp]
    lib.tvolap_nup_capture_begin.argtypes = [c_vp]
    lib.tvolap_nup_capture_end.argtypes = [c_vp]
    lib.tvolap_nup_graph_launch.argtypes = [c_vp]
    lib.tvolap_nup_last_error.argtypes = [c_vp]
    lib.tvolap_nup_last_error.restype = ctypes.c_char_p
    lib.tvolap_cmp_last_error.argtypes = []
    lib.tvolap_cmp_last_error.restype = ctypes.c_char_p
    lib.tvolap_offline_last_error.argtypes = []
    lib.tvolap_offline_last_error.restype = ctypes.c_char_p
    for name in EXPORTED:
        fn = getattr(lib, name)
        if name in ("tvolap_last_error", "tvolap_version", "tvolap_offline_last_error",
                    "tvolap_offline_workspace_bytes", "tvolap_cmp_blocks", "tvolap_cmp_workspace_bytes",
                    "tvolap_cmp_last_error", "tvolap_nup_last_error"):
            continue
        fn.restype = c_int


def load():
    """Load libtvolap.so (once). Raises if it is missing or if loading it
    would put a second HIP runtime into the process."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2310_00319_amd.build` "
            "(there is no CPU fallback)")
    before = _hip_runtimes_mapped()
    lib = ctypes.CDLL(LIB_PATH, mode=ctypes.RTLD_LOCAL)
    after = _hip_runtimes_mapped()
    if len(after) > 1:
        raise RuntimeError(f"two HIP runtimes are mapped into the process: {after} (was {before})")
    _declare(lib)
    _lib = lib
    return lib


def check_offline(code: int):
    if code != TVOLAP_OK:
        raise TvolapError(code, load().tvolap_offline_last_error().decode(errors="replace"))


def check(code: int, handle=None):
    if code != TVOLAP_OK:
        msg = load().tvolap_last_error(handle).decode(errors="replace")
        raise TvolapError(code, msg)


def check_cmp(code: int):
    if code != TVOLAP_OK:
        raise TvolapError(code, load().tvolap_cmp_last_error().decode(errors="replace"))


def check_nup(code: int, handle=None):
    if code != TVOLAP_OK:
        raise TvolapError(code, load().tvolap_nup_last_error(handle).decode(errors="replace"))
