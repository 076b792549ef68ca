"""The comparison algorithms of Sec. 3 (OLA, OLS, WOLA, CF-TDC) on the GPU:
argument marshalling for the library's offline comparison entry points. Every
step runs in the library's kernels; this module checks shapes, allocates the
output and the workspace, and passes pointers."""
from __future__ import annotations

import ctypes

import torch

from ._lib import TvolapCmpShape, check_cmp, load

METHODS = {"ola": 0, "ols": 1, "wola": 2}
WINDOWS = {"rect": 0, "hann": 1, "sqrt_hann": 2}


def _check(x: torch.Tensor, taps: torch.Tensor):
    if x.dim() != 2 or x.dtype != torch.float32 or not x.is_cuda or not x.is_contiguous():
        raise ValueError("x must be a contiguous CUDA float32 tensor [C][N]")
    if taps.dim() != 3 or taps.dtype != torch.float32 or not taps.is_cuda or not taps.is_contiguous() \
            or taps.shape[0] != x.shape[0]:
        raise ValueError("taps must be a contiguous CUDA float32 tensor [C][K][n_taps]")


def _sched(schedule, rows: int, C: int):
    if schedule is None:
        return None
    if schedule.dtype != torch.int32 or not schedule.is_cuda or not schedule.is_contiguous() \
            or tuple(schedule.shape) != (rows, C):
        raise ValueError(f"schedule must be a contiguous CUDA int32 tensor [{rows}][{C}]")
    return ctypes.c_void_p(schedule.data_ptr())


def shape(method: str, block: int, x: torch.Tensor, taps: torch.Tensor, analysis: str = "sqrt_hann",
          synthesis: str = "sqrt_hann") -> TvolapCmpShape:
    s = TvolapCmpShape()
    s.method, s.block = METHODS[method], int(block)
    s.n_channels, s.n_slots, s.n_taps = x.shape[0], taps.shape[1], taps.shape[2]
    s.n_samples = x.shape[1]
    s.analysis, s.synthesis = WINDOWS[analysis], WINDOWS[synthesis]
    return s


def n_blocks(method: str, block: int, n_samples: int) -> int:
    """Schedule rows of a method's block grid."""
    hop = block // 2 if method == "wola" else block
    return -(-n_samples // hop) + (1 if method == "wola" else 0)


def block_convolution(method: str, x: torch.Tensor, taps: torch.Tensor, block: int,
                      schedule: torch.Tensor | None = None, analysis: str = "sqrt_hann",
                      synthesis: str = "sqrt_hann") -> torch.Tensor:
    """OLA / OLS / WOLA of x [C][N] with responses taps [C][K][n_taps] (n_taps
    <= block), the response of block b being schedule[b][c]."""
    _check(x, taps)
    s = shape(method, block, x, taps, analysis, synthesis)
    lib = load()
    rows = lib.tvolap_cmp_blocks(ctypes.byref(s))
    if rows < 0:
        check_cmp(-1)
    nbytes = lib.tvolap_cmp_workspace_bytes(ctypes.byref(s))
    ws = torch.empty(int(nbytes), dtype=torch.uint8, device=x.device)
    y = torch.empty_like(x)
    check_cmp(lib.tvolap_cmp_forward(ctypes.byref(s), ctypes.c_void_p(x.data_ptr()),
                                     ctypes.c_void_p(taps.data_ptr()), _sched(schedule, rows, x.shape[0]),
                                     ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
    return y


def cf_tdc(x: torch.Tensor, taps: torch.Tensor, hop: int, schedule: torch.Tensor | None = None) -> torch.Tensor:
    """Cross-faded direct convolution: the response of block l = b - 1 (hop L)
    is schedule[b][c], ceil(N/L) + 1 rows; Hann cross-fades of L samples."""
    _check(x, taps)
    C, N = x.shape
    y = torch.empty_like(x)
    check_cmp(load().tvolap_cftdc_forward(int(hop), C, taps.shape[1], N, taps.shape[2],
                                          ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(taps.data_ptr()),
                                          _sched(schedule, -(-N // hop) + 1, C), ctypes.c_void_p(y.data_ptr()),
                                          ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
    return y
