"""Differentiable, offline TVOLAP (whole signals resident on the GPU).

``tvolap(x, H, hop, schedule)`` is a ``torch.autograd.Function`` over the
library's offline forward and adjoint kernels; the binding only checks shapes,
allocates the outputs and the workspace, and passes pointers. Gradients are
with respect to the input and to the partition spectra H (PyTorch's complex
convention: dLoss/dRe + i dLoss/dIm). The input spectra are recomputed from x
in the backward pass, not stored.
"""
from __future__ import annotations

import ctypes

import torch

from ._lib import TvolapOfflineShape, check_offline, load


def _shape(x: torch.Tensor, H: torch.Tensor, hop: int) -> TvolapOfflineShape:
    if x.dim() != 2 or x.dtype != torch.float32 or not x.is_cuda or not x.is_contiguous():
        raise ValueError("x must be a contiguous CUDA float32 tensor [C][N]")
    C, N = x.shape
    if H.dim() != 4 or H.dtype != torch.complex64 or not H.is_cuda or not H.is_contiguous():
        raise ValueError("H must be a contiguous CUDA complex64 tensor [C][K][M][2L+1]")
    if H.shape[0] != C or H.shape[3] != 2 * hop + 1:
        raise ValueError(f"H must be [{C}][K][M][{2 * hop + 1}]")
    s = TvolapOfflineShape()
    s.hop, s.n_channels, s.n_slots, s.n_partitions, s.n_samples = hop, C, H.shape[1], H.shape[2], N
    return s


def n_blocks(n_samples: int, hop: int) -> int:
    """Blocks of the offline form: ceil(N / L) + 1 (the first covers [-L, L))."""
    return -(-n_samples // hop) + 1


def _sched_ptr(schedule, shape):
    if schedule is None:
        return None
    nb = n_blocks(shape.n_samples, shape.hop)
    if schedule.dtype != torch.int32 or not schedule.is_cuda or not schedule.is_contiguous() \
            or tuple(schedule.shape) != (nb, shape.n_channels):
        raise ValueError(f"schedule must be a contiguous CUDA int32 tensor [{nb}][{shape.n_channels}]")
    return ctypes.c_void_p(schedule.data_ptr())


def _workspace(shape, device):
    nbytes = load().tvolap_offline_workspace_bytes(ctypes.byref(shape))
    if nbytes < 0:
        check_offline(-1)
    return torch.empty(int(nbytes), dtype=torch.uint8, device=device)


def ir_spectra(taps: torch.Tensor, hop: int, n_partitions: int | None = None) -> torch.Tensor:
    """Partition spectra H [C][K][M][2L+1] (complex64) of taps [C][K][n_taps]."""
    if taps.dim() != 3 or taps.dtype != torch.float32 or not taps.is_cuda or not taps.is_contiguous():
        raise ValueError("taps must be a contiguous CUDA float32 tensor [C][K][n_taps]")
    C, K, n = taps.shape
    M = n_partitions if n_partitions is not None else -(-n // (2 * hop))
    s = TvolapOfflineShape()
    s.hop, s.n_channels, s.n_slots, s.n_partitions, s.n_samples = hop, C, K, M, 1
    H = torch.empty((C, K, M, 2 * hop + 1), dtype=torch.complex64, device=taps.device)
    check_offline(load().tvolap_offline_ir_spectra(ctypes.byref(s), ctypes.c_void_p(taps.data_ptr()), int(n),
                                                   ctypes.c_void_p(H.data_ptr()),
                                                   ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
    return H


class _Tvolap(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, H, schedule, hop):
        shape = _shape(x, H, hop)
        y = torch.empty_like(x)
        ws = _workspace(shape, x.device)
        stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        check_offline(load().tvolap_offline_forward(
            ctypes.byref(shape), ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(H.data_ptr()),
            _sched_ptr(schedule, shape), ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
            ws.numel(), stream))
        ctx.save_for_backward(x, H, schedule if schedule is not None else torch.empty(0, device=x.device))
        ctx.has_sched = schedule is not None
        ctx.hop = hop
        return y

    @staticmethod
    def backward(ctx, gy):
        x, H, schedule = ctx.saved_tensors
        schedule = schedule if ctx.has_sched else None
        shape = _shape(x, H, ctx.hop)
        gy = gy.contiguous()
        dx = torch.empty_like(x) if ctx.needs_input_grad[0] else None
        dH = torch.empty_like(H) if ctx.needs_input_grad[1] else None
        ws = _workspace(shape, x.device)
        stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        check_offline(load().tvolap_offline_backward(
            ctypes.byref(shape), ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(H.data_ptr()),
            _sched_ptr(schedule, shape), ctypes.c_void_p(gy.data_ptr()),
            ctypes.c_void_p(dx.data_ptr()) if dx is not None else None,
            ctypes.c_void_p(dH.data_ptr()) if dH is not None else None,
            ctypes.c_void_p(ws.data_ptr()), ws.numel(), stream))
        return dx, dH, None, None


def tvolap(x: torch.Tensor, H: torch.Tensor, hop: int, schedule: torch.Tensor | None = None) -> torch.Tensor:
    """y [C][N] = time-variant partitioned convolution of x [C][N] with the
    partition spectra H [C][K][M][2L+1] under schedule [nblk][C] (set per
    block, nblk = ceil(N/L) + 1; None = set 0)."""
    return _Tvolap.apply(x, H, schedule, int(hop))


def forward_noalloc(x: torch.Tensor, H: torch.Tensor, hop: int, schedule: torch.Tensor | None = None,
                    out: torch.Tensor | None = None) -> torch.Tensor:
    """The forward of ``tvolap`` through the library's allocation-free entry
    point (its working memory is a static per-GPU array; no workspace). With
    ``out`` given the call allocates nothing at all, so it may run under HIP
    graph capture. Not differentiable."""
    shape = _shape(x, H, hop)
    y = torch.empty_like(x) if out is None else out
    if y.shape != x.shape or y.dtype != torch.float32 or not y.is_cuda or not y.is_contiguous():
        raise ValueError("out must be a contiguous CUDA float32 tensor shaped like x")
    check_offline(load().tvolap_offline_forward_noalloc(
        ctypes.byref(shape), ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(H.data_ptr()),
        _sched_ptr(schedule, shape), ctypes.c_void_p(y.data_ptr()),
        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
    return y
