"""Streaming TVOLAP convolver: a thin wrapper over the C ABI.

Argument marshalling only: every step of the method runs in the library's
gfx950 kernels. Tensors supply device pointers, torch supplies the stream.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from ._lib import DTYPES, TvolapConfig, TvolapInfo, check, load


def _i32_host(a, n: int, what: str):
    arr = np.ascontiguousarray(np.asarray(a, dtype=np.int32))
    if arr.shape != (n,):
        raise ValueError(f"{what} must have shape ({n},)")
    return arr


class Convolver:
    """Multichannel time-variant partitioned convolver on one GPU.

    hop               L (64, 128, 256 or 512); blocks/partitions 2L, transforms 4L.
    n_channels        C outputs.
    max_taps          longest IR.
    n_inputs          I input signals (default C, identity map).
    input_of_channel  [C] input index of each channel.
    taps_of_channel   [C] IR length of each channel (default max_taps).
    n_slots           K IR slots per channel.
    dtype             storage of IR spectra and delay line: "f32", "bf16", "f16".
    max_batch         largest number of blocks per batched call (process(..., batch=n)).
    n_outputs         0: one output row per channel; E > 0: a mixdown into E buses.
    output_of_channel [C] bus of each channel (with n_outputs > 0).
    """

    def __init__(self, hop: int, n_channels: int, max_taps: int, n_inputs: int | None = None,
                 input_of_channel=None, taps_of_channel=None, n_slots: int = 1, dtype: str = "f32",
                 device=None, stream: torch.cuda.Stream | None = None, max_batch: int = 16,
                 n_outputs: int = 0, output_of_channel=None):
        self._lib = load()
        self._h = ctypes.c_void_p()
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else torch.device(device).index or 0)
        self.hop = int(hop)
        self.n_channels = int(n_channels)
        self.n_inputs = int(n_inputs if n_inputs is not None else n_channels)
        self.n_slots = int(n_slots)
        self.dtype = dtype
        self.max_batch = int(max_batch)
        self.n_outputs = int(n_outputs) if n_outputs else self.n_channels
        if dtype not in DTYPES:
            raise ValueError(f"dtype must be one of {sorted(DTYPES)}")
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            self._keep = []
            cfg = TvolapConfig()
            cfg.hop = self.hop
            cfg.n_channels = self.n_channels
            cfg.n_inputs = self.n_inputs
            if input_of_channel is not None:
                a = _i32_host(input_of_channel, self.n_channels, "input_of_channel")
                self._keep.append(a)
                cfg.input_of_channel = a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
            cfg.max_taps = int(max_taps)
            if taps_of_channel is not None:
                t = _i32_host(taps_of_channel, self.n_channels, "taps_of_channel")
                self._keep.append(t)
                cfg.taps_of_channel = t.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
            cfg.n_slots = self.n_slots
            cfg.spectra_dtype = DTYPES[dtype]
            cfg.stream = ctypes.c_void_p(self.stream.cuda_stream)
            cfg.max_batch = self.max_batch
            if n_outputs:
                if output_of_channel is None:
                    raise ValueError("output_of_channel is required with n_outputs")
                o = _i32_host(output_of_channel, self.n_channels, "output_of_channel")
                self._keep.append(o)
                cfg.n_outputs = int(n_outputs)
                cfg.output_of_channel = o.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
            check(self._lib.tvolap_create(ctypes.byref(cfg), ctypes.byref(self._h)), None)
            self._keep = []

    # ------------------------------------------------------------ lifetime
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.tvolap_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------ IRs
    def set_ir(self, channel: int, slot: int, taps):
        """Load an IR (numpy array / CPU tensor, or a CUDA float32 tensor)."""
        if isinstance(taps, torch.Tensor) and taps.is_cuda:
            t = taps.detach()
            if t.dtype != torch.float32 or not t.is_contiguous():
                raise ValueError("device taps must be a contiguous float32 tensor")
            check(self._lib.tvolap_set_ir(self._h, int(channel), int(slot), ctypes.c_void_p(t.data_ptr()),
                                          int(t.numel()), 1), self._h)
            return
        a = np.ascontiguousarray(np.asarray(taps.cpu() if isinstance(taps, torch.Tensor) else taps,
                                            dtype=np.float32))
        check(self._lib.tvolap_set_ir(self._h, int(channel), int(slot), a.ctypes.data_as(ctypes.c_void_p),
                                      int(a.shape[0]), 0), self._h)

    def set_irs(self, slot: int, taps: torch.Tensor):
        """Load slot `slot` of every channel in one launch from a contiguous CUDA
        float32 tensor [n_channels][n] (row c: taps of channel c; taps beyond
        a channel's length are ignored, missing ones are zero)."""
        if not isinstance(taps, torch.Tensor) or not taps.is_cuda or taps.dtype != torch.float32 \
                or taps.dim() != 2 or taps.shape[0] != self.n_channels or not taps.is_contiguous():
            raise ValueError("taps must be a contiguous CUDA float32 tensor [n_channels][n]")
        check(self._lib.tvolap_set_irs(self._h, int(slot), ctypes.c_void_p(taps.data_ptr()), int(taps.shape[1])),
              self._h)

    def select_ir(self, slot_of_channel):
        a = _i32_host(slot_of_channel, self.n_channels, "slot_of_channel")
        check(self._lib.tvolap_select_ir(self._h, a.ctypes.data_as(ctypes.c_void_p)), self._h)

    # ------------------------------------------------------------ processing
    def _check_2d(self, t: torch.Tensor, rows: int, what: str):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32:
            raise ValueError(f"{what} must be a CUDA float32 tensor")
        if t.dim() != 2 or t.shape[0] != rows or t.shape[1] < self.hop or t.stride(1) != 1:
            raise ValueError(f"{what} must be [{rows}][>= {self.hop}] with unit stride along samples")

    def process_block(self, x: torch.Tensor, out: torch.Tensor | None = None,
                      slots: torch.Tensor | None = None) -> torch.Tensor:
        """One block: x [I][>=L] (first L samples used) -> out [E][>=L] (E = C without a mixdown)."""
        self._check_2d(x, self.n_inputs, "x")
        if out is None:
            out = torch.empty((self.n_outputs, self.hop), device=x.device, dtype=torch.float32)
        self._check_2d(out, self.n_outputs, "out")
        sp = None
        if slots is not None:
            if not slots.is_cuda or slots.dtype != torch.int32 or slots.numel() != self.n_channels \
                    or not slots.is_contiguous():
                raise ValueError("slots must be a contiguous CUDA int32 tensor of n_channels entries")
            sp = ctypes.c_void_p(slots.data_ptr())
        check(self._lib.tvolap_process_block(self._h, ctypes.c_void_p(x.data_ptr()), int(x.stride(0)),
                                             ctypes.c_void_p(out.data_ptr()), int(out.stride(0)), sp), self._h)
        return out

    def process(self, x: torch.Tensor, schedule: torch.Tensor | None = None,
                out: torch.Tensor | None = None, batch: int = 1) -> torch.Tensor:
        """Stream a resident signal: x [I][n*L] -> out [E][n*L]; schedule
        [n][C] int32 (device) gives the slots of every block. batch = 1: one
        process_block per L samples; batch > 1: process_blocks over up to
        `batch` blocks at a time (same results)."""
        L = self.hop
        self._check_2d(x, self.n_inputs, "x")
        n = x.shape[1] // L
        if out is None:
            out = torch.empty((self.n_outputs, n * L), device=x.device, dtype=torch.float32)
        self._check_2d(out, self.n_outputs, "out")
        if out.shape[1] < n * L:
            raise ValueError("out too short")
        if schedule is not None:
            if not schedule.is_cuda or schedule.dtype != torch.int32 or not schedule.is_contiguous() \
                    or schedule.dim() != 2 or schedule.shape[0] < n or schedule.shape[1] != self.n_channels:
                raise ValueError("schedule must be a contiguous CUDA int32 tensor [n_calls][n_channels]")
        h = self._h
        xp, xs = x.data_ptr(), int(x.stride(0))
        op, os_ = out.data_ptr(), int(out.stride(0))
        sp = schedule.data_ptr() if schedule is not None else None
        row = self.n_channels * 4
        if batch > 1:
            if batch > self.max_batch:
                raise ValueError(f"batch {batch} exceeds max_batch {self.max_batch}")
            fnb = self._lib.tvolap_process_blocks
            for c in range(0, n, batch):
                k = min(batch, n - c)
                rc = fnb(h, xp + 4 * L * c, xs, k, op + 4 * L * c, os_,
                         (sp + row * c) if sp is not None else None, self.n_channels)
                if rc != 0:
                    check(rc, h)
            return out
        fn = self._lib.tvolap_process_block
        for c in range(n):
            rc = fn(h, xp + 4 * L * c, xs, op + 4 * L * c, os_, (sp + row * c) if sp is not None else None)
            if rc != 0:
                check(rc, h)
        return out

    def configure(self, fused=1, chunk: int = 0, waves: int = 0, grid: int = 0):
        """fused: 1 = one launch per block, 2 = two launches, 0 (or False) = three."""
        check(self._lib.tvolap_configure(self._h, int(fused), int(chunk), int(waves), int(grid)), self._h)

    def autotune(self, iters: int = 20) -> float:
        best = ctypes.c_float()
        check(self._lib.tvolap_autotune(self._h, int(iters), ctypes.byref(best)), self._h)
        return best.value

    def configure_batch(self, chunk: int = 0, vec: int = 0, waves: int = 0, time_block: int = 0, group: int = 0,
                        engine: int = 0):
        """Schedule of batched calls (process with batch > 1); engine 1 = vector
        ALU, 2 = matrix cores (f32 spectra), 0 = 1."""
        check(self._lib.tvolap_configure_batch(self._h, int(chunk), int(vec), int(waves), int(time_block),
                                               int(group), int(engine)), self._h)

    def autotune_batch(self, iters: int = 5) -> float:
        best = ctypes.c_float()
        check(self._lib.tvolap_autotune_batch(self._h, int(iters), ctypes.byref(best)), self._h)
        return best.value

    def capture_begin(self):
        check(self._lib.tvolap_capture_begin(self._h), self._h)

    def capture_end(self):
        check(self._lib.tvolap_capture_end(self._h), self._h)

    def graph_launch(self):
        check(self._lib.tvolap_graph_launch(self._h), self._h)

    def reset(self):
        check(self._lib.tvolap_reset(self._h), self._h)

    # ------------------------------------------------------------ introspection
    def info(self) -> dict:
        inf = TvolapInfo()
        check(self._lib.tvolap_get_info(self._h, ctypes.byref(inf)), self._h)
        return inf.as_dict()

    def partitions(self) -> np.ndarray:
        a = np.zeros(self.n_channels, dtype=np.int32)
        check(self._lib.tvolap_get_partitions(self._h, a.ctypes.data_as(ctypes.c_void_p)), self._h)
        return a

    def set_timing(self, enable: bool):
        check(self._lib.tvolap_set_timing(self._h, 1 if enable else 0), self._h)

    def get_timing(self) -> dict:
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        n = ctypes.c_int64()
        check(self._lib.tvolap_get_timing(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                          ctypes.byref(n)), self._h)
        return {"ms_in": a.value, "ms_mac": b.value, "ms_out": c.value, "blocks": n.value}
