"""Non-uniform partitions: a short-partition head (hop L1, latency 2 L1) and a
long-partition tail (hop r L1) of every response, through the library's
tvolap_nup_* entry points. Argument marshalling only."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from ._lib import DTYPES, TvolapNupConfig, check_nup, load


class NupConvolver:
    """hop L1; tail_ratio r (tail hop r L1); head_partitions M1 >= max(1, r - 1);
    the other arguments as Convolver (one response length for all channels)."""

    def __init__(self, hop: int, tail_ratio: int, head_partitions: int, n_channels: int, max_taps: int,
                 n_inputs: int | None = None, input_of_channel=None, n_slots: int = 1, dtype: str = "f32",
                 stream: torch.cuda.Stream | None = None):
        self._lib = load()
        self._h = ctypes.c_void_p()
        self.hop = int(hop)
        self.tail_ratio = int(tail_ratio)
        self.head_partitions = int(head_partitions)
        self.n_channels = int(n_channels)
        self.n_inputs = int(n_inputs if n_inputs is not None else n_channels)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        cfg = TvolapNupConfig()
        b = cfg.base
        b.hop, b.n_channels, b.n_inputs, b.max_taps = self.hop, self.n_channels, self.n_inputs, int(max_taps)
        keep = None
        if input_of_channel is not None:
            keep = np.ascontiguousarray(np.asarray(input_of_channel, dtype=np.int32))
            if keep.shape != (self.n_channels,):
                raise ValueError(f"input_of_channel must have shape ({self.n_channels},)")
            b.input_of_channel = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        b.n_slots = int(n_slots)
        b.spectra_dtype = DTYPES[dtype]
        b.stream = ctypes.c_void_p(self.stream.cuda_stream)
        cfg.tail_ratio = self.tail_ratio
        cfg.head_partitions = self.head_partitions
        check_nup(self._lib.tvolap_nup_create(ctypes.byref(cfg), ctypes.byref(self._h)), None)
        del keep

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.tvolap_nup_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def period(self) -> int:
        return int(self._lib.tvolap_nup_period(self._h))

    def set_ir(self, channel: int, slot: int, taps):
        a = np.ascontiguousarray(np.asarray(taps, dtype=np.float32))
        check_nup(self._lib.tvolap_nup_set_ir(self._h, int(channel), int(slot), a.ctypes.data_as(ctypes.c_void_p),
                                              int(a.shape[0]), 0), self._h)

    def select_ir(self, slot_of_channel):
        a = np.ascontiguousarray(np.asarray(slot_of_channel, dtype=np.int32))
        check_nup(self._lib.tvolap_nup_select_ir(self._h, a.ctypes.data_as(ctypes.c_void_p)), self._h)

    def process(self, x: torch.Tensor, schedule: torch.Tensor | None = None, out: torch.Tensor | None = None,
                n_calls: int | None = None) -> torch.Tensor:
        """x [I][n L1] -> out [C][n L1]; schedule [n][C] int32 (device) or None."""
        L = self.hop
        n = x.shape[1] // L if n_calls is None else int(n_calls)
        if out is None:
            out = torch.empty((self.n_channels, n * L), device=x.device, dtype=torch.float32)
        fn = self._lib.tvolap_nup_process_block
        xp, xs, op, os_ = x.data_ptr(), int(x.stride(0)), out.data_ptr(), int(out.stride(0))
        sp = schedule.data_ptr() if schedule is not None else None
        row = 4 * self.n_channels
        for c in range(n):
            rc = fn(self._h, xp + 4 * L * c, xs, op + 4 * L * c, os_, (sp + row * c) if sp is not None else None)
            if rc != 0:
                check_nup(rc, self._h)
        return out

    def reset(self):
        check_nup(self._lib.tvolap_nup_reset(self._h), self._h)

    def autotune(self, iters: int = 10):
        check_nup(self._lib.tvolap_nup_autotune(self._h, int(iters)), self._h)

    def capture_begin(self):
        check_nup(self._lib.tvolap_nup_capture_begin(self._h), self._h)

    def capture_end(self):
        check_nup(self._lib.tvolap_nup_capture_end(self._h), self._h)

    def graph_launch(self):
        check_nup(self._lib.tvolap_nup_graph_launch(self._h), self._h)
