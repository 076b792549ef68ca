"""Helpers shared by the GPU parity tests: run a synthetic workload through the
HIP library and through the FP64 oracle, and compare per channel."""
from __future__ import annotations

import sys

import numpy as np

import oracle as orc


def log(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_rms_per_channel(got: np.ndarray, ref: np.ndarray) -> np.ndarray:
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    num = np.sqrt(np.sum((got - ref) ** 2, axis=-1))
    den = np.sqrt(np.sum(ref ** 2, axis=-1))
    return num / np.maximum(den, 1e-300)


def max_abs_err_per_channel(got: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """Largest element error of each channel relative to the channel's largest
    reference magnitude: an element-wise bound that a short burst of wrong
    samples (a wrong block at a switch) cannot hide in the RMS of the stream."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    return np.max(np.abs(got - ref), axis=-1) / np.maximum(np.max(np.abs(ref), axis=-1), 1e-300)


# Element-wise bar for FP32 storage: every sample within 1e-4 of the channel's
# peak (the rel-RMS bar is 1e-5; single samples may sit a few times above the
# RMS error, never orders of magnitude).
ELEM_TOL_F32 = 1e-4


def oracle_streams(wl, channels=None, dtype: str = "f32") -> np.ndarray:
    """FP64 oracle stream outputs [len(channels)][n_calls*L] of a workload.
    dtype "f32" = exact oracle; "bf16"/"f16" = spectra rounded before the MAC."""
    chans = list(range(wl.n_channels)) if channels is None else list(channels)
    L = wl.hop
    x = wl.padded_input().astype(np.float64)
    out = np.zeros((len(chans), wl.n_calls * L))
    for j, c in enumerate(chans):
        H = orc.channel_spectra([t.astype(np.float64) for t in wl.taps[c]], L, int(wl.taps_of_channel[c]))
        xin = x[int(wl.input_of_channel[c])]
        if dtype == "f32":
            out[j] = orc.tvolap_stream(xin, H, wl.schedule[:, c], L, wl.n_calls)
        else:
            out[j] = orc.quantized_tvolap_streams(xin[None, :], [0], [H], wl.schedule[:, [c]], L,
                                                  wl.n_calls, dtype)[0]
    return out


def oracle_bus_streams(wl, buses, dtype: str = "f32") -> np.ndarray:
    """FP64 oracle of a mixdown: bus e is the sum of the oracle streams of the
    channels c with buses[c] == e. Returns [n_buses][n_calls*L]."""
    buses = np.asarray(buses)
    per = oracle_streams(wl, None, dtype)
    out = np.zeros((int(buses.max()) + 1, per.shape[1]))
    for c in range(wl.n_channels):
        out[int(buses[c])] += per[c]
    return out


MODES = {
    "fused": dict(fused=1),
    "plain": dict(fused=0),
    "two_kernel": dict(fused=2),
    "persistent": dict(fused=1, grid=7),
    "tiny_chunks": dict(fused=1, chunk=2, waves=8),
    "two_kernel_tiny": dict(fused=2, chunk=3, waves=8, grid=5),
    "plain_tiny_chunks": dict(fused=0, chunk=3, waves=8),
}


def make_convolver(wl, dtype: str = "f32", stream=None, mode: str = "fused", max_batch: int = 16, buses=None):
    """buses: None (one output per channel) or [C] bus of each channel (mixdown)."""
    from paper_2310_00319_amd import Convolver

    mix = {} if buses is None else dict(n_outputs=int(np.max(buses)) + 1, output_of_channel=buses)
    conv = Convolver(hop=wl.hop, n_channels=wl.n_channels, max_taps=wl.max_taps(),
                     n_inputs=wl.n_inputs, input_of_channel=wl.input_of_channel,
                     taps_of_channel=wl.taps_of_channel, n_slots=wl.n_slots, dtype=dtype, stream=stream,
                     max_batch=max_batch, **mix)
    if mode != "fused":
        conv.configure(**MODES[mode])
    for c in range(wl.n_channels):
        for s in range(wl.n_slots):
            conv.set_ir(c, s, wl.taps[c][s])
    return conv


def gpu_streams(wl, dtype: str = "f32", conv=None, mode: str = "fused", batch: int = 1, buses=None):
    """Whole workload through the library with a device-resident schedule.
    Returns the [C][n_calls*L] output (one row per bus with `buses`) as float64 numpy."""
    import torch

    own = conv is None
    if own:
        conv = make_convolver(wl, dtype, mode=mode, buses=buses)
    x = torch.from_numpy(wl.padded_input()).cuda()
    sched = torch.from_numpy(np.ascontiguousarray(wl.schedule, dtype=np.int32)).cuda()
    out = conv.process(x, sched, batch=batch)
    torch.cuda.synchronize()
    res = out.cpu().numpy().astype(np.float64)
    if own:
        conv.close()
    return res


def gpu_streams_graph(wl, dtype: str = "f32", batch: int = 64, channels=None, tune: bool = True, buses=None,
                      schedule: dict | None = None):
    """The benchmark's launch configuration: calls of `batch` blocks (max_batch
    = batch, batched schedule autotuned), captured once as a HIP graph on a
    side stream and replayed. Returns [len(channels)][n_calls*L] float64
    (`channels` index the buses with a mixdown). `schedule`: configure_batch
    arguments instead of the autotuner."""
    import torch

    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        conv = make_convolver(wl, dtype, stream=stream, max_batch=batch, buses=buses)
        if schedule is not None:
            conv.configure_batch(**schedule)
        elif tune:
            conv.autotune_batch(iters=2)
        x = torch.from_numpy(wl.padded_input()).cuda()
        sched = torch.from_numpy(np.ascontiguousarray(wl.schedule, dtype=np.int32)).cuda()
        out = torch.zeros((conv.n_outputs, wl.n_calls * wl.hop), device="cuda")
        stream.synchronize()
        conv.capture_begin()
        conv.process(x, sched, out, batch=batch)
        conv.capture_end()
        conv.reset()
        conv.graph_launch()
        stream.synchronize()
        chans = list(range(conv.n_outputs)) if channels is None else list(channels)
        res = out[chans].cpu().numpy().astype(np.float64)
        conv.close()
    return res

