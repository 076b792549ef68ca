"""Benchmark: TVOLAP throughput on one MI355X.

A step is one pass of the whole hot path over the workload's signal: every
block of the 5 s (binaural) input runs through window + transform-in, the
spectral MAC against the partition spectra of the slot selected for that block,
transform-out and overlap-add, for all channels, with the IR slot of every
channel switching every block. Inputs, IR bank, schedule and outputs are
resident in HBM before timing starts.

By default blocks go through the library 64 at a time (tvolap_process_blocks:
the same output as one call per block up to the order of additions), and the
calls of a step are replayed from one captured HIP graph; the same run also
times strict streaming with one call per block (realtime_one_block_per_call).

Prints one JSON line with the roofline of the dominant kernel (its average
launch duration from HIP events that the library records around it on its
stream), an accuracy check of the same configuration against the FP64 oracle,
and a CPU baseline (the oracle on a bounded sample of the same workload).
"""
from __future__ import annotations

import argparse
import json
import os
import resource
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
# FP32 fused multiply-add issue rate without packed-FP32 instructions (which
# this build does not emit): 256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz.
# With packed FP32 the chip's published vector figure is twice this, 157.3.
VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# 16-bit spectra are multiplied with two-element dot products (4 flop per lane
# per instruction) accumulating in FP32: twice the FMA rate.
DOT2_PEAK_TFLOPS = 2 * VALU_PEAK_TFLOPS
# Dense matrix-core (MFMA) peaks of the chip: FP32, and bf16/f16 inputs.
MFMA_F32_PEAK_TFLOPS = 157.3
MFMA_16_PEAK_TFLOPS = 2500.0

WORKLOADS = {
    "binaural": dict(desc="64 sources x 2 ears = 128 channels, L=256 (blocks 512, FFT 1024), 96000-tap IRs "
                          "(188 partitions), 4 recurring IR sets per channel, block l using set l mod 4 (a switch "
                          "at every block; the same sets recur within a call), 5 s at 48 kHz; the "
                          "fresh_response_sets legs give a new set at every block",
                     fn="binaural", dtype="f32"),
    "binaural_bf16": dict(desc="as binaural, IR spectra and delay line stored bf16", fn="binaural", dtype="bf16"),
    "binaural_f16": dict(desc="as binaural, IR spectra and delay line stored f16", fn="binaural", dtype="f16"),
    "binaural_mix": dict(desc="as binaural, the 128 channels mixed down into the two ear outputs (channel c to ear "
                              "c mod 2)", fn="binaural", dtype="f32", buses="ear"),
    "binaural_r2": dict(desc="as binaural with hop 128 (blocks 256, FFT 512): the 2-s IRs fall into 375 partitions",
                        fn="binaural", kw=dict(hop=128), dtype="f32"),
    "uneven": dict(desc="512 channels, L=128, IR lengths log-uniform 4800..192000 taps, 2 slots, "
                        "each channel toggles with p=0.1 per block, 2 s at 48 kHz", fn="uneven", dtype="f32"),
    "plain": dict(desc="1 channel, L=128, 4096-tap IRs, 2 slots switched every 50 blocks, 10 s at 48 kHz",
                  fn="plain", dtype="f32"),
    "nup": dict(desc="binaural sources and ears (128 channels), 96000-tap IRs at a 128-sample latency: non-uniform "
                     "partitions (head hop 64, 7 partitions of 128 taps; tail hop 512, 93 partitions of 1024 taps) "
                     "against uniform partitions at hop 64 (750 partitions), 4 IR slots switched every block, "
                     "5 s at 48 kHz", fn="binaural", kw=dict(hop=64), dtype="f32"),
    "autograd": dict(desc="32 channels, L=256, 8192-tap IRs (16 partitions), 2 s at 48 kHz, MSE loss against "
                          "a target made by hidden IRs, gradients for H and x", fn="autograd", dtype="f32"),
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


KERNEL_SOURCES = ("tvolap_kernels.hip", "fft_lds.hpp", "tvolap_internal.h")


def kernel_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2310_00319_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(case: str):
    """HBM bytes per launch from a committed rocprofv3 PMC summary of this case
    (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when no summary covers
    the case or the kernel sources changed since the counters were taken. A
    summary may hold several cases, each starting at its traffic_case line."""
    import glob
    want = kernel_sources_sha256()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        blocks, kv = [], None
        with open(path) as fh:
            for line in fh:
                if ":" not in line or line.startswith((" ", "|", "#")):
                    continue
                k, v = line.split(":", 1)
                k = k.split(" (")[0].strip()
                if k == "traffic_case":
                    kv = {}
                    blocks.append(kv)
                if kv is not None:
                    kv[k] = v.strip()
        for kv in blocks:
            if kv.get("traffic_case") == case and kv.get("kernel_sources_sha256") == want:
                try:
                    return int(kv["traffic_bytes_per_launch"]), os.path.relpath(path, ROOT)
                except (KeyError, ValueError):
                    return None
    return None


def tmac_unique_bytes(wl, batch: int, store_bytes: int) -> int:
    """Bytes that the spectral MAC of batched calls must read at least over one
    pass of the workload: per call, every partition spectrum of every slot a
    channel uses in the call once, and per input and parity class the
    delay-line spectra its blocks reach once (M_i + blocks - 1 rows)."""
    L = wl.hop
    row = 2 * L * store_bytes
    Mc = np.array([-(-int(t) // (2 * L)) for t in wl.taps_of_channel], dtype=np.int64)
    Mi = np.zeros(wl.n_inputs, dtype=np.int64)
    for c in range(wl.n_channels):
        i = int(wl.input_of_channel[c])
        Mi[i] = max(Mi[i], Mc[c])
    total = 0
    for c0 in range(0, wl.n_calls, batch):
        n = min(batch, wl.n_calls - c0)
        for cls in (0, 1):
            nb = len(range(cls, n, 2))
            if nb:
                total += int((Mi + nb - 1).sum()) * row
        slots = np.clip(wl.schedule[c0:c0 + n], 0, wl.n_slots - 1)           # [n][C]
        distinct = np.array([len(np.unique(slots[:, c])) for c in range(wl.n_channels)])
        total += int((distinct * Mc).sum()) * row
    return total


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def _oracle_channels(wl, channels, budget_s: float, keep: list | None = None):
    """FP64 oracle streams of `channels` in order until the budget is spent:
    (channels done, wall s, CPU s)."""
    import oracle as orc

    x = wl.padded_input().astype(np.float64)
    t_wall = time.perf_counter()
    r0 = resource.getrusage(resource.RUSAGE_SELF)
    done = 0
    for c in channels:
        H = orc.channel_spectra([t.astype(np.float64) for t in wl.taps[c]], wl.hop, int(wl.taps_of_channel[c]))
        y = orc.tvolap_stream(x[wl.input_of_channel[c]], H, wl.schedule[:, c], wl.hop, wl.n_calls)
        if keep is not None:
            keep.append(y)
        done += 1
        if time.perf_counter() - t_wall > budget_s:
            break
    wall = time.perf_counter() - t_wall
    r1 = resource.getrusage(resource.RUSAGE_SELF)
    return done, wall, (r1.ru_utime - r0.ru_utime) + (r1.ru_stime - r0.ru_stime)


def _oracle_shard(job):
    """Worker of the multi-core leg (a fresh interpreter: spawned, so it holds
    no GPU state): regenerate the workload from its seeds, then run the oracle
    on this worker's channels until the budget is spent."""
    name, channels, budget_s = job
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[v] = "1"
    import synth
    spec = WORKLOADS[name]
    wl = getattr(synth, spec["fn"])(**spec.get("kw", {}))
    done, wall, _ = _oracle_channels(wl, channels, budget_s)
    return done, wall


def cpu_baseline(wl, name: str, budget_s: float, keep: list | None = None) -> dict:
    """The FP64 oracle on the host, two ways: one process on the first channels
    until the budget is spent (outputs appended to ``keep`` for the accuracy
    check), and channel shards in one single-threaded process per core of this
    process's CPU share (at most 16), for the same budget each. value = the
    multi-core rate."""
    import multiprocessing as mp

    done, wall, cpu = _oracle_channels(wl, range(wl.n_channels), budget_s, keep)
    one = done * wl.n_calls * wl.hop / wall
    try:
        share = len(os.sched_getaffinity(0))
    except AttributeError:
        share = os.cpu_count() or 1
    workers = max(1, min(16, share, wl.n_channels))
    per = [list(range(k, wl.n_channels, workers)) for k in range(workers)]
    multi = None
    try:
        with mp.get_context("spawn").Pool(workers) as pool:
            t0 = time.perf_counter()
            res = pool.map(_oracle_shard, [(name, ch, budget_s) for ch in per])
            span = time.perf_counter() - t0
        # each worker's rate over its own compute time, summed: the aggregate
        # rate with every worker busy (generating the inputs is excluded)
        rate = sum(r[0] * wl.n_calls * wl.hop / max(r[1], 1e-9) for r in res)
        multi = {"value": rate, "workers": workers, "channels": int(sum(r[0] for r in res)), "wall_s": round(span, 1)}
    except Exception as e:   # the single-process figure still stands
        log(f"multi-core oracle leg failed: {e!r}")
    single = {"value": one, "cores": max(1, int(round(cpu / wall))),
              "sample": f"first {done} of {wl.n_channels} channels over the full {wl.n_calls}-block stream "
                        f"({wall:.1f} s wall, {cpu:.1f} s CPU)"}
    if multi is None:
        return {"value": one, "unit": "channel-samples/s", "cores": single["cores"], "kind": "oracle",
                "cpu": _cpu_model(), "host_cpu_count": os.cpu_count(), "cpu_share": share,
                "sample": "FP64 oracle, one process: " + single["sample"]}
    return {"value": multi["value"], "unit": "channel-samples/s", "cores": workers, "kind": "oracle",
            "cpu": _cpu_model(), "host_cpu_count": os.cpu_count(), "cpu_share": share,
            "sample": (f"FP64 oracle, channel shards in {workers} single-threaded processes for about "
                       f"{budget_s:.0f} s each ({multi['channels']} channels over the full {wl.n_calls}-block "
                       f"stream, {multi['wall_s']} s wall with input generation); rate = the sum of the workers' "
                       "rates"),
            "single_process": single}


def head_bus_accuracy(wl, buses, got, budget_s: float) -> dict:
    """Mixdown accuracy: the oracle of every channel over the first blocks of
    the stream (as many as the budget allows; the outputs up to a block depend
    only on the input up to it), summed per bus and compared with ``got``."""
    import dataclasses

    import oracle as orc

    t0 = time.perf_counter()
    H0 = orc.channel_spectra([t.astype(np.float64) for t in wl.taps[0]], wl.hop, int(wl.taps_of_channel[0]))
    x0 = wl.padded_input()[0, : 16 * wl.hop].astype(np.float64)
    orc.tvolap_stream(x0, H0, wl.schedule[:16, 0], wl.hop, 16)
    per_call = max(1e-6, (time.perf_counter() - t0) / 16)
    n = int(max(8, min(wl.n_calls, budget_s / (per_call * wl.n_channels))))
    L = wl.hop
    head = dataclasses.replace(wl, x=wl.x[:, : n * L], schedule=wl.schedule[:n])
    x = head.padded_input().astype(np.float64)
    E = int(np.max(buses)) + 1
    ref = np.zeros((E, n * L))
    for c in range(wl.n_channels):
        H = orc.channel_spectra([t.astype(np.float64) for t in wl.taps[c]], L, int(wl.taps_of_channel[c]))
        ref[int(buses[c])] += orc.tvolap_stream(x[wl.input_of_channel[c]], H, head.schedule[:, c], L, n)
    g = got[:, : n * L]
    rel = np.sqrt(np.sum((g - ref) ** 2, axis=1) / np.maximum(np.sum(ref ** 2, axis=1), 1e-300))
    snr = -20.0 * np.log10(np.maximum(rel, 1e-30))
    return {"vs": "FP64 oracle (unquantized), summed per output bus", "buses": E,
            "blocks_checked": n, "max_rel_rms": float(f"{rel.max():.3e}"),
            "snr_db": {"min": round(float(snr.min()), 2), "max": round(float(snr.max()), 2)}}


def practical_hbm_rates(mib: int = 1024, reps: int = 10) -> dict:
    """What plain streaming kernels reach on this GPU, for context beside the
    8 TB/s peak: torch's device copy (read + write) and a full sum (read), over
    a MIB-MiB float32 buffer, timed with events on torch's stream."""
    import torch
    a = torch.ones(mib * (1 << 18), device="cuda")
    b = torch.empty_like(a)
    nbytes = a.numel() * 4
    b.copy_(a)
    s = a.sum()
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    e[0].record()
    for _ in range(reps):
        b.copy_(a)
    e[1].record()
    for _ in range(reps):
        s = a.sum()
    e[2].record()
    torch.cuda.synchronize()
    copy_ms = e[0].elapsed_time(e[1]) / reps
    read_ms = e[1].elapsed_time(e[2]) / reps
    del a, b, s
    torch.cuda.empty_cache()
    return {"torch_copy_gbs": round(2 * nbytes / (copy_ms * 1e-3) / 1e9, 1),
            "torch_sum_gbs": round(nbytes / (read_ms * 1e-3) / 1e9, 1),
            "buffer_mib": mib, "note": "torch copy_ (bytes read + written) and sum (bytes read) of one buffer; "
                                       "context only, the roofline peak stays 8 TB/s"}


USE_GRAPHS = True   # bench.py --no-graph: issue every call directly (hardware-counter passes)


def pinned_block(args) -> dict | None:
    """The one-block schedule given on the command line (--no-autotune with
    --chunk/--waves/--grid), or None for the autotuner."""
    if not args.no_autotune:
        return None
    return dict(fused=1, chunk=args.chunk, waves=args.waves, grid=args.grid)


def graph_step_ms(conv, step_fn, steps: int, warmup: int = 1) -> float:
    """Capture step_fn() once as a HIP graph on the convolver's stream, replay
    it warmup + steps times and return the milliseconds per replay, from events
    recorded on that stream (torch's current stream here) around the timed
    replays. Without graphs (--no-graph) step_fn() itself is timed."""
    import torch
    if USE_GRAPHS:
        conv.capture_begin()
        step_fn()
        conv.capture_end()
        run = conv.graph_launch
    else:
        run = step_fn
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        run()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def block_roofline(info: dict, us_per_launch: float, case: str) -> dict:
    """Roofline of the one-block kernel: the spectral MAC's algorithmic bytes of
    one block (every active partition spectrum and every same-parity
    delay-line spectrum of each input, once) over the average launch duration,
    against the 8 TB/s HBM peak."""
    kbytes = info["mac_bytes_per_block"]
    gbs = kbytes / (us_per_launch * 1e-6) / 1e9
    tr = measured_traffic(case)
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": tr[0] if tr else None,
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "traffic_source": tr[1] if tr else None,
            "kernel": "k_block (one launch per block: input spectra, spectral MAC of eq. 8, inverse transform and "
                      "overlap-add of the channels)",
            "bytes_per_launch": int(kbytes), "avg_launch_us": round(us_per_launch, 3),
            "duration_source": "graph replay of one launch per block, HIP events on the launch stream "
                               "(launch gaps included)"}


def streaming_leg(conv, wl, x, sched, out, steps: int, case: str, pinned: dict | None = None) -> dict:
    """Strict streaming: one process_block per block (latency 2L), per-block
    schedule autotuned (or `pinned`: configure() arguments), the calls of one
    pass captured as a HIP graph."""
    if pinned:
        conv.configure(**pinned)
        tuned = None
    else:
        tuned = conv.autotune(iters=10)
    info = conv.info()
    conv.reset()
    ms = graph_step_ms(conv, lambda: conv.process(x, sched, out, batch=1), steps)
    us = 1e3 * ms / wl.n_calls
    return {"value": round(wl.n_channels * wl.hop / (us * 1e-6), 1), "unit": "channel-samples/s",
            "us_per_block": round(us, 3), "real_time_factor": round((wl.hop / wl.fs) / (us * 1e-6), 1),
            "latency_samples": 2 * wl.hop, "graph": True, "steps": steps,
            "roofline": block_roofline(info, us, case),
            "schedule": {"chunk": info["mac_chunk"], "waves": info["mac_waves"], "grid": info["mac_grid"],
                         "work_items": info["n_work_items"], "autotuned_us_per_block": tuned}}


def fresh_legs(args, base, stream) -> dict:
    """Head tracking without recurring response sets: the binaural sources and
    ears with 64 sets per ear, block l using set l mod 64, so no set repeats
    within a 64-block call. Three measurements: 64-block calls from a graph,
    strict streaming (one call per block) from a graph, and strict streaming
    where every block first loads the next block's set from taps
    (tvolap_set_irs for all 128 ears, then tvolap_process_block), one graph for
    the whole pass. The partition spectra are loaded from the same taps in
    every case, so the three outputs agree."""
    import torch

    import synth
    from paper_2310_00319_amd import Convolver

    t0 = time.perf_counter()
    wl = synth.binaural_fresh(base=base)
    log(f"fresh response sets generated in {time.perf_counter() - t0:.1f} s: K={wl.n_slots}")
    C, K, L = wl.n_channels, wl.n_slots, wl.hop
    conv = Convolver(hop=L, n_channels=C, max_taps=wl.max_taps(), n_inputs=wl.n_inputs,
                     input_of_channel=wl.input_of_channel, taps_of_channel=wl.taps_of_channel, n_slots=K,
                     dtype="f32", stream=stream, max_batch=64)
    # taps of every set resident on the device ([K][C][n]), loaded slot by slot
    pool = torch.empty((K, C, wl.max_taps()), device="cuda", dtype=torch.float32)
    for k in range(K):
        pool[k].copy_(torch.from_numpy(np.stack([wl.taps[c][k] for c in range(C)])))
        conv.set_irs(k, pool[k])
    torch.cuda.synchronize()
    x = torch.from_numpy(wl.padded_input()).cuda()
    sched = torch.from_numpy(np.ascontiguousarray(wl.schedule, dtype=np.int32)).cuda()
    out_b = torch.empty((C, wl.n_calls * L), device="cuda")
    out_s = torch.empty_like(out_b)
    out_i = torch.empty_like(out_b)
    steps = max(2, args.steps // 2)
    res = {"workload": f"binaural, {K} response sets per ear, block l uses set l mod {K} (no set recurs within "
                       f"{K} blocks)", "ir_sets": K, "bank_bytes": conv.info()["bank_bytes"]}
    # 64-block calls
    if args.no_autotune:
        # the schedule the batched autotuner picks for this workload: vector
        # ALU, time groups of 8 blocks, 2 bins per lane, one channel per item
        conv.configure_batch(chunk=args.bchunk, vec=args.bvec or 2, waves=args.bwaves, time_block=args.btb or 8,
                             group=args.bgroup or 1, engine=1)
        tuned = None
    else:
        tuned = conv.autotune_batch(iters=2)
    info = conv.info()
    conv.reset()
    ms = graph_step_ms(conv, lambda: conv.process(x, sched, out_b, batch=64), steps)
    calls = -(-wl.n_calls // 64)
    conv.set_timing(True)
    conv.get_timing()
    conv.process(x, sched, out_b, batch=64)
    tm = conv.get_timing()
    conv.set_timing(False)
    mac_us = 1e3 * tm["ms_mac"] / calls
    kbytes = tmac_unique_bytes(wl, 64, 8) / calls
    gbs = kbytes / (mac_us * 1e-6) / 1e9
    mfma = info["batch_engine"] == 2
    tr = measured_traffic("binaural_fresh batch64 " + ("k_tmfma" if mfma else "k_tmac"))
    res["blocks_per_call_64"] = {
        "value": round(C * wl.n_calls * L / (ms * 1e-3), 1), "unit": "channel-samples/s",
        "us_per_block": round(1e3 * ms / wl.n_calls, 3), "buffering_ms": round(1e3 * 64 * L / wl.fs, 1),
        "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": tr[0] if tr else None,
                     "traffic_source": tr[1] if tr else None,
                     "kernel": "batched spectral MAC of eq. 8 (" + ("matrix-core engine with its vector-ALU units" if mfma
                                                                    else "k_tmac, vector ALU") + ")",
                     "bytes_per_launch": int(kbytes), "avg_launch_us": round(mac_us, 3),
                     "bytes_note": "unique bytes of a call: the partition spectra of all 64 sets once, the delay-line "
                                   "spectra the call's blocks reach once per input and parity"},
        "phase_us_per_block": {"in": round(1e3 * tm["ms_in"] / tm["blocks"], 3),
                               "mac": round(1e3 * tm["ms_mac"] / tm["blocks"], 3),
                               "out": round(1e3 * tm["ms_out"] / tm["blocks"], 3)},
        "schedule": {"engine": {1: "vector ALU", 2: "matrix cores"}[info["batch_engine"]],
                     "time_block": info["batch_time_block"], "chunk": info["batch_chunk"],
                     "vec": info["batch_vec"], "waves": info["batch_waves"], "group": info["batch_group"],
                     "autotuned_us_per_block": tuned}}
    # one block per call
    conv.reset()
    res["one_block_per_call"] = streaming_leg(conv, wl, x, sched, out_s, steps, "binaural_fresh stream k_block",
                                              pinned_block(args))
    # one block per call, each preceded by loading the next block's set from taps
    conv.reset()

    def ingest_pass():
        for c in range(wl.n_calls):
            k = c % K
            conv.set_irs(k, pool[k])
            conv.process_block(x[:, c * L:(c + 1) * L], out_i[:, c * L:(c + 1) * L], sched[c])

    ms_i = graph_step_ms(conv, ingest_pass, steps)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(K):
        conv.set_irs(k, pool[k])
    e1.record()
    torch.cuda.synchronize()
    us_set = 1e3 * e0.elapsed_time(e1) / K
    us_i = 1e3 * ms_i / wl.n_calls
    parts = info["sum_partitions"]
    res["one_block_per_call_with_taps_every_block"] = {
        "value": round(C * L / (us_i * 1e-6), 1), "unit": "channel-samples/s", "us_per_block": round(us_i, 3),
        "real_time_factor": round((L / wl.fs) / (us_i * 1e-6), 1),
        "ingest_us_per_block": round(us_set, 2), "ingest_share": round(us_set / us_i, 3),
        "ingest_partition_transforms_per_s": round(parts / (us_set * 1e-6), 1),
        "note": "per block: tvolap_set_irs (partition, zero pad, transform and store the 24064 partition spectra "
                "of the next set from device taps [128][96000]) then tvolap_process_block; the whole pass is one "
                "captured graph"}
    # agreement of the three paths (the same taps and schedule)
    conv.reset()
    conv.process(x, sched, out_b, batch=64)
    conv.reset()
    conv.process(x, sched, out_s, batch=1)
    conv.reset()
    if USE_GRAPHS:
        conv.graph_launch()                   # the ingest pass
    else:
        ingest_pass()
    torch.cuda.synchronize()
    ob, os_, oi = out_b.double(), out_s.double(), out_i.double()
    res["ingest_equals_prebanked_bitwise"] = bool(torch.equal(out_i, out_s))
    res["batched_vs_one_block_max_rel_rms"] = float(f"{float(((ob - os_).norm(dim=1) / os_.norm(dim=1)).max()):.3e}")
    if not args.no_cpu_baseline:
        import oracle as orc
        xs = wl.padded_input().astype(np.float64)
        errs = []
        for c in (0, C - 1):
            H = orc.channel_spectra([t.astype(np.float64) for t in wl.taps[c]], L, int(wl.taps_of_channel[c]))
            ref = orc.tvolap_stream(xs[wl.input_of_channel[c]], H, wl.schedule[:, c], L, wl.n_calls)
            for o in (ob, os_):
                g = o[c].cpu().numpy()
                errs.append(float(np.linalg.norm(g - ref) / np.linalg.norm(ref)))
        res["accuracy"] = {"vs": "FP64 oracle", "channels": [0, C - 1], "max_rel_rms": float(f"{max(errs):.3e}")}
    conv.close()
    del pool
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="binaural", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--mode", default="fused", choices=["fused", "two", "plain"],
                    help="fused: one kernel per block; two: transform-in + MAC, then transform-out; "
                         "plain: transform-in, MAC, transform-out kernels")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--waves", type=int, default=0)
    ap.add_argument("--grid", type=int, default=0)
    ap.add_argument("--batch", type=int, default=64,
                    help="blocks per call (1 = strict streaming, one block per call; >1 = batched calls)")
    ap.add_argument("--bchunk", type=int, default=0, help="batched MAC: partitions per work item")
    ap.add_argument("--bvec", type=int, default=0, help="batched MAC: complex bins per lane (1 or 2)")
    ap.add_argument("--bwaves", type=int, default=0, help="batched MAC: waves per workgroup (1, 2, 4 or 8)")
    ap.add_argument("--btb", type=int, default=0, help="batched MAC: blocks per time group (8, 16 or 32)")
    ap.add_argument("--bgroup", type=int, default=0, help="batched MAC: channels per work item (1 or 2)")
    ap.add_argument("--bengine", type=int, default=0,
                    help="batched MAC engine: 1 = vector ALU, 2 = matrix cores (f32 spectra)")
    ap.add_argument("--no-ingest", action="store_true", help="skip the IR-bank ingestion timing")
    ap.add_argument("--no-autograd", action="store_true", help="skip the forward/backward timing of the "
                                                                  "differentiable form")
    ap.add_argument("--fresh-only", action="store_true",
                    help="only the legs with 64 response sets per ear (binaural)")
    ap.add_argument("--no-fresh", action="store_true",
                    help="skip the legs with 64 response sets per ear (no set recurs within 64 blocks)")
    ap.add_argument("--no-realtime", action="store_true",
                    help="skip the extra one-block-per-call measurement")
    ap.add_argument("--no-graph", dest="graph", action="store_false",
                    help="issue the calls of a step directly instead of replaying one captured HIP graph")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-MiB float32 buffer 5 times (hardware-counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        a = torch.ones(args.calibrate_copy * (1 << 18), device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": a.numel() * 4, "copies": 5}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); channels are independent, "
              "so more GPUs would shard channels with no communication", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_2310_00319_amd import Convolver

    global USE_GRAPHS
    USE_GRAPHS = args.graph
    spec = WORKLOADS[args.workload]
    log(f"workload {args.workload}: {spec['desc']}")
    t0 = time.perf_counter()
    wl = getattr(synth, spec["fn"])(**spec.get("kw", {}))
    log(f"generated in {time.perf_counter() - t0:.1f} s: C={wl.n_channels} I={wl.n_inputs} L={wl.hop} "
        f"calls={wl.n_calls}")
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        if args.workload == "autograd":
            return run_autograd(args, spec, wl)
        if args.workload == "nup":
            return run_nup(args, spec, wl, stream)
        if args.fresh_only:
            fresh = fresh_legs(args, wl, stream)
            print(json.dumps({"fresh_response_sets": fresh}), flush=True)
            return
        return run(args, spec, wl, stream)


def run_nup(args, spec, wl, stream):
    """Non-uniform partitions (short head, long tail) against uniform ones at
    the same latency (hop 64, 2L = 128 samples): one call per 64 samples, each
    pass captured as a HIP graph (a whole number of the non-uniform handle's
    ring period), HIP events on the stream."""
    import torch

    from paper_2310_00319_amd import Convolver
    from paper_2310_00319_amd.nup import NupConvolver

    L, C, K = wl.hop, wl.n_channels, wl.n_slots
    r, M1 = 8, 7
    x = torch.from_numpy(wl.padded_input()).cuda()
    sched = torch.from_numpy(np.ascontiguousarray(wl.schedule, dtype=np.int32)).cuda()
    out = torch.zeros((C, wl.n_calls * L), device="cuda")
    nup = NupConvolver(hop=L, tail_ratio=r, head_partitions=M1, n_channels=C, max_taps=wl.max_taps(),
                       n_inputs=wl.n_inputs, input_of_channel=wl.input_of_channel, n_slots=K, stream=stream)
    for c in range(C):
        for k in range(K):
            nup.set_ir(c, k, wl.taps[c][k])
    nup.autotune(iters=10)
    P = nup.period
    n = (wl.n_calls // P) * P

    def timed(conv, fn):
        conv.capture_begin()
        fn()
        conv.capture_end()
        conv.graph_launch()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            conv.graph_launch()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps

    t0 = time.perf_counter()
    ms_nup = timed(nup, lambda: nup.process(x, sched, out, n_calls=n))
    elapsed = time.perf_counter() - t0
    nup.reset()
    nup.process(x, sched, out, n_calls=n)
    torch.cuda.synchronize()
    got = out[:, : n * L].double().cpu().numpy()
    nup.close()
    uni = Convolver(hop=L, n_channels=C, max_taps=wl.max_taps(), n_inputs=wl.n_inputs,
                    input_of_channel=wl.input_of_channel, n_slots=K, stream=stream)
    for c in range(C):
        for k in range(K):
            uni.set_ir(c, k, wl.taps[c][k])
    uni.autotune(iters=10)
    info = uni.info()
    uni.reset()
    ms_uni = timed(uni, lambda: uni.process(x[:, : n * L], sched, out[:, : n * L], batch=1))
    uni.close()
    us_nup = 1e3 * ms_nup / n
    us_uni = 1e3 * ms_uni / n
    accuracy = None
    if not args.no_cpu_baseline:
        from oracle import nup_ref
        xs = wl.padded_input().astype(np.float64)
        errs = []
        for c in (0, C - 1):
            ref = nup_ref.nup_stream(xs[wl.input_of_channel[c]], [t.astype(np.float64) for t in wl.taps[c]],
                                     wl.schedule[:, c], L, M1, r, int(wl.taps_of_channel[c]), n)
            errs.append(float(np.linalg.norm(got[c] - ref) / np.linalg.norm(ref)))
        accuracy = {"vs": "FP64 non-uniform oracle", "channels": [0, C - 1], "max_rel_rms": float(f"{max(errs):.3e}")}
    res = {
        "metric": "channel-samples/s at a 128-sample latency, 2-s IRs: non-uniform partitions",
        "value": round(C * L / (us_nup * 1e-6), 1), "unit": "channel-samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": 1, "ms_per_step": round(1e3 * elapsed / args.steps, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"nup: {spec['desc']}", "channels": C, "hop": L, "tail_hop": r * L,
                   "head_partitions": M1, "ir_taps": int(wl.max_taps()), "calls_per_step": n},
        "us_per_call": round(us_nup, 3), "latency_samples": 2 * L,
        "real_time_factor": round((L / wl.fs) / (us_nup * 1e-6), 1),
        "uniform_same_latency": {"value": round(C * L / (us_uni * 1e-6), 1), "us_per_call": round(us_uni, 3),
                                 "partitions_per_channel": int(info["sum_partitions"] // C),
                                 "mac_bytes_per_block": int(info["mac_bytes_per_block"])},
        "speedup_vs_uniform": round(us_uni / us_nup, 3),
        "roofline": None, "cpu_baseline": None, "accuracy": accuracy,
    }
    print(json.dumps(res), flush=True)


def autograd_times(wl, steps: int, warmup: int) -> dict:
    """Offline differentiable form: MSE loss against the hidden-IR target,
    forward and backward (gradients for H and x) timed separately with events."""
    import torch

    from paper_2310_00319_amd import functional as F

    C, N, L = wl.n_channels, wl.n_samples, wl.hop
    taps = torch.from_numpy(np.stack([wl.taps[c][0] for c in range(C)])[:, None, :].copy()).cuda()
    H = F.ir_spectra(taps, L).requires_grad_(True)
    x = torch.from_numpy(wl.x).cuda().requires_grad_(True)
    target = torch.from_numpy(wl.target).cuda()

    def fwd():
        return torch.mean((F.tvolap(x, H, L) - target) ** 2)

    for _ in range(warmup):
        fwd().backward()
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    f_ms = b_ms = 0.0
    t0 = time.perf_counter()
    for k in range(steps):
        x.grad = None
        H.grad = None
        e[0].record()
        loss = fwd()
        e[1].record()
        loss.backward()
        e[2].record()
        torch.cuda.synchronize()
        f_ms += e[0].elapsed_time(e[1])
        b_ms += e[1].elapsed_time(e[2])
    elapsed = time.perf_counter() - t0
    return {"forward_ms": round(f_ms / steps, 4), "backward_ms": round(b_ms / steps, 4),
            "backward_forward_ratio": round(b_ms / f_ms, 3), "ms_per_step": round(1e3 * elapsed / steps, 4),
            "channels": C, "hop": L, "partitions": int(H.shape[2]), "samples": N,
            "partitions_note": "input spectra recomputed in the backward pass, not stored"}


def run_autograd(args, spec, wl):
    """Offline differentiable form: MSE loss against the hidden-IR target,
    forward and backward (gradients for H and x) timed separately."""
    C, N, L = wl.n_channels, wl.n_samples, wl.hop
    t = autograd_times(wl, args.steps, args.warmup)
    res = {
        "metric": "channel-samples/s of one forward + backward pass (offline differentiable TVOLAP)",
        "value": round(C * N / (t["ms_per_step"] / 1e3), 1),
        "unit": "channel-samples/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": t["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"autograd: {spec['desc']}", "channels": C, "hop": L, "ir_taps": int(wl.max_taps()),
                   "partitions": t["partitions"], "samples": N},
        "forward_ms": t["forward_ms"], "backward_ms": t["backward_ms"],
        "backward_forward_ratio": t["backward_forward_ratio"],
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(res), flush=True)


def run(args, spec, wl, stream):
    import torch

    from paper_2310_00319_amd import Convolver

    buses = None
    mix = {}
    if spec.get("buses") == "ear":
        buses = (np.arange(wl.n_channels) % 2).astype(np.int32)
        mix = dict(n_outputs=2, output_of_channel=buses)
        if args.mode == "fused":
            args.mode = "plain"      # a mixdown runs the separate transform-out launch
    conv = Convolver(hop=wl.hop, n_channels=wl.n_channels, max_taps=wl.max_taps(), n_inputs=wl.n_inputs,
                     input_of_channel=wl.input_of_channel, taps_of_channel=wl.taps_of_channel,
                     n_slots=wl.n_slots, dtype=spec["dtype"], stream=stream, max_batch=max(16, args.batch), **mix)
    t0 = time.perf_counter()
    for c in range(wl.n_channels):
        for s in range(wl.n_slots):
            conv.set_ir(c, s, wl.taps[c][s])
    torch.cuda.synchronize()
    t_setir = time.perf_counter() - t0
    info0 = conv.info()
    # IR-bank ingestion: every slot of every channel again, one launch per
    # slot from device taps (writes the same spectra)
    ingest = None
    if not args.no_ingest:
        rows = []
        for k in range(wl.n_slots):
            r = np.zeros((wl.n_channels, wl.max_taps()), np.float32)
            for c in range(wl.n_channels):
                t = wl.taps[c][k]
                r[c, :len(t)] = t
            rows.append(torch.from_numpy(r).cuda())
        for k in range(wl.n_slots):
            conv.set_irs(k, rows[k])
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        reps = 3
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            for k in range(wl.n_slots):
                conv.set_irs(k, rows[k])
        e1.record()
        torch.cuda.synchronize()
        us = 1e3 * e0.elapsed_time(e1) / (reps * wl.n_slots)
        parts = info0["sum_partitions"]
        ingest = {"us_per_slot_all_channels": round(us, 2), "partitions_per_slot": int(parts),
                  "partition_transforms_per_s": round(parts / (us * 1e-6), 1),
                  "taps_per_s": round(parts * 2 * wl.hop / (us * 1e-6), 1)}
        del rows
    tuned_us = None
    tuned_batch_us = None
    if args.batch > 1 and (args.bchunk or args.bvec or args.bwaves or args.btb or args.bgroup or args.bengine):
        conv.configure_batch(chunk=args.bchunk, vec=args.bvec, waves=args.bwaves, time_block=args.btb,
                             group=args.bgroup, engine=args.bengine)
    elif args.batch > 1 and not args.no_autotune:
        t0 = time.perf_counter()
        tuned_batch_us = conv.autotune_batch(iters=3)
        log(f"batched schedule autotuned in {time.perf_counter() - t0:.2f} s: best {tuned_batch_us:.2f} us/block")
    if (args.mode != "fused" and buses is None) or args.chunk or args.waves or args.grid or args.no_autotune:
        conv.configure(fused={"fused": 1, "two": 2, "plain": 0}[args.mode], chunk=args.chunk, waves=args.waves,
                       grid=args.grid)
    else:
        t0 = time.perf_counter()
        tuned_us = conv.autotune(iters=10)
        log(f"autotuned in {time.perf_counter() - t0:.2f} s: best {tuned_us:.2f} us/block")
    info = conv.info()
    log(f"IR bank loaded in {t_setir:.2f} s; info {info}")

    x = torch.from_numpy(wl.padded_input()).cuda()
    sched = torch.from_numpy(np.ascontiguousarray(wl.schedule, dtype=np.int32)).cuda()
    out = torch.empty((conv.n_outputs, wl.n_calls * wl.hop), device="cuda", dtype=torch.float32)
    torch.cuda.synchronize()

    if args.graph:
        if args.batch > 1:
            conv.process(x[:, : wl.hop * args.batch], sched, out[:, : wl.hop * args.batch], batch=args.batch)
            conv.reset()   # batch buffers are allocated outside the capture
        conv.capture_begin()
        conv.process(x, sched, out, batch=args.batch)
        conv.capture_end()
        log("captured one step as a HIP graph")

    def step():
        if args.graph:
            conv.graph_launch()
        else:
            conv.process(x, sched, out, batch=args.batch)

    for w in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup {w + 1}/{args.warmup} done")

    per_kernel = not args.no_kernel_timing and not args.graph and (args.mode != "fused" or args.batch > 1)
    kernel_pass = not args.no_kernel_timing and args.graph and args.batch > 1
    if per_kernel:
        conv.set_timing(True)
        conv.get_timing()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    for k in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    log(f"timed {args.steps} steps in {elapsed:.3f} s")
    timing = conv.get_timing() if per_kernel else None
    conv.set_timing(False)
    if kernel_pass:
        # kernel durations do not depend on how the launches were issued: time
        # the same calls once more without the graph, with the library's events
        conv.set_timing(True)
        conv.get_timing()
        for k in range(max(1, args.steps // 2)):
            conv.process(x, sched, out, batch=args.batch)
        timing = conv.get_timing()
        conv.set_timing(False)
        timing_steps = max(1, args.steps // 2)
    else:
        timing_steps = args.steps
    calls_per_step = -(-wl.n_calls // args.batch)
    if not per_kernel and not kernel_pass and not args.no_kernel_timing:
        # One kernel per block: the events that bracket the timed region on the
        # convolver's stream give its average launch duration (inter-launch
        # gaps included, so this is an upper bound on the kernel's time).
        timing = {"ms_in": 0.0, "ms_mac": gpu_ms / args.steps * (1.0 if info["fused"] == 1 else 0.0),
                  "ms_out": 0.0, "blocks": wl.n_calls}
        if info["fused"] != 1:
            timing = None

    streaming = None
    if args.batch > 1 and not args.no_realtime:
        streaming = streaming_leg(conv, wl, x, sched, out, max(2, args.steps // 2), f"{args.workload} stream k_block",
                                  pinned_block(args))
        log(f"strict streaming: {streaming['us_per_block']} us per block, "
            f"{streaming['roofline']['frac']} of HBM peak")

    autograd = None
    if args.workload == "binaural" and not args.no_autograd:
        import synth
        autograd = autograd_times(synth.autograd(), max(3, args.steps // 2), 1)
        autograd["workload"] = WORKLOADS["autograd"]["desc"]
        log(f"autograd: {autograd}")

    fresh = None
    if args.workload == "binaural" and not args.no_fresh:
        fresh = fresh_legs(args, wl, torch.cuda.current_stream())
        log(f"fresh response sets: {json.dumps(fresh)}")

    ms_per_step = 1e3 * elapsed / args.steps
    blocks = wl.n_calls
    ch_samples = wl.n_channels * blocks * wl.hop
    value = ch_samples / (ms_per_step / 1e3)
    us_per_block = 1e3 * ms_per_step / blocks
    rtf = (wl.hop / wl.fs) / (us_per_block * 1e-6)

    roof = None
    if timing and timing["blocks"] > 0 and args.batch > 1:
        # dominant kernel: k_tmac, one launch per call over its blocks. Two
        # floors: the unique bytes it must read at 8 TB/s, and its complex
        # multiply-adds (8 flop each) at the FP32 FMA issue rate; the larger one
        # is the bound the kernel is measured against.
        launches = timing_steps * calls_per_step
        mac_ms = timing["ms_mac"] / launches
        store = 8 if spec["dtype"] == "f32" else 4
        kbytes = tmac_unique_bytes(wl, args.batch, store) / calls_per_step
        kflops = 8.0 * info["sum_partitions"] * 2 * wl.hop * wl.n_calls / calls_per_step
        gbs = kbytes / (mac_ms * 1e-3) / 1e9
        tfs = kflops / (mac_ms * 1e-3) / 1e12
        floor_hbm = kbytes / (HBM_PEAK_GBS * 1e9)
        mfma = info["batch_engine"] == 2
        kname = ("k_tmfma" if spec["dtype"] == "f32" else "k_tmfma16") if mfma else "k_tmac"
        if mfma:
            alu_peak = MFMA_F32_PEAK_TFLOPS if spec["dtype"] == "f32" else MFMA_16_PEAK_TFLOPS
        else:
            alu_peak = VALU_PEAK_TFLOPS if spec["dtype"] == "f32" else DOT2_PEAK_TFLOPS
        floor_alu = kflops / (alu_peak * 1e12)
        per_block = info["mac_bytes_per_block"] * wl.n_calls / calls_per_step
        tr = measured_traffic(f"{args.workload} batch{args.batch} {kname}")
        hbm = {"achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
               "bytes_per_launch": int(kbytes), "floor_us": round(floor_hbm * 1e6, 2)}
        alu = {"achieved": round(tfs, 2), "peak": round(alu_peak, 2), "unit": "TFLOP/s",
               "frac": round(tfs / alu_peak, 4), "flops_per_launch": int(kflops),
               "floor_us": round(floor_alu * 1e6, 2),
               "peak_note": ("dense matrix-core peak of the input type (16-bin 4x4 MFMAs)" if mfma else
                             "FP32 FMA issue rate without packed-FP32 instructions (256 CU x 4 SIMD x 16 lanes x "
                             "2 flop x 2.4 GHz); the published packed figure is 157.3" if spec["dtype"] == "f32"
                             else "two-element 16-bit dot products with FP32 accumulation: 256 CU x 4 SIMD x 16 "
                                  "lanes x 4 flop x 2.4 GHz")}
        cname = "mfma" if mfma else "alu"
        main, other = (("hbm", hbm), (cname, alu)) if floor_hbm >= floor_alu else ((cname, alu), ("hbm", hbm))
        roof = {"bound": main[0], "achieved": main[1]["achieved"], "peak": main[1]["peak"], "unit": main[1]["unit"],
                "frac": main[1]["frac"], "traffic": tr[0] if tr else None,
                "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "traffic_source": tr[1] if tr else None,
                "kernel": ((kname + " (time-blocked spectral MAC of eq. 8 on matrix cores)" if mfma else
                            "k_tmac (time-blocked spectral MAC of eq. 8 over a batch of blocks)")),
                "avg_launch_us": round(mac_ms * 1e3, 3), main[0]: main[1], other[0]: other[1],
                "bytes_note": "unique delay-line and partition spectra of each call",
                "per_block_bytes_per_launch": int(per_block),
                "effective_gbs_per_block_bytes": round(per_block / (mac_ms * 1e-3) / 1e9, 1),
                "phase_us_per_block": {"in": round(1e3 * timing["ms_in"] / timing["blocks"], 3),
                                       "mac": round(1e3 * timing["ms_mac"] / timing["blocks"], 3),
                                       "out": round(1e3 * timing["ms_out"] / timing["blocks"], 3)}}
    elif timing and timing["blocks"] > 0:
        mac_ms = timing["ms_mac"] / timing["blocks"]
        if info["fused"] == 1:
            kbytes = info["block_bytes"]
            kname = "k_block (fused: transform-in, spectral MAC of eq. 8, transform-out + overlap-add)"
        elif info["fused"] == 2:
            kbytes = info["mac_bytes_per_block"]
            kname = "k_block (transform-in fused into the spectral MAC of eq. 8)"
        else:
            kbytes = info["mac_bytes_per_block"]
            kname = "k_mac (spectral MAC of eq. 8)"
        achieved = kbytes / (mac_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": kname,
                "bytes_per_launch": kbytes,
                "avg_launch_us": round(mac_ms * 1e3, 3),
                "phase_us_per_block": {"in": round(1e3 * timing["ms_in"] / timing["blocks"], 3),
                                       "mac": round(1e3 * mac_ms, 3),
                                       "out": round(1e3 * timing["ms_out"] / timing["blocks"], 3)}}

    if roof is not None and roof["bound"] == "hbm":
        roof["hbm_practical"] = practical_hbm_rates()

    cpu = None
    accuracy = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        ref = []
        cpu = cpu_baseline(wl, args.workload, args.cpu_budget, ref)
        # accuracy of the same configuration: one fresh pass (untimed) from a
        # reset state, compared per channel with the oracle channels above
        conv.reset()
        conv.process(x, sched, out, batch=args.batch)
        torch.cuda.synchronize()
        if buses is not None:
            accuracy = head_bus_accuracy(wl, buses, out.double().cpu().numpy(), args.cpu_budget)
        else:
            got = out[: len(ref)].double().cpu().numpy()
            ref = np.stack(ref)
            rel = np.sqrt(np.sum((got - ref) ** 2, axis=1) / np.maximum(np.sum(ref ** 2, axis=1), 1e-300))
            snr = -20.0 * np.log10(np.maximum(rel, 1e-30))
            accuracy = {"vs": "FP64 oracle (unquantized)", "channels": int(len(ref)),
                        "max_rel_rms": float(f"{rel.max():.3e}"),
                        "snr_db": {"min": round(float(snr.min()), 2), "median": round(float(np.median(snr)), 2),
                                   "max": round(float(snr.max()), 2)}}
        log(f"accuracy: {accuracy}")

    res = {
        "metric": "channel-samples/s at L=256, 2-s IRs (FP32 vs BF16/batched); % HBM peak",
        "value": round(value, 1),
        "unit": "channel-samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",   # transforms and accumulation; spectra storage is config.spectra_dtype
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {spec['desc']}", "channels": wl.n_channels,
                   "inputs": wl.n_inputs, "hop": wl.hop, "ir_taps": int(wl.max_taps()),
                   "partitions_total": info["sum_partitions"], "blocks_per_step": blocks,
                   "spectra_dtype": spec["dtype"], "outputs": conv.n_outputs},
        "us_per_block": round(us_per_block, 3),
        "real_time_factor": round(rtf, 1),
        "roofline": roof,
        "cpu_baseline": cpu,
        "accuracy": accuracy,
        "ir_bank_load_s": round(t_setir, 3),
        "ir_bank_ingest": ingest,
        "graph": bool(args.graph),
        "blocks_per_call": args.batch,
        "streaming_one_block_per_call": streaming,
        "fresh_response_sets": fresh,
        "autograd_forward_backward": autograd,
        "schedule": {"mode": {1: "fused", 2: "two", 0: "plain"}[info["fused"]], "chunk": info["mac_chunk"],
                     "waves": info["mac_waves"], "grid": info["mac_grid"], "work_items": info["n_work_items"],
                     "autotuned_us_per_block": tuned_us,
                     "batch": {"chunk": info["batch_chunk"], "vec": info["batch_vec"], "waves": info["batch_waves"],
                               "time_block": info["batch_time_block"], "group": info["batch_group"],
                               "engine": {1: "vector ALU", 2: "matrix cores"}[info["batch_engine"]],
                               "tile_width": info["batch_tile_width"], "work_items": info["batch_work_items"],
                               "autotuned_us_per_block": tuned_batch_us}},
    }
    conv.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
