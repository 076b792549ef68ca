"""FP64 oracle of TVOLAP with non-uniform partitions: a head of short
partitions for low latency and a tail of long partitions for a low cost per
sample (Jaeger et al., arXiv 2310.00319, Sec. 1: uniform and non-uniform
partitioning of the impulse response in partitioned convolution; the
time-variant partitioned method of Sec. 2 applied to each part).

TEST INFRASTRUCTURE ONLY: imported by tests, never by the GPU library or its
binding.

Definition (a reading: the paper describes TVOLAP with uniform partitions and
names non-uniform partitioning only as prior art for time-invariant
convolution):
  * Head: hop L1, responses truncated to their first D = 2 L1 M1 taps, i.e. M1
    partitions of 2 L1 (Sec. 2 at hop L1).
  * Tail: hop L2 = r L1 (r >= 1), responses from tap D on, M2 partitions of
    2 L2 (Sec. 2 at hop L2), and the output delayed by D samples.
  * y(t) = y_head(t) + y_tail(t - D), each part a TVOLAP output with its own
    block grid, so the head cross-fades switches over L1 samples and the tail
    over L2.
  * Schedule. A streaming call c (L1 new samples) selects the set of head block
    c - 1. Tail block l2 (tail call c2 = l2 + 1) contributes from output time
    l2 L2 + D on, where head block l1 = r l2 + 2 M1 starts: it takes the set of
    that head block, i.e. of head call c = r (c2 - 1) + 2 M1 + 1, and is
    computed in that call. With r = 1 this is uniform TVOLAP at hop L1.
  * Causality. Tail call c2 needs the input up to (c2 + 1) L2, which head call
    c has received whenever M1 >= r - 1 (D >= (2r - 2) L1); its L2 output
    samples are emitted over head calls c .. c + r - 1. The stream output is y
    delayed by L1 (latency 2 L1 as with uniform partitions at hop L1).

Pins (tests/test_nup_pins.py): brute-force convolution for one response;
r = 1 reproduces uniform TVOLAP at hop L1 for any schedule; the time-domain
block definition of each part with numpy.convolve; causality of the stream
against future inputs and selections.
"""
from __future__ import annotations

import numpy as np

from .tvolap_ref import num_partitions, partition_spectra, tvolap_stream

__all__ = ["nup_split", "nup_tail_schedule", "nup_stream"]


def nup_split(h: np.ndarray, L1: int, M1: int, L2: int, n_taps: int) -> tuple:
    """Head and tail partition spectra of one response: ([M1][2L1+1],
    [M2][2L2+1]) with D = 2 L1 M1 and M2 = ceil((n_taps - D) / 2 L2) (>= 1)."""
    h = np.asarray(h, dtype=np.float64)
    D = 2 * L1 * M1
    head = h[:D]
    tail = h[D:] if h.shape[0] > D else np.zeros(1)
    M2 = num_partitions(max(n_taps - D, 1), L2)
    return partition_spectra(head, L1, M1), partition_spectra(tail, L2, M2)


def nup_tail_schedule(schedule: np.ndarray, r: int, M1: int, n_tail_calls: int) -> np.ndarray:
    """Set of tail call c2 = the set of head call r (c2 - 1) + 2 M1 + 1 (rows
    past the schedule's end repeat its last row)."""
    idx = r * (np.arange(n_tail_calls) - 1) + 2 * M1 + 1
    idx = np.clip(idx, 0, len(schedule) - 1)
    return np.asarray(schedule)[idx]


def nup_stream(x: np.ndarray, sets: list, schedule: np.ndarray, L1: int, M1: int, r: int, n_taps: int,
               n_calls: int) -> np.ndarray:
    """Stream output of n_calls head calls (y(t) for t in [-L1, (n_calls - 1) L1))
    of one channel; ``schedule[c]`` is the set selected by call c."""
    L2 = r * L1
    D = 2 * L1 * M1
    pairs = [nup_split(h, L1, M1, L2, n_taps) for h in sets]
    H1 = np.stack([p[0] for p in pairs])
    H2 = np.stack([p[1] for p in pairs])
    head = tvolap_stream(x, H1, np.asarray(schedule)[:n_calls], L1, n_calls)   # y_head on [-L1, ...)
    n2 = -(-(n_calls * L1 + D) // L2) + 2
    xt = np.zeros(n2 * L2)
    xa = np.asarray(x, dtype=np.float64)[: n2 * L2]
    xt[: xa.shape[0]] = xa
    tail = tvolap_stream(xt, H2, nup_tail_schedule(schedule, r, M1, n2), L2, n2)  # y_tail on [-L2, ...)
    out = head.copy()
    # out[i] = y(i - L1); y_tail(tau) sits at tail[tau + L2], added at tau = i - L1 - D
    for i in range(n_calls * L1):
        tau = i - L1 - D
        if tau >= 0 and tau + L2 < tail.shape[0]:
            out[i] += tail[tau + L2]
    return out
