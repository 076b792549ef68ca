"""Independent formulations of TVOLAP used to pin the oracle.

None of these calls the oracle or an FFT. Each one reaches the paper's result
by a different road:

* ``block_definition``: the time-domain meaning of eq. 8 (Sec. 2). Because 4L
  is at least 2L + 2L - 1, the product of two zero-padded 4L spectra is the
  linear convolution of a windowed 2L input block with a 2L partition, so the
  output is the sum over blocks l and partitions m of (xhat_{l-2m} * h_m) placed
  at time lL. Computed with numpy.convolve only.
* ``crossfade_closed_form``: a closed form derived from eq. 1, 8 and 13. Tap d
  of IR set s reaches output time t from input sample t - d through the block
  l whose window then weights it by w(t - (d mod 2L) - lL). Summing over the
  blocks that use set s gives that set's activity c_s(tau) = sum over l with
  g(l) = s of w(tau - lL), so
      y(t) = sum_s sum_{r < 2L} c_s(t - r) (x * h_s^(r))(t),
  where h_s^(r) keeps the taps d = r (mod 2L) of set s. With one set this is
  plain convolution because the windows sum to one.
* ``naive_dft``: an O(n^2) DFT loop.
"""
from __future__ import annotations

import math

import numpy as np


def hann_half_amplitude(L: int) -> np.ndarray:
    """w(n) = sin^2(pi n / 2L), n < 2L: the periodic Hann window at amplitude 1/2
    written through the half-angle identity rather than eq. 2's cosine."""
    return np.array([math.sin(math.pi * n / (2 * L)) ** 2 for n in range(2 * L)])


def _sched(schedule, l):
    b = l + 1
    if b < 0:
        b = 0
    if b >= len(schedule):
        b = len(schedule) - 1
    return int(schedule[b])


def block_definition(x, sets, schedule, L, n_out):
    """y(t), t in [0, n_out), from blocks l >= -1 as sum_m (xhat_{l-2m} * h_m)(t - lL)."""
    x = np.asarray(x, dtype=np.float64)
    N = x.shape[0]
    w = hann_half_amplitude(L)
    n_taps = max(len(s) for s in sets)
    M = max(1, -(-n_taps // (2 * L)))
    parts = []
    for s in sets:
        flat = np.zeros(2 * L * M)
        flat[: len(s)] = s
        parts.append(flat.reshape(M, 2 * L))

    def xhat(j):
        out = np.zeros(2 * L)
        for n in range(2 * L):
            t = j * L + n
            if 0 <= t < N:
                out[n] = x[t] * w[n]
        return out

    y = np.zeros(n_out + 8 * L)
    last_block = -(-n_out // L)
    for l in range(-1, last_block + 1):
        s = _sched(schedule, l)
        for m in range(M):
            j = l - 2 * m
            if j < -1:
                break
            seg = np.convolve(xhat(j), parts[s][m])          # length 4L - 1
            start = l * L
            for n, v in enumerate(seg):
                t = start + n
                if 0 <= t < y.shape[0]:
                    y[t] += v
    return y[:n_out]


def crossfade_closed_form(x, sets, schedule, L, n_out):
    """y(t) = sum_s sum_r c_s(t - r) (x * h_s^(r))(t) for t in [0, n_out)."""
    x = np.asarray(x, dtype=np.float64)
    w = hann_half_amplitude(L)
    K = len(sets)

    def activity(s, tau):
        # blocks whose window covers tau: l = floor(tau/L) - 1 and floor(tau/L)
        total = 0.0
        base = tau // L
        for l in (base - 1, base):
            n = tau - l * L
            if 0 <= n < 2 * L and _sched(schedule, l) == s:
                total += w[n]
        return total

    y = np.zeros(n_out)
    for s in range(K):
        h = np.asarray(sets[s], dtype=np.float64)
        for r in range(min(2 * L, len(h))):
            hr = np.zeros_like(h)
            hr[r::2 * L] = h[r::2 * L]
            if not np.any(hr):
                continue
            conv = np.convolve(x, hr)[:n_out]
            conv = np.concatenate([conv, np.zeros(n_out - conv.shape[0])])
            c = np.array([activity(s, t - r) for t in range(n_out)])
            y += c * conv
    return y


def naive_dft(a: np.ndarray, sign: int = -1) -> np.ndarray:
    n = a.shape[0]
    out = np.zeros(n, dtype=np.complex128)
    for k in range(n):
        acc = 0j
        for t in range(n):
            acc += a[t] * complex(math.cos(2 * math.pi * t * k / n), sign * math.sin(2 * math.pi * t * k / n))
        out[k] = acc
    return out
