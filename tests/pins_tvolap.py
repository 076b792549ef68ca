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
* ``quantized_stream_naive``: reduced-precision storage (spectra rounded to
  bf16/f16 before eq. 8) through O(n^2) DFTs and a significand rounding
  written from the format definitions (``round_significand``).
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


# ------------------------------------------------------------------ reduced-precision storage

# (significand bits, smallest normal exponent) of the storage formats
_FORMATS = {"f32": (24, -126), "bf16": (8, -126), "f16": (11, -14)}


def round_significand(v: float, bits: int, emin: int) -> float:
    """v rounded to ``bits`` significant bits, ties to even, with gradual
    underflow below 2**emin. Written with frexp and exact power-of-two
    scaling; no float32/float16 casts and no bit patterns."""
    if v == 0.0 or not math.isfinite(v):
        return v
    _, e = math.frexp(v)                    # |v| in [2**(e-1), 2**e)
    q = 2.0 ** (max(e - 1, emin) - (bits - 1))   # spacing of the format at v
    r = v / q                               # exact: q is a power of two
    n = math.floor(r)
    frac = r - n
    if frac > 0.5 or (frac == 0.5 and n % 2 == 1):
        n += 1
    return n * q


def store_round(v: complex, dtype: str) -> complex:
    """Storage rounding of one complex value, component-wise: bf16 goes through
    float32 first (the value is a float32 before it is stored), f16 and f32
    round the float64 value once."""
    def one(a):
        if dtype == "bf16":
            return round_significand(round_significand(a, *_FORMATS["f32"]), *_FORMATS["bf16"])
        return round_significand(a, *_FORMATS[dtype])
    return complex(one(v.real), one(v.imag))


def quantized_stream_naive(x, sets, schedule, L, n_calls, dtype):
    """Streaming output of one channel (n_calls * L samples on the axis that
    starts at t = -L) with stored spectra rounded to ``dtype``: input blocks
    and partitions transformed by an O(n^2) DFT, both rounded, the eq. 8 sum
    over partitions as plain loops, an O(n^2) inverse over the Hermitian
    extension and the 4L-sample outputs added at hop L."""
    x = np.asarray(x, dtype=np.float64)
    N = x.shape[0]
    w = hann_half_amplitude(L)
    n_taps = max(len(s) for s in sets)
    M = max(1, -(-n_taps // (2 * L)))
    B = 2 * L + 1

    def spectrum(seg2L):
        padded = np.concatenate([np.asarray(seg2L, dtype=np.float64), np.zeros(2 * L)])
        return naive_dft(padded)[:B]

    def rnd(v):
        return np.array([store_round(complex(z), dtype) for z in v])

    H = []
    for s in sets:
        flat = np.zeros(2 * L * M)
        flat[: len(s)] = s
        H.append([rnd(spectrum(flat[2 * L * m: 2 * L * (m + 1)])) for m in range(M)])
    X = []
    for b in range(n_calls):                       # block l = b - 1
        seg = np.zeros(2 * L)
        for n in range(2 * L):
            t = (b - 1) * L + n
            if 0 <= t < N:
                seg[n] = x[t] * w[n]
        X.append(rnd(spectrum(seg)))
    out = np.zeros(n_calls * L + 4 * L)
    for b in range(n_calls):
        Y = np.zeros(B, dtype=np.complex128)
        s = int(schedule[b])
        for m in range(M):
            j = b - 2 * m
            if j < 0:
                break
            for k in range(B):
                Y[k] += H[s][m][k] * X[j][k]
        for n in range(4 * L):                     # real inverse, 1/4L
            acc = Y[0].real + Y[B - 1].real * (-1.0) ** n
            for k in range(1, B - 1):
                a = 2.0 * math.pi * n * k / (4 * L)
                acc += 2.0 * (Y[k].real * math.cos(a) - Y[k].imag * math.sin(a))
            out[b * L + n] += acc / (4 * L)
    return out[: n_calls * L]
