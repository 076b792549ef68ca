"""FP64 oracle for TVOLAP, written from the paper (Jaeger, Simmer, Bitzer, Blau,
"Time-Variant Overlap-Add in Partitions", arXiv 2310.00319, Sec. 2).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the CPU
baseline leg of the benchmark, never by the GPU library or its binding.

Everything is float64 NumPy. The steps follow Sec. 2 in the paper's order:
window the input blocks (eq. 1-2), partition the impulse responses (eq. 3),
zero pad and transform both (eq. 4-7), multiply every second input spectrum
with the partition spectra and sum (eq. 8), transform back (eq. 9) and
overlap-add (eq. 10-13). numpy.fft serves as the DFT primitive; the adjoint
uses explicit DFT matrices instead.

Time axis. The streaming form consumes L new samples per call. Call c (c >= 0)
completes input block l = c - 1, which covers x(t) for t in [(c-1)L, (c+1)L),
and emits y(t) for t in [(c-1)L, cL). Stream outputs are therefore y on the
axis that starts at t = -L; ``tvolap_offline`` returns the part on [0, N).

Readings where the paper is silent, ambiguous or self-inconsistent:
  R-gain   The Hann window of eq. 2 is taken with amplitude 1/2 so that windows
           at hop L sum to one (unity gain, as the paper's M = 1 equivalence
           with Hann-analysis/rectangular-synthesis WOLA and its comparison
           against cross-faded direct convolution require).
  R-part   Eq. 3's partition index: partition m holds taps [2Lm, 2Lm + 2L).
  R-ola    Eq. 10's "preceding" block is the previous block of the same parity
           (l - 2), the only one whose right half is time-aligned with the left
           half of block l; with the literal l - 1 the output is misaligned by L.
  R-start  The input is zero before t = 0 and the delay line starts zeroed;
           the first block is l = -1 (covering [-L, L)).
  R-ragged N_IR that is not a multiple of 2L: M = ceil(N_IR / 2L), last
           partition zero padded; all IR sets of a channel share its M.
  R-switch The IR set active at block l supplies all M partitions of eq. 8 for
           that block (all partitions are exchanged together).
  R-bins   Only the 2L + 1 non-negative-frequency bins are kept; the inverse
           transform takes the Hermitian extension and ignores the imaginary
           parts at k = 0 and k = 2L.

Pins (tests/test_oracle_pins.py; each reaches the result by another road):
  hann_window                        half-angle form sin^2, overlap-sum one
  partition_*/input_*/spectral_mac/
  inverse_blocks/overlap_add/
  tvolap_stream/tvolap_offline       brute-force linear convolution (one IR),
                                     the time-domain block definition and the
                                     closed-form tap-phase cross-fade (any
                                     schedule), the polarity-switch curve of
                                     Sec. 3 (Fig. 3), hand-worked L = 2 goldens
  numpy.fft as the DFT primitive     an O(n^2) DFT loop
  tvolap_adjoint                     central finite differences (the MSE loss
                                     is exactly quadratic)
  quantize                           hand-checked round-to-nearest-even cases
  quantized_tvolap_streams           an independent route: O(n^2) DFTs, a
                                     separately written significand rounding,
                                     the eq. 8 sum as plain loops, an O(n^2)
                                     inverse and a time-domain overlap-add
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "hann_window", "num_partitions", "partition_ir", "partition_spectra",
    "channel_spectra", "input_blocks", "input_spectra", "spectral_mac",
    "inverse_blocks", "overlap_add", "tvolap_stream",
    "tvolap_offline", "tvolap_adjoint", "quantize", "quantized_tvolap_streams",
]


# ---------------------------------------------------------------- windows / partitions

def hann_window(L: int) -> np.ndarray:
    """Periodic Hann window of length 2L (Sec. 2, eq. 2), amplitude 1/2 (R-gain):
    w(n) = (1 - cos(2 pi n / 2L)) / 2 for 0 <= n < 2L."""
    n = np.arange(2 * L, dtype=np.float64)
    return 0.5 * (1.0 - np.cos(2.0 * np.pi * n / (2 * L)))


def num_partitions(n_taps: int, L: int) -> int:
    """M = ceil(N_IR / 2L) (Sec. 3 gives M = N_IR / 2L; R-ragged)."""
    return max(1, -(-int(n_taps) // (2 * L)))


def partition_ir(h: np.ndarray, L: int, M: int) -> np.ndarray:
    """Eq. 3: M non-overlapping rectangular partitions of length 2L (R-part).
    Returns [M][2L]; taps beyond len(h) are zero."""
    h = np.asarray(h, dtype=np.float64)
    if h.shape[0] > 2 * L * M:
        raise ValueError("impulse response longer than M partitions of 2L taps")
    flat = np.zeros(2 * L * M)
    flat[: h.shape[0]] = h
    return flat.reshape(M, 2 * L)


def partition_spectra(h: np.ndarray, L: int, M: int) -> np.ndarray:
    """Eqs. 6-7: partitions zero padded to 4L, then a 4L-point DFT.
    Returns H(k, m) as [M][2L+1] complex128 (k = 0..2L, R-bins)."""
    parts = partition_ir(h, L, M)
    padded = np.concatenate([parts, np.zeros_like(parts)], axis=1)   # eq. 7
    return np.fft.rfft(padded, axis=1)                                 # eq. 6


def channel_spectra(taps_of_slots: list, L: int, n_taps: int | None = None) -> np.ndarray:
    """Spectra of all IR sets (slots) of one channel: [K][M][2L+1], M from the
    channel's IR length ``n_taps`` (default: the longest slot)."""
    if n_taps is None:
        n_taps = max(int(np.asarray(t).shape[0]) for t in taps_of_slots)
    M = num_partitions(n_taps, L)
    return np.stack([partition_spectra(t, L, M) for t in taps_of_slots])


# ---------------------------------------------------------------- input side

def input_blocks(x: np.ndarray, L: int, n_blocks: int) -> np.ndarray:
    """Eq. 1: xhat(n', l) = x(lL + n') w(n'), n' < 2L, for l = -1 .. n_blocks - 2
    (row b holds block l = b - 1). x is zero outside [0, N) (R-start)."""
    x = np.asarray(x, dtype=np.float64)
    N = x.shape[0]
    w = hann_window(L)
    out = np.zeros((n_blocks, 2 * L))
    n = np.arange(2 * L)
    for b in range(n_blocks):
        t = (b - 1) * L + n                      # absolute time of sample n' = n
        ok = (t >= 0) & (t < N)
        out[b, ok] = x[t[ok]] * w[ok]
    return out


def input_spectra(xhat: np.ndarray, L: int) -> np.ndarray:
    """Eqs. 4-5: blocks zero padded to 4L (eq. 5), 4L-point DFT (eq. 4).
    Returns X(k, l) as [n_blocks][2L+1]."""
    padded = np.concatenate([xhat, np.zeros_like(xhat)], axis=1)
    return np.fft.rfft(padded, axis=1)


# ---------------------------------------------------------------- spectral MAC

def spectral_mac(Hsets: np.ndarray, schedule: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Eq. 8 in direct form (R-switch):
        Y(k, l) = sum_{m < M} H_{g(l)}(k, m) X(k, l - 2m),
    with X(., l') = 0 for l' < -1 (R-start). ``Hsets`` is [K][M][2L+1],
    ``schedule[b]`` is the set g(l) of block l = b - 1, X is [n_blocks][2L+1]."""
    n_blocks = X.shape[0]
    M = Hsets.shape[1]
    Y = np.zeros_like(X)
    for b in range(n_blocks):
        H = Hsets[int(schedule[b])]
        for m in range(M):
            j = b - 2 * m
            if j < 0:
                break
            Y[b] += H[m] * X[j]
    return Y


# ---------------------------------------------------------------- output side

def inverse_blocks(Y: np.ndarray, L: int) -> np.ndarray:
    """Eq. 9: y(n', l) = (1/4L) sum_k Y(k, l) e^{+j 2 pi n' k / 4L}, n' < 4L,
    over the Hermitian extension of the 2L + 1 bins (R-bins)."""
    return np.fft.irfft(Y, n=4 * L, axis=1)


def overlap_add(y: np.ndarray, L: int, n_out: int) -> np.ndarray:
    """Eqs. 10-13 with R-ola. Step one: yhat(n', l) = y(n' + 2L, l - 2) + y(n', l)
    for n' < 2L. Step two: out(t) = sum_l yhat(t - lL, l). Rows of ``y`` are
    blocks l = b - 1; the result covers t = -L .. -L + n_out - 1."""
    n_blocks = y.shape[0]
    yhat = np.zeros((n_blocks + 2, 2 * L))     # two more rows take the last right halves
    for b in range(n_blocks + 2):
        if b < n_blocks:
            yhat[b] += y[b, : 2 * L]            # y^CL, eq. 11
        if 0 <= b - 2 < n_blocks:
            yhat[b] += y[b - 2, 2 * L:]         # y^PR, eq. 10 (R-ola)
    out = np.zeros(max(n_out, (n_blocks + 3) * L))
    for b in range(n_blocks + 2):               # eq. 13: block l at t = lL, index b*L
        out[b * L: b * L + 2 * L] += yhat[b]
    return out[:n_out]


# ---------------------------------------------------------------- drivers

def tvolap_stream(x: np.ndarray, Hsets: np.ndarray, schedule: np.ndarray, L: int,
                  n_calls: int) -> np.ndarray:
    """One channel, n_calls streaming calls. Returns the n_calls*L emitted samples,
    i.e. y(t) for t in [-L, (n_calls - 1)L). ``schedule[c]`` is the set used by
    call c (block l = c - 1)."""
    xhat = input_blocks(x, L, n_calls)
    X = input_spectra(xhat, L)
    Y = spectral_mac(np.asarray(Hsets), np.asarray(schedule), X)
    y = inverse_blocks(Y, L)
    # The last block whose output reaches the emitted window is l = n_calls - 2,
    # which is row n_calls - 1; its right half lies beyond the window.
    return overlap_add(y, L, n_calls * L)


def tvolap_offline(x: np.ndarray, Hsets: np.ndarray, schedule: np.ndarray, L: int) -> np.ndarray:
    """One channel, whole signal: y(t) for t in [0, N). ``schedule`` has one
    entry per block l = -1 .. ceil(N/L) - 1 (length ceil(N/L) + 1)."""
    N = int(np.asarray(x).shape[0])
    n_calls = -(-N // L) + 1
    s = tvolap_stream(x, Hsets, schedule, L, n_calls)
    return s[L: L + N]


# ---------------------------------------------------------------- adjoint

def _dft_rows(L: int) -> tuple:
    """Explicit DFT matrices for the adjoint (no FFT library involved):
    E4[n, k] = exp(-j 2 pi n k / 4L) for n < 4L, k <= 2L."""
    n = np.arange(4 * L)[:, None]
    k = np.arange(2 * L + 1)[None, :]
    return np.exp(-2j * np.pi * n * k / (4 * L))


def tvolap_adjoint(x: np.ndarray, Hsets: np.ndarray, schedule: np.ndarray, L: int,
                   gy: np.ndarray) -> tuple:
    """Gradients of a real loss through the offline TVOLAP of one channel.

    ``gy`` is dLoss/dy(t) for t in [0, N). Returns (dH, dx): dH has the shape of
    ``Hsets`` and holds dLoss/dRe H + j dLoss/dIm H for every bin; dx is
    dLoss/dx(t). The steps run the forward steps backwards:
      eq. 10-13  g_l(n') = gy(lL + n'), n' < 4L (each full block lands at lL);
      eq. 9      G_l(k) = (c_k / 4L) sum_n g_l(n) e^{-j 2 pi n k / 4L},
                 c_k = 1 at k = 0, 2L and 2 elsewhere (the Hermitian extension
                 counts interior bins twice; R-bins drops Im at k = 0, 2L);
      eq. 8      dH_s(k, m) = sum_{l: g(l) = s} G_l(k) conj(X(k, l - 2m)),
                 dX(k, j) = sum_m G_{j+2m}(k) conj(H_{g(j+2m)}(k, m));
      eq. 4-5    dxhat_j(n) = sum_{k <= 2L} Re(dX(k, j) e^{+j 2 pi n k / 4L}), n < 2L;
      eq. 1      dx(t) = sum_j w(t - jL) dxhat_j(t - jL).
    """
    x = np.asarray(x, dtype=np.float64)
    Hsets = np.asarray(Hsets)
    N = x.shape[0]
    n_blocks = -(-N // L) + 1
    K, M, B = Hsets.shape
    E4 = _dft_rows(L)                                        # [4L][2L+1]
    ck = np.full(B, 2.0)
    ck[0] = ck[-1] = 1.0

    # forward quantities that the adjoint needs (X only)
    X = input_spectra(input_blocks(x, L, n_blocks), L)

    # eq. 10-13 backwards: gy on the axis starting at -L
    g_axis = np.zeros(n_blocks * L + 4 * L)
    g_axis[L: L + N] = np.asarray(gy, dtype=np.float64)
    g = np.stack([g_axis[b * L: b * L + 4 * L] for b in range(n_blocks)])
    # eq. 9 backwards
    G = (g @ E4) * (ck / (4 * L))
    G[:, 0] = G[:, 0].real
    G[:, -1] = G[:, -1].real
    # eq. 8 backwards
    dH = np.zeros_like(Hsets, dtype=np.complex128)
    dX = np.zeros_like(X)
    for b in range(n_blocks):
        s = int(schedule[b])
        for m in range(M):
            j = b - 2 * m
            if j < 0:
                break
            dH[s, m] += G[b] * np.conj(X[j])
            dX[j] += G[b] * np.conj(Hsets[s, m])
    # eq. 4-5 backwards: only the first 2L (non-padded) samples carry input
    dxhat = (dX @ np.conj(E4[: 2 * L]).T).real               # [n_blocks][2L]
    # eq. 1 backwards
    w = hann_window(L)
    dx = np.zeros(N)
    n = np.arange(2 * L)
    for b in range(n_blocks):
        t = (b - 1) * L + n
        ok = (t >= 0) & (t < N)
        dx[t[ok]] += w[ok] * dxhat[b, ok]
    return dH, dx


# ---------------------------------------------------------------- reduced-precision storage

def quantize(a: np.ndarray, dtype: str) -> np.ndarray:
    """Round every real component to ``dtype`` ("f32", "bf16" or "f16") with
    round-to-nearest-even and return it as float64 / complex128.

    bf16 keeps the top 16 bits of the float32 pattern: the value is first
    rounded to float32 (RNE), then to bf16 (RNE on the dropped 16 bits)."""
    a = np.asarray(a)
    if np.iscomplexobj(a):
        return quantize(a.real, dtype) + 1j * quantize(a.imag, dtype)
    if dtype == "f32":
        return a.astype(np.float32).astype(np.float64)
    if dtype == "f16":
        return a.astype(np.float16).astype(np.float64)
    if dtype == "bf16":
        u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
        lsb = (u >> np.uint64(16)) & np.uint64(1)
        r = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
        return r.astype(np.uint32).view(np.float32).astype(np.float64)
    raise ValueError(dtype)


def quantized_tvolap_streams(x, input_of_channel, Hsets_per_channel, schedule, L, n_calls,
                             dtype: str) -> np.ndarray:
    """Multichannel streaming output [C][n_calls*L] with the stored spectra
    rounded to ``dtype``: channel c filters x[input_of_channel[c]] with its IR
    sets ``Hsets_per_channel[c]`` ([K][M_c][2L+1]) under ``schedule[:, c]``;
    the partition spectra H and the delay-line spectra X are quantized before
    the MAC of eq. 8, which then runs in float64. The transforms stay float64
    (reduced-precision storage with full-precision arithmetic)."""
    C = len(Hsets_per_channel)
    out = np.zeros((C, n_calls * L))
    for c in range(C):
        xin = x[int(input_of_channel[c])]
        X = quantize(input_spectra(input_blocks(xin, L, n_calls), L), dtype)
        H = quantize(np.asarray(Hsets_per_channel[c]), dtype)
        Y = spectral_mac(H, schedule[:, c], X)
        out[c] = overlap_add(inverse_blocks(Y, L), L, n_calls * L)
    return out
