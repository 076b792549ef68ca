"""FP64 oracle of the paper's comparison algorithms (Jaeger, Simmer, Bitzer,
Blau, arXiv 2310.00319, Sec. 3): block convolution by overlap-add (OLA) and
overlap-save (OLS), weighted overlap-add (WOLA) and two direct time-domain
convolutions cross-faded at the output (CF-TDC).

TEST INFRASTRUCTURE ONLY: imported by tests and by the benchmark's CPU
baseline, never by the GPU library or its binding.

All functions are offline: a whole signal x (zero outside [0, N)) goes in and
y(t) for t in [0, N) comes out, aligned with the input (the block buffering
latency of a streaming implementation is left out). The impulse response
active in a block is chosen per block by a schedule; a switch exchanges the
whole response at a block boundary. numpy.fft is the DFT primitive.

Block grids (B: block length = N_IR, the paper's default for the comparators):
  OLA   block j = 0, 1, ... takes x[jB, (j+1)B), zero pads to 2B, multiplies
        with the 2B-point spectrum of h_{g(j)}, transforms back and adds the
        2B samples at jB. The tail of the last block before a switch is
        computed with the old response.
  OLS   block j = 0, 1, ... transforms x[(j-1)B, (j+1)B) (2B samples), multiplies
        with the 2B-point spectrum of h_{g(j)}, transforms back and keeps the
        last B samples as y[jB, (j+1)B): the samples free of circular wrap.
  WOLA  hop R = B/2; block j = -1, 0, 1, ... takes x[jR, jR + B) weighted by an
        analysis window, zero pads to 2B, filters as OLA does, weights the
        output with a synthesis window and adds it at jR. Windows (periodic,
        length B): "hann" (1 - cos(2 pi n / B)) / 2, "sqrt_hann" sin(pi n / B),
        "rect". A rectangular synthesis keeps all 2B output samples; a
        square-root Hann synthesis weights the first B output samples and drops
        the rest.
  CF-TDC with hop L: the output is sum_s c_s(t) (x * h_s)(t), where the
        activity of response s, c_s(t) = sum over blocks l = -1, 0, ... with
        g(l) = s of w(t - lL), w the Hann window of length 2L (amplitude 1/2),
        is a Hann cross-fade of L samples at every switch. Direct convolution
        of the whole signal with every response, then the cross-fade.

Readings where the paper is silent:
  C-win    The support of WOLA's synthesis window is not stated. A square-root
           Hann synthesis window is applied to the first B output samples of a
           block (aligned with the analysis window); with square-root Hann
           analysis the product of the two windows is the Hann window, whose
           copies at hop B/2 sum to one, so a one-tap response is reproduced
           exactly and longer responses are truncated to B output samples per
           block (the approximation such a WOLA accepts). A rectangular
           synthesis keeps the whole 2B-sample block; with Hann analysis this
           is exact for responses of up to B taps (TVOLAP with one partition).
  C-fade   CF-TDC's cross-fade is the Hann fade of TVOLAP's own blocks (length
           L per switch, on the same block grid), so the two differ only where
           the responses differ tap phase by tap phase (Sec. 3, Fig. 5).
  C-start  Block grids start at t = 0 (OLA, OLS) or t = -B/2 (WOLA, CF-TDC:
           block -1), so every output sample has full window coverage.

Pins (tests/test_comparator_pins.py):
  ols                brute-force linear convolution with the response active
                     in each block
  ola                the time-domain block definition with numpy.convolve; one
                     response: brute-force convolution
  wola               the time-domain block definition with numpy.convolve;
                     Hann/rectangular with one partition equals the TVOLAP
                     oracle; the polarity switch of Fig. 3 in closed form (a
                     cosine half of B/2 samples)
  cf_tdc             equals the TVOLAP oracle for responses whose taps sit at
                     multiples of 2L; differs from it only within 3L samples
                     of a switch for general responses
  op counts          the paper's printed table values
"""
from __future__ import annotations

import numpy as np

__all__ = ["window", "cmp_n_blocks", "ola", "ols", "wola", "cf_tdc", "ops_per_sample"]


def window(kind: str, B: int) -> np.ndarray:
    """Periodic window of length B: rect, hann (amplitude 1/2) or sqrt_hann."""
    n = np.arange(B, dtype=np.float64)
    if kind == "rect":
        return np.ones(B)
    if kind == "hann":
        return 0.5 * (1.0 - np.cos(2.0 * np.pi * n / B))
    if kind == "sqrt_hann":
        return np.sin(np.pi * n / B)
    raise ValueError(kind)


def cmp_n_blocks(method: str, N: int, B: int) -> int:
    """Blocks of a method's grid for N samples (row b of a schedule is block
    b for OLA/OLS and block b - 1 for WOLA)."""
    if method in ("ola", "ols"):
        return -(-N // B)
    if method == "wola":
        return -(-N // (B // 2)) + 1
    raise ValueError(method)


def _seg(x: np.ndarray, t0: int, n: int) -> np.ndarray:
    """x[t0, t0 + n) with zeros outside [0, N)."""
    out = np.zeros(n)
    a, b = max(t0, 0), min(t0 + n, x.shape[0])
    if b > a:
        out[a - t0: b - t0] = x[a:b]
    return out


def _spectrum(h: np.ndarray, F: int) -> np.ndarray:
    h = np.asarray(h, dtype=np.float64)
    if h.shape[0] > F // 2:
        raise ValueError("response longer than the block")
    return np.fft.rfft(h, F)


def ola(x: np.ndarray, irs: list, sched: np.ndarray, B: int) -> np.ndarray:
    """Overlap-add with block B and FFT 2B; sched[j] = response of block j."""
    x = np.asarray(x, dtype=np.float64)
    N = x.shape[0]
    nb = cmp_n_blocks("ola", N, B)
    H = [_spectrum(h, 2 * B) for h in irs]
    y = np.zeros(nb * B + 2 * B)
    for j in range(nb):
        X = np.fft.rfft(_seg(x, j * B, B), 2 * B)
        y[j * B: j * B + 2 * B] += np.fft.irfft(X * H[int(sched[j])], 2 * B)
    return y[:N]


def ols(x: np.ndarray, irs: list, sched: np.ndarray, B: int) -> np.ndarray:
    """Overlap-save with block B and FFT 2B; sched[j] = response of block j."""
    x = np.asarray(x, dtype=np.float64)
    N = x.shape[0]
    nb = cmp_n_blocks("ols", N, B)
    H = [_spectrum(h, 2 * B) for h in irs]
    y = np.zeros(nb * B)
    for j in range(nb):
        X = np.fft.rfft(_seg(x, (j - 1) * B, 2 * B))
        y[j * B: (j + 1) * B] = np.fft.irfft(X * H[int(sched[j])], 2 * B)[B:]
    return y[:N]


def wola(x: np.ndarray, irs: list, sched: np.ndarray, B: int, analysis: str = "sqrt_hann",
         synthesis: str = "sqrt_hann") -> np.ndarray:
    """Weighted overlap-add with block B, hop B/2, FFT 2B; sched[j + 1] =
    response of block j (j = -1, 0, ...)."""
    x = np.asarray(x, dtype=np.float64)
    N = x.shape[0]
    R = B // 2
    nb = cmp_n_blocks("wola", N, B)
    wa = window(analysis, B)
    ws = window(synthesis, B) if synthesis != "rect" else None
    H = [_spectrum(h, 2 * B) for h in irs]
    y = np.zeros((nb + 4) * R + 2 * B)
    for b in range(nb):
        j = b - 1
        X = np.fft.rfft(wa * _seg(x, j * R, B), 2 * B)
        yb = np.fft.irfft(X * H[int(sched[b])], 2 * B)
        t0 = j * R + R          # y is stored from t = -R
        if ws is None:
            y[t0: t0 + 2 * B] += yb
        else:
            y[t0: t0 + B] += ws * yb[:B]
    return y[R: R + N]


def cf_tdc(x: np.ndarray, irs: list, sched: np.ndarray, L: int) -> np.ndarray:
    """Direct convolution with every response and a Hann cross-fade of L
    samples at each switch; sched[l + 1] = response of block l (l = -1, 0, ...),
    ceil(N / L) + 1 rows."""
    x = np.asarray(x, dtype=np.float64)
    N = x.shape[0]
    nb = -(-N // L) + 1
    w = 0.5 * (1.0 - np.cos(2.0 * np.pi * np.arange(2 * L) / (2 * L)))
    act = np.zeros((len(irs), (nb + 2) * L))      # stored from t = -L
    for b in range(nb):
        act[int(sched[b]), b * L: b * L + 2 * L] += w
    y = np.zeros(N)
    for s, h in enumerate(irs):
        if not np.any(act[s, L: L + N]):
            continue
        z = np.convolve(x, np.asarray(h, dtype=np.float64))[:N]
        y += act[s, L: L + N] * z
    return y


def ops_per_sample(method: str, n_ir: int, two_l: int | None = None) -> float:
    """Arithmetic operations per output sample, from the counts of Sec. 3:
    a real FFT of length 2n (decimation in time) costs 5 log2(n) + 14 per
    sample; OLA = forward + inverse + a complex product (6) + an addition;
    WOLA doubles OLA for the 50 % overlap and adds two window products and an
    addition; TVOLAP with blocks 2L and M = N_IR / 2L partitions needs
    20 log2(2L) + 56 for its transforms, 16 M for the products and additions
    and 4 for the window and the overlap-add; direct convolution 2 N_IR."""
    lg = np.log2
    if method == "tdc":
        return 2.0 * n_ir
    if method == "ola":
        return 2 * (5 * lg(n_ir) + 14) + 6 + 1
    if method == "wola":
        return 2 * (2 * (5 * lg(n_ir) + 14) + 6 + 1 + 3)
    if method == "tvolap":
        M = n_ir / two_l
        return 20 * lg(two_l) + 56 + 16 * M + 4
    raise ValueError(method)
