"""Pins of the FP64 oracle against results fixed by the paper and by mathematics.

Each check uses something other than the oracle's own formulas: brute-force
linear convolution, the time-domain block definition, the closed-form cross-fade
between IR sets, hand-worked outputs, an O(n^2) DFT, finite differences. The
planted-mistake tests at the end plant plausible errors in a copy of the
oracle's steps and confirm that some pin fails for each of them.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as orc
import pins_tvolap as pins

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_worked_L2.json")


def rel_rms(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.sqrt(np.sum((a - b) ** 2) / max(np.sum(b ** 2), 1e-300)))


def sets_spectra(sets, L):
    return orc.channel_spectra([np.asarray(s, dtype=np.float64) for s in sets], L)


# ------------------------------------------------------------------ DFT primitive

@pytest.mark.parametrize("n", [8, 16, 32])
def test_rfft_matches_naive_dft(n):
    a = np.random.default_rng(n).standard_normal(n)
    ref = pins.naive_dft(a)[: n // 2 + 1]
    assert np.max(np.abs(np.fft.rfft(a) - ref)) < 1e-12
    spec = np.fft.rfft(a)
    full = np.concatenate([spec, np.conj(spec[1:-1][::-1])])
    back = pins.naive_dft(full, sign=+1).real / n
    assert np.max(np.abs(np.fft.irfft(spec, n) - back)) < 1e-12


# ------------------------------------------------------------------ window

def test_window_values_and_overlap_sum():
    for L in (2, 3, 8, 64, 256):
        w = orc.hann_window(L)
        assert np.allclose(w, pins.hann_half_amplitude(L), atol=1e-15, rtol=0)
        s = w[:L] + w[L:]
        assert np.max(np.abs(s - 1.0)) < 1e-15          # windows at hop L sum to one
    assert np.max(np.abs(orc.hann_window(2) - np.array([0.0, 0.5, 1.0, 0.5]))) < 1e-15


# ------------------------------------------------------------------ time invariant

@pytest.mark.parametrize("L,n_taps,N", [
    (2, 2, 9), (2, 7, 40), (4, 16, 64), (4, 17, 61), (8, 1, 100), (8, 100, 301),
    (16, 32, 257), (16, 500, 700), (64, 300, 1000), (64, 1280, 2500), (128, 4096, 3000),
])
def test_time_invariant_equals_linear_convolution(L, n_taps, N):
    r = np.random.default_rng(L * 1000 + n_taps)
    h = r.standard_normal(n_taps)
    x = r.standard_normal(N)
    y = orc.tvolap_offline(x, sets_spectra([h], L), np.zeros(N // L + 2, int), L)
    ref = np.convolve(x, h)[:N]
    assert rel_rms(y, ref) < 1e-12


def test_streaming_is_offline_delayed_by_hop():
    """Call c emits y[(c-1)L : cL]: a delta IR returns the input L samples later."""
    L, N = 8, 100
    x = np.random.default_rng(3).standard_normal(N)
    n_calls = -(-N // L) + 1
    s = orc.tvolap_stream(x, sets_spectra([[1.0]], L), np.zeros(n_calls, int), L, n_calls)
    assert np.max(np.abs(s[:L])) < 1e-15
    assert np.max(np.abs(s[L: L + N] - x)) < 1e-13


# ------------------------------------------------------------------ time variant

def _random_sets(r, K, n_taps):
    return [r.standard_normal(n_taps) * np.exp(-np.arange(n_taps) / (n_taps / 3)) for _ in range(K)]


@pytest.mark.parametrize("L,K,n_taps,N,p", [
    (2, 2, 9, 50, 0.3), (4, 3, 30, 120, 0.5), (8, 2, 64, 200, 0.2), (8, 4, 50, 160, 1.0),
])
def test_time_variant_equals_block_definition(L, K, n_taps, N, p):
    r = np.random.default_rng(L + 10 * K + n_taps)
    sets = _random_sets(r, K, n_taps)
    x = r.standard_normal(N)
    nb = N // L + 3
    sched = np.zeros(nb, int)
    for b in range(1, nb):
        sched[b] = r.integers(0, K) if r.random() < p else sched[b - 1]
    y = orc.tvolap_offline(x, sets_spectra(sets, L), sched, L)
    ref = pins.block_definition(x, sets, sched, L, N)
    assert rel_rms(y, ref) < 1e-12


@pytest.mark.parametrize("L,K,n_taps,N", [(2, 2, 9, 40), (4, 3, 21, 100), (8, 2, 70, 180)])
def test_time_variant_equals_closed_form_crossfade(L, K, n_taps, N):
    r = np.random.default_rng(7 * L + K)
    sets = _random_sets(r, K, n_taps)
    x = r.standard_normal(N)
    nb = N // L + 3
    sched = r.integers(0, K, size=nb)
    y = orc.tvolap_offline(x, sets_spectra(sets, L), sched, L)
    ref = pins.crossfade_closed_form(x, sets, sched, L, N)
    assert rel_rms(y, ref) < 1e-12


@pytest.mark.parametrize("L,M,ls", [(4, 4, 6), (8, 4, 5), (16, 4, 7)])
def test_fig3_polarity_switch_is_cosine_half_of_length_L(L, M, ls):
    """Sec. 3, Fig. 3: ones convolved with a delta whose polarity flips; with
    M partitions the transition lasts N_IR / (2M) = L samples and follows
    cos(pi u / L) (the 'narrow cosine half')."""
    N = (ls + 4) * L
    h = np.zeros(2 * L * M)
    h[0] = 1.0
    sched = np.array([0 if (b - 1) < ls else 1 for b in range(N // L + 3)])
    y = orc.tvolap_offline(np.ones(N), sets_spectra([h, -h], L), sched, L)
    t = np.arange(N)
    u = t - ls * L
    ref = np.where(u < 0, 1.0, np.where(u >= L, -1.0, np.cos(np.pi * np.clip(u, 0, L) / L)))
    assert np.max(np.abs(y - ref)) < 1e-12


def test_comb_ir_equals_output_crossfade():
    """For IRs whose taps all sit at multiples of 2L, TVOLAP is exactly the
    output-side Hann cross-fade between the two filtered signals."""
    L, M, ls, N = 8, 5, 9, 240
    r = np.random.default_rng(11)
    h = np.zeros(2 * L * M)
    p = np.zeros(2 * L * M)
    h[:: 2 * L] = r.standard_normal(M)
    p[:: 2 * L] = r.standard_normal(M)
    x = r.standard_normal(N)
    sched = np.array([0 if (b - 1) < ls else 1 for b in range(N // L + 3)])
    y = orc.tvolap_offline(x, sets_spectra([h, p], L), sched, L)
    t = np.arange(N)
    u = t - ls * L
    c_old = np.where(u < 0, 1.0, np.where(u >= L, 0.0, 0.5 * (1 + np.cos(np.pi * np.clip(u, 0, L) / L))))
    ref = c_old * np.convolve(x, h)[:N] + (1 - c_old) * np.convolve(x, p)[:N]
    assert rel_rms(y, ref) < 1e-12


# ------------------------------------------------------------------ hand-worked goldens

def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


@pytest.mark.parametrize("name", ["H1_step_switch_to_zero", "H2_tap_in_second_partition",
                                  "H3_impulse_alignment"])
def test_hand_worked_offline(name):
    case = _golden()["cases"][name]
    L = case["L"]
    x = np.array(case["x"], dtype=np.float64)
    sched = list(case["schedule"])
    nb = x.shape[0] // L + 3
    sched = np.array(sched + [sched[-1]] * (nb - len(sched)))
    y = orc.tvolap_offline(x, sets_spectra(case["sets"], L), sched, L)
    want = np.array(case["y"], dtype=np.float64)
    assert np.max(np.abs(y[: want.shape[0]] - want)) < 1e-13


def test_hand_worked_streamed():
    g = _golden()
    st = g["streamed"]["H1_streamed"]
    case = g["cases"][st["case"]]
    L = case["L"]
    s = orc.tvolap_stream(np.array(case["x"], float), sets_spectra(case["sets"], L),
                          np.array(st["slot_per_call"]), L, st["n_calls"])
    assert np.max(np.abs(s - np.array(st["stream"], float))) < 1e-13


# ------------------------------------------------------------------ adjoint

def _loss(x, Hsets, sched, L, target):
    y = orc.tvolap_offline(x, Hsets, sched, L)
    return float(np.mean((y - target) ** 2))


@pytest.mark.parametrize("L,K,n_taps,N", [(4, 1, 20, 60), (8, 2, 40, 120)])
def test_adjoint_matches_central_differences(L, K, n_taps, N):
    """The MSE loss is quadratic in (H, x), so central differences are exact up
    to rounding at any step size."""
    r = np.random.default_rng(100 + L)
    x = r.standard_normal(N)
    H = sets_spectra(_random_sets(r, K, n_taps), L) + 0.1 * (r.standard_normal((K, -(-n_taps // (2 * L)), 2 * L + 1))
                                                            + 1j * r.standard_normal((K, -(-n_taps // (2 * L)), 2 * L + 1)))
    target = r.standard_normal(N)
    sched = r.integers(0, K, size=N // L + 2)
    y = orc.tvolap_offline(x, H, sched, L)
    gy = 2.0 * (y - target) / N
    dH, dx = orc.tvolap_adjoint(x, H, sched, L, gy)
    eps = 1e-3
    checks = []
    M = H.shape[1]
    for (s, m, k) in [(0, 0, 0), (0, 0, 2 * L), (K - 1, M - 1, 1), (0, M // 2, L), (K - 1, 0, 2 * L - 1)]:
        for part in (1.0, 1j):
            Hp = H.copy()
            Hm = H.copy()
            Hp[s, m, k] += eps * part
            Hm[s, m, k] -= eps * part
            fd = (_loss(x, Hp, sched, L, target) - _loss(x, Hm, sched, L, target)) / (2 * eps)
            an = dH[s, m, k].real if part == 1.0 else dH[s, m, k].imag
            checks.append((fd, an))
    for t in [0, 1, L, N // 2, N - 1]:
        xp = x.copy()
        xm = x.copy()
        xp[t] += eps
        xm[t] -= eps
        fd = (_loss(xp, H, sched, L, target) - _loss(xm, H, sched, L, target)) / (2 * eps)
        checks.append((fd, dx[t]))
    scale = max(abs(a) for _, a in checks)
    for fd, an in checks:
        assert abs(fd - an) <= 1e-9 * scale
    # the imaginary parts at k = 0 and k = 2L never reach the output
    assert np.max(np.abs(dH[:, :, 0].imag)) == 0.0
    assert np.max(np.abs(dH[:, :, -1].imag)) == 0.0


# ------------------------------------------------------------------ quantization primitive

def test_quantize_bf16_round_to_nearest_even():
    one = 1.0
    ulp = 2.0 ** -7                                   # bf16 spacing at 1
    vals = np.array([one + ulp / 2, one + 3 * ulp / 2, one + ulp / 2 + 2 ** -20, -(one + ulp / 2),
                     3.0, 1e-3])
    q = orc.quantize(vals, "bf16")
    assert q[0] == 1.0                                # tie -> even mantissa
    assert q[1] == one + 2 * ulp                      # tie -> even mantissa (rounds up)
    assert q[2] == one + ulp                          # above the tie
    assert q[3] == -1.0
    assert q[4] == 3.0
    assert abs(q[5] - 1e-3) <= 1e-3 * 2 ** -8


def test_quantize_f16_matches_ieee_half():
    v = np.array([1.0 + 2 ** -11, 1.0 + 3 * 2 ** -11, 65504.0, 2.0 ** -24])
    q = orc.quantize(v, "f16")
    assert q[0] == 1.0 and q[1] == 1.0 + 2 ** -9 and q[2] == 65504.0 and q[3] == 2.0 ** -24


def test_round_significand_agrees_with_hardware_formats():
    """The pin's own rounding reproduces IEEE conversions where numpy has them
    (float32, float16), including ties, subnormals and the largest half."""
    r = np.random.default_rng(8)
    vals = list(r.standard_normal(200) * 10.0 ** r.integers(-6, 4, size=200))
    vals += [1.0 + 2 ** -11, 1.0 + 3 * 2 ** -11, 65504.0, 2.0 ** -24, 3 * 2.0 ** -25, 2.0 ** -14 * 1.5]
    vals += [1.0 + 2 ** -24, 1.0 + 3 * 2 ** -24, 2.0 ** -149 * 1.5, -(2.0 ** -130) * 1.25]
    for v in vals:
        assert pins.round_significand(v, 11, -14) == float(np.float16(v))
        assert pins.round_significand(v, 24, -126) == float(np.float32(v))


QCASES = [(4, 2, 21, 70, "bf16"), (4, 2, 21, 70, "f16"), (8, 3, 40, 110, "bf16"), (8, 3, 40, 110, "f16")]


def _qcase(L, K, n_taps, N):
    r = np.random.default_rng(1000 + 17 * L + K)
    sets = _random_sets(r, K, n_taps)
    x = r.standard_normal(N)
    n_calls = -(-N // L) + 1
    sched = r.integers(0, K, size=n_calls)
    return sets, x, sched, n_calls


@pytest.mark.parametrize("L,K,n_taps,N,dtype", QCASES)
def test_quantized_streams_match_independent_route(L, K, n_taps, N, dtype):
    """Reduced-precision storage: the oracle (numpy.fft spectra rounded by
    ``quantize``, FP64 MAC) equals the O(n^2) route with its own rounding."""
    sets, x, sched, n_calls = _qcase(L, K, n_taps, N)
    got = orc.quantized_tvolap_streams(x[None, :], [0], [sets_spectra(sets, L)], sched[:, None], L, n_calls,
                                       dtype)[0]
    ref = pins.quantized_stream_naive(x, sets, sched, L, n_calls, dtype)
    assert rel_rms(got, ref) < 1e-12
    # and the rounding is visible: the unrounded stream differs by about one
    # unit of the format
    exact = orc.tvolap_stream(x, sets_spectra(sets, L), sched, L, n_calls)
    assert rel_rms(exact, ref) > {"bf16": 1e-4, "f16": 1e-5}[dtype]


def _quantized_mutant(kind, x, sets, sched, L, n_calls, dtype):
    """A copy of the oracle's reduced-precision steps with one planted mistake."""
    H = sets_spectra(sets, L)
    X = orc.input_spectra(orc.input_blocks(x, L, n_calls), L)
    if kind != "x_unrounded":
        X = orc.quantize(X, dtype)
    if kind != "h_unrounded":
        H = orc.quantize(H, dtype)
    Y = orc.spectral_mac(H, sched, X)
    if kind == "round_y":
        Y = orc.quantize(Y, dtype)
    if kind == "round_y_not_hx":
        Y = orc.quantize(orc.spectral_mac(sets_spectra(sets, L), sched,
                                          orc.input_spectra(orc.input_blocks(x, L, n_calls), L)), dtype)
    return orc.overlap_add(orc.inverse_blocks(Y, L), L, n_calls * L)


@pytest.mark.parametrize("kind", ["x_unrounded", "h_unrounded", "round_y", "round_y_not_hx"])
@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_quantized_pin_rejects_planted_mistakes(kind, dtype):
    L, K, n_taps, N = 4, 2, 21, 70
    sets, x, sched, n_calls = _qcase(L, K, n_taps, N)
    ref = pins.quantized_stream_naive(x, sets, sched, L, n_calls, dtype)
    bad = _quantized_mutant(kind, x, sets, sched, L, n_calls, dtype)
    assert rel_rms(bad, ref) > 1e-9
    good = _quantized_mutant("none", x, sets, sched, L, n_calls, dtype)
    assert rel_rms(good, ref) < 1e-12


# ------------------------------------------------------------------ planted mistakes

class _Mutant:
    """A copy of the oracle's forward steps with one planted mistake."""

    def __init__(self, kind):
        self.kind = kind

    def offline(self, x, Hsets, sched, L):
        x = np.asarray(x, float)
        N = x.shape[0]
        nb = -(-N // L) + 1
        w = orc.hann_window(L)
        if self.kind == "gain2":
            w = 2 * w
        xh = np.zeros((nb, 2 * L))
        for b in range(nb):
            for n in range(2 * L):
                t = (b - 1) * L + n
                if 0 <= t < N:
                    xh[b, n] = x[t] * w[n]
        X = np.fft.rfft(np.concatenate([xh, np.zeros_like(xh)], 1), axis=1)
        M = Hsets.shape[1]
        Y = np.zeros_like(X)
        for b in range(nb):
            for m in range(M):
                if self.kind == "drop_last" and m == M - 1:
                    continue
                step = 1 if self.kind == "consecutive" else 2
                j = b - step * m
                if j < 0:
                    break
                s = sched[b]
                if self.kind == "transposed":
                    s = sched[j]                      # set of the input block's time
                Hm = Hsets[s][m]
                if self.kind == "conj":
                    Hm = np.conj(Hm)
                Y[b] += Hm * X[j]
        y = np.fft.irfft(Y, 4 * L, axis=1)
        out = np.zeros(nb * L + 4 * L)
        for b in range(nb):
            if self.kind == "ola_l1":
                # eq. 10 read literally: right half of block l - 1
                out[b * L: b * L + 2 * L] += y[b, :2 * L]
                if b >= 1:
                    out[b * L: b * L + 2 * L] += y[b - 1, 2 * L:]
            else:
                out[b * L: b * L + 4 * L] += y[b]
        return out[L: L + N]


def _pins_pass(offline):
    """Run a compact set of pins against ``offline``; return True if all pass."""
    ok = True
    r = np.random.default_rng(99)
    L = 4
    h = r.standard_normal(30)
    x = r.standard_normal(80)
    y = offline(x, sets_spectra([h], L), np.zeros(40, int), L)
    ok &= rel_rms(y, np.convolve(x, h)[:80]) < 1e-12
    sets = _random_sets(r, 2, 25)
    sched = r.integers(0, 2, size=40)
    y = offline(x, sets_spectra(sets, L), sched, L)
    ok &= rel_rms(y, pins.block_definition(x, sets, sched, L, 80)) < 1e-12
    case = _golden()["cases"]["H3_impulse_alignment"]
    y = offline(np.array(case["x"], float), sets_spectra(case["sets"], 2), np.zeros(10, int), 2)
    ok &= np.max(np.abs(y - np.array(case["y"]))) < 1e-12
    return bool(ok)


def test_pins_accept_the_oracle():
    assert _pins_pass(orc.tvolap_offline)


@pytest.mark.parametrize("kind", ["gain2", "consecutive", "drop_last", "transposed", "conj", "ola_l1"])
def test_pins_reject_planted_mistakes(kind):
    assert not _pins_pass(_Mutant(kind).offline)
