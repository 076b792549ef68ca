"""CPU pins of the comparison-algorithm oracle (Sec. 3: OLA, OLS, WOLA,
CF-TDC) against results fixed by other roads: brute-force linear convolution,
the time-domain block definitions written with numpy.convolve, closed forms of
the polarity switch of Fig. 3, the TVOLAP oracle (M = 1 equivalence, comb
responses), and the operation counts of Tables 1 and 2."""
import numpy as np
import pytest

import oracle as orc
from oracle import comparators_ref as cmp

TIGHT = 1e-12


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def _irs(r, K, n):
    return [r.standard_normal(n) * np.exp(-np.arange(n) / (n / 4)) for _ in range(K)]


@pytest.mark.parametrize("B,N_IR", [(8, 8), (16, 11), (32, 32), (64, 40)])
def test_ols_is_convolution_with_the_active_response(B, N_IR):
    r = np.random.default_rng(B)
    N = B * 9 + 5
    x = r.standard_normal(N)
    irs = _irs(r, 3, N_IR)
    sched = r.integers(0, 3, size=cmp.cmp_n_blocks("ols", N, B))
    y = cmp.ols(x, irs, sched, B)
    full = [np.convolve(x, h)[:N] for h in irs]
    ref = np.array([full[sched[t // B]][t] for t in range(N)])
    assert rel(y, ref) <= TIGHT


@pytest.mark.parametrize("B,N_IR", [(8, 8), (16, 13), (64, 64)])
def test_ola_block_definition_and_time_invariance(B, N_IR):
    r = np.random.default_rng(100 + B)
    N = B * 7 + 3
    x = r.standard_normal(N)
    irs = _irs(r, 2, N_IR)
    sched = r.integers(0, 2, size=cmp.cmp_n_blocks("ola", N, B))
    y = cmp.ola(x, irs, sched, B)
    ref = np.zeros(N + 3 * B)
    for j in range(len(sched)):
        xj = x[j * B: (j + 1) * B]
        ref[j * B: j * B + len(xj) + N_IR - 1] += np.convolve(xj, irs[sched[j]])
    assert rel(y, ref[:N]) <= TIGHT
    y1 = cmp.ola(x, irs[:1], np.zeros_like(sched), B)
    assert rel(y1, np.convolve(x, irs[0])[:N]) <= TIGHT


@pytest.mark.parametrize("analysis,synthesis", [("sqrt_hann", "sqrt_hann"), ("hann", "rect"), ("sqrt_hann", "rect")])
def test_wola_block_definition(analysis, synthesis):
    B, N_IR = 16, 12
    R = B // 2
    r = np.random.default_rng(7)
    N = B * 6 + 5
    x = r.standard_normal(N)
    irs = _irs(r, 3, N_IR)
    sched = r.integers(0, 3, size=cmp.cmp_n_blocks("wola", N, B))
    y = cmp.wola(x, irs, sched, B, analysis, synthesis)
    n = np.arange(B)
    wa = {"hann": 0.5 - 0.5 * np.cos(2 * np.pi * n / B), "sqrt_hann": np.sin(np.pi * n / B)}[analysis]
    ref = np.zeros(N + 6 * B)
    off = R
    for b in range(len(sched)):
        j = b - 1
        xj = np.array([x[t] if 0 <= t < N else 0.0 for t in range(j * R, j * R + B)])
        z = np.convolve(wa * xj, irs[sched[b]])
        if synthesis == "rect":
            ref[off + j * R: off + j * R + len(z)] += z
        else:
            ref[off + j * R: off + j * R + B] += np.sin(np.pi * n / B) * z[:B]
    assert rel(y, ref[off: off + N]) <= TIGHT


def test_wola_hann_rect_time_invariant_is_convolution():
    B = 32
    r = np.random.default_rng(8)
    x = r.standard_normal(B * 10)
    h = r.standard_normal(B)
    y = cmp.wola(x, [h], np.zeros(cmp.cmp_n_blocks("wola", x.size, B), int), B, "hann", "rect")
    assert rel(y, np.convolve(x, h)[: x.size]) <= TIGHT


@pytest.mark.parametrize("L", [4, 16, 64])
def test_tvolap_one_partition_is_wola_hann_analysis_rect_synthesis(L):
    """Sec. 3: with one partition TVOLAP is WOLA with a Hann analysis and a
    rectangular synthesis window (block 2L, hop L)."""
    r = np.random.default_rng(L)
    N = L * 21 + 3
    x = r.standard_normal(N)
    irs = [r.standard_normal(2 * L) for _ in range(3)]
    nb = -(-N // L) + 1
    sched = r.integers(0, 3, size=nb)
    H = np.stack([orc.partition_spectra(h, L, 1) for h in irs])
    y_tv = orc.tvolap_offline(x, H, sched, L)
    y_w = cmp.wola(x, irs, sched, 2 * L, "hann", "rect")
    assert rel(y_w, y_tv) <= TIGHT


@pytest.mark.parametrize("method", ["ola", "ols"])
def test_fig3_polarity_switch_is_abrupt_for_ola_and_ols(method):
    B = 32
    N = B * 8
    js = 4
    x = np.ones(N)
    d = np.zeros(B)
    d[0] = 1.0
    sched = (np.arange(cmp.cmp_n_blocks(method, N, B)) >= js).astype(int)
    y = getattr(cmp, method)(x, [d, -d], sched, B)
    ref = np.where(np.arange(N) < js * B, 1.0, -1.0)
    assert np.max(np.abs(y - ref)) <= 1e-12


def test_fig3_polarity_switch_wola_is_a_cosine_half_of_half_the_block():
    """WOLA with square-root Hann windows, x = 1, response +delta, then -delta
    from block j_s on (blocks start every R = B/2 samples): the output is +1
    before j_s R, -1 from j_s R + R on, and cos(pi (t - j_s R) / R) in between,
    where the last old block's Hann weight falls while the first new one's
    rises: a cosine half of N_IR / 2 samples (Sec. 3, Fig. 3)."""
    B = 64
    R = B // 2
    N = B * 8
    x = np.ones(N)
    d = np.zeros(B)
    d[0] = 1.0
    nb = cmp.cmp_n_blocks("wola", N, B)
    js = 6                                   # schedule row js + 1 is block js
    sched = (np.arange(nb) - 1 >= js).astype(int)
    y = cmp.wola(x, [d, -d], sched, B, "sqrt_hann", "sqrt_hann")
    t = np.arange(N)
    f0 = js * R
    ref = np.where(t < f0, 1.0, np.where(t >= f0 + R, -1.0, np.cos(np.pi * (t - f0) / R)))
    assert np.max(np.abs(y - ref)) <= 1e-12


@pytest.mark.parametrize("L", [4, 8, 32])
def test_cf_tdc_equals_tvolap_for_comb_responses(L):
    """Responses with taps only at multiples of 2L: TVOLAP is exactly the
    output-side Hann cross-fade of the two filtered signals (CF-TDC)."""
    r = np.random.default_rng(300 + L)
    N = L * 30 + 1
    x = r.standard_normal(N)
    M = 5
    irs = []
    for _ in range(3):
        h = np.zeros(2 * L * M)
        h[:: 2 * L] = r.standard_normal(M)
        irs.append(h)
    nb = -(-N // L) + 1
    sched = r.integers(0, 3, size=nb)
    H = np.stack([orc.partition_spectra(h, L, M) for h in irs])
    assert rel(cmp.cf_tdc(x, irs, sched, L), orc.tvolap_offline(x, H, sched, L)) <= 1e-12


def test_cf_tdc_differs_from_tvolap_only_near_a_switch():
    """General responses, one switch at block l_s: TVOLAP and CF-TDC agree
    exactly outside [l_s L, l_s L + 3L) (the tap-phase cross-fade of TVOLAP
    ends 2L - 1 samples after the output fade), and differ inside (Fig. 5)."""
    L, M = 16, 3
    r = np.random.default_rng(5)
    N = L * 40
    x = r.standard_normal(N)
    irs = [r.standard_normal(2 * L * M) for _ in range(2)]
    nb = -(-N // L) + 1
    ls = 17
    sched = (np.arange(nb) - 1 >= ls).astype(int)
    H = np.stack([orc.partition_spectra(h, L, M) for h in irs])
    d = np.abs(orc.tvolap_offline(x, H, sched, L) - cmp.cf_tdc(x, irs, sched, L))
    t = np.arange(N)
    inside = (t >= ls * L) & (t < ls * L + 3 * L)
    assert d[~inside].max() <= 1e-12
    assert d[inside].max() > 1e-3


def test_operation_counts_match_tables_1_and_2():
    """MFLOPS at 48 kHz from the per-sample counts of Sec. 3 against Tables 1
    and 2. Two printed entries disagree with the paper's own formulas (WOLA at
    N_IR = 2048 prints (2 * 145 + 3) fs; TVOLAP at N_IR = 512 prints WOLA's
    count less its synthesis window): the formulas are kept, the printed values
    are checked as those products."""
    fs = 48000
    mf = lambda ops: round(ops * fs / 1e6, 3)
    assert mf(cmp.ops_per_sample("tdc", 2048)) == 196.608
    assert mf(cmp.ops_per_sample("ola", 2048)) == 6.96
    assert mf(cmp.ops_per_sample("tvolap", 2048, 512)) == 14.592
    assert mf(cmp.ops_per_sample("wola", 2048)) == 14.208
    assert mf(2 * 145 + 3) == 14.064                      # the printed WOLA value
    assert mf(cmp.ops_per_sample("tdc", 512)) == 49.152
    assert mf(cmp.ops_per_sample("ola", 512)) == 6.0
    assert mf(cmp.ops_per_sample("wola", 512)) == 12.288
    assert mf(cmp.ops_per_sample("tvolap", 512, 512)) == 12.288
    assert mf(cmp.ops_per_sample("wola", 512) - 2) == 12.192   # the printed TVOLAP value
