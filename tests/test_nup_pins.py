"""CPU pins of the non-uniform-partition oracle (head of short partitions,
tail of long ones): brute-force convolution for one response; with r = 1 the
split reproduces uniform TVOLAP for any schedule; the time-domain block
definition of each part (numpy.convolve only); the stream is causal in its
inputs and selections when M1 >= r - 1."""
import numpy as np
import pytest

import oracle as orc
from oracle import nup_ref
from pins_tvolap import block_definition

TIGHT = 1e-12


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("L1,M1,r,n_taps", [(2, 1, 1, 7), (4, 3, 4, 200), (8, 2, 2, 150), (4, 7, 8, 333),
                                            (16, 3, 4, 1000)])
def test_time_invariant_is_convolution(L1, M1, r, n_taps):
    rng = np.random.default_rng(L1 * 100 + r)
    n_calls = 60
    x = rng.standard_normal(n_calls * L1)
    h = rng.standard_normal(n_taps)
    y = nup_ref.nup_stream(x, [h], np.zeros(n_calls, int), L1, M1, r, n_taps, n_calls)
    ref = np.concatenate([np.zeros(L1), np.convolve(x, h)])[: n_calls * L1]
    assert rel(y, ref) <= TIGHT


@pytest.mark.parametrize("L1,M1,n_taps", [(4, 2, 60), (8, 3, 130)])
def test_one_level_is_uniform_tvolap(L1, M1, n_taps):
    """r = 1: head and tail are the first M1 and the remaining partitions of
    the uniform split at hop L1, the tail's set is the call's set: the result
    is uniform TVOLAP."""
    rng = np.random.default_rng(L1)
    n_calls = 50
    x = rng.standard_normal(n_calls * L1)
    sets = [rng.standard_normal(n_taps) for _ in range(3)]
    sched = rng.integers(0, 3, size=n_calls)
    y = nup_ref.nup_stream(x, sets, sched, L1, M1, 1, n_taps, n_calls)
    H = orc.channel_spectra(sets, L1, n_taps)
    assert rel(y, orc.tvolap_stream(x, H, sched, L1, n_calls)) <= TIGHT


def test_parts_follow_the_time_domain_block_definition():
    """Head at hop L1 (first D taps, the call's sets) plus tail at hop L2 (taps
    from D on, the set of head call r (c2 - 1) + 2 M1 + 1), delayed by D, each
    from numpy.convolve block sums."""
    L1, M1, r, n_taps = 4, 4, 4, 170
    L2, D = r * L1, 2 * L1 * M1
    rng = np.random.default_rng(9)
    n_calls = 64
    x = rng.standard_normal(n_calls * L1)
    sets = [rng.standard_normal(n_taps) for _ in range(3)]
    sched = rng.integers(0, 3, size=n_calls)
    y = nup_ref.nup_stream(x, sets, sched, L1, M1, r, n_taps, n_calls)
    n_out = (n_calls - 1) * L1
    head = block_definition(x, [s[:D] for s in sets], sched, L1, n_out + L1)
    n2 = n_calls // r + 2
    t_sched = nup_ref.nup_tail_schedule(sched, r, M1, n2)
    tail = block_definition(x, [s[D:] for s in sets], t_sched, L2, n_out + L1)
    ytil = head.copy()
    ytil[D:] += tail[: ytil.shape[0] - D]
    assert rel(y[L1:], ytil[:n_out]) <= TIGHT


def test_stream_is_causal():
    """Output of call c depends on inputs up to (c + 1) L1 and selections up to
    call c only (M1 = r - 1, the shortest head allowed)."""
    L1, r = 4, 4
    M1 = r - 1
    n_taps = 300
    rng = np.random.default_rng(3)
    n_calls = 80
    x = rng.standard_normal(n_calls * L1)
    sets = [rng.standard_normal(n_taps) for _ in range(2)]
    sched = rng.integers(0, 2, size=n_calls)
    y = nup_ref.nup_stream(x, sets, sched, L1, M1, r, n_taps, n_calls)
    for c in (13, 31, 50):
        x2 = x.copy()
        x2[(c + 1) * L1:] = rng.standard_normal(x2[(c + 1) * L1:].shape)
        s2 = sched.copy()
        s2[c + 1:] = 1 - s2[c + 1:]
        y2 = nup_ref.nup_stream(x2, sets, s2, L1, M1, r, n_taps, n_calls)
        assert np.array_equal(y[: (c + 1) * L1], y2[: (c + 1) * L1])
