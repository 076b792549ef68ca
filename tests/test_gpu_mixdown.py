"""GPU parity of the output mixdown: bus e is the sum of the outputs of the
channels mapped to it (linearity of eqs. 8-13 over channels; the library adds
the channels' spectra of a bus before one inverse transform). Reference: the
sum of the FP64 oracle streams of the bus's channels, same 1e-5 relative-RMS
bar per bus as per channel.
"""
import dataclasses

import numpy as np
import pytest

import synth
from gpu_common import gpu_streams, gpu_streams_graph, log, make_convolver, oracle_bus_streams, rel_rms_per_channel

pytestmark = pytest.mark.gpu

TOL_F32 = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2310_00319_amd as pkg
    pkg.load()
    yield


def _buses(C: int, E: int, seed: int) -> np.ndarray:
    """A seeded channel -> bus map in which every bus has a channel."""
    b = np.random.default_rng(seed).integers(0, E, C).astype(np.int32)
    b[np.random.default_rng(seed + 1).permutation(C)[:E]] = np.arange(E, dtype=np.int32)
    return b


MIX_CASES = [
    # seed, L, C, I, N, taps range, K, p_switch, buses
    (11, 64, 5, 5, 64 * 40 + 5, (1, 2000), 2, 0.3, 2),
    (12, 128, 6, 3, 128 * 30 + 77, (300, 5000), 3, 0.5, 3),
    (13, 256, 8, 4, 256 * 20 + 1, (512, 6000), 2, 1.0, 1),     # every channel into one bus
    (14, 512, 3, 3, 512 * 16, (1024, 9000), 2, 0.2, 3),        # one channel per bus, permuted
    (15, 64, 13, 4, 64 * 50, (50, 3000), 4, 0.4, 4),           # fan-out 4, ragged M
]


def _wl(case):
    seed, L, C, I, N, tr, K, p, E = case
    wl = synth.random_small(seed=seed, hop=L, n_channels=C, n_inputs=I, n_samples=N,
                            taps_range=tr, n_slots=K, p_switch=p)
    return wl, _buses(C, E, seed)


@pytest.mark.parametrize("batch", [1, 5, 16])
@pytest.mark.parametrize("case", MIX_CASES, ids=[f"s{c[0]}_L{c[1]}_E{c[8]}" for c in MIX_CASES])
def test_mixdown_matches_sum_of_channel_oracles(case, batch):
    wl, buses = _wl(case)
    log(f"mixdown case {case} batch {batch} buses {buses.tolist()}")
    got = gpu_streams(wl, batch=batch, buses=buses)
    ref = oracle_bus_streams(wl, buses)
    assert got.shape == ref.shape
    err = rel_rms_per_channel(got, ref)
    log(f"mixdown: max rel-RMS {err.max():.3e} over {len(err)} buses")
    assert np.all(np.isfinite(got)) and err.max() <= TOL_F32


def test_mixdown_batched_equals_single_and_sum_of_channels():
    """Batched and single-block calls agree to FP32 rounding, and each bus is
    the sum of the per-channel outputs of a run without a mixdown."""
    wl, buses = _wl(MIX_CASES[4])
    log("mixdown batched vs single vs per-channel sum")
    single = gpu_streams(wl, buses=buses)
    batched = gpu_streams(wl, batch=16, buses=buses)
    per = gpu_streams(wl, batch=16)
    summed = np.zeros_like(single)
    for c in range(wl.n_channels):
        summed[buses[c]] += per[c]
    assert rel_rms_per_channel(batched, single).max() <= 1e-6
    assert rel_rms_per_channel(batched, summed).max() <= 1e-6


def test_mixdown_configuration_rules():
    """A mixdown runs the separate transform-out launch: fused modes are
    refused, autotuning keeps fused = 0, and outputs have one row per bus."""
    import torch
    wl, buses = _wl(MIX_CASES[1])
    log("mixdown configuration rules")
    conv = make_convolver(wl, buses=buses)
    assert conv.n_outputs == 3 and conv.info()["n_outputs"] == 3
    with pytest.raises(Exception, match="fused"):
        conv.configure(fused=1)
    conv.autotune(iters=2)
    assert conv.info()["fused"] == 0
    conv.autotune_batch(iters=1)
    x = torch.zeros((wl.n_inputs, wl.hop), device="cuda")
    with pytest.raises(ValueError):
        conv.process_block(x, torch.zeros((wl.n_channels, wl.hop), device="cuda"))
    conv.reset()
    got = gpu_streams(wl, conv=conv, batch=7)
    conv.close()
    assert rel_rms_per_channel(got, oracle_bus_streams(wl, buses)).max() <= TOL_F32


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_mixdown_reduced_precision(dtype):
    wl, buses = _wl(MIX_CASES[4])
    log(f"mixdown {dtype}")
    got = gpu_streams(wl, dtype, batch=16, buses=buses)
    err_q = rel_rms_per_channel(got, oracle_bus_streams(wl, buses, dtype=dtype))
    assert err_q.max() <= 2e-4


@pytest.mark.parametrize("batch", [1, 16])
def test_mixdown_graph_replay(batch):
    wl, buses = _wl(MIX_CASES[1])
    log(f"mixdown graph batch {batch}")
    got = gpu_streams_graph(wl, batch=batch, buses=buses)
    assert rel_rms_per_channel(got, oracle_bus_streams(wl, buses)).max() <= TOL_F32


def test_full_binaural_mixdown_bench_configuration():
    """The benchmark's mixdown: 128 channels into the two ear buses (c mod 2),
    64-block calls from a graph. The first 192 blocks of each ear are checked
    against the oracle of all 128 channels (outputs up to a block depend only
    on the input up to it); the whole stream against the per-channel path."""
    log("full binaural, ear mixdown, 64-block calls from a graph")
    wl = synth.binaural()
    buses = (np.arange(wl.n_channels) % 2).astype(np.int32)
    got = gpu_streams_graph(wl, batch=64, buses=buses)
    n = 192
    L = wl.hop
    head = dataclasses.replace(wl, x=wl.x[:, : n * L], schedule=wl.schedule[:n])
    ref = oracle_bus_streams(head, buses)
    err = rel_rms_per_channel(got[:, : n * L], ref)
    log(f"binaural mixdown: max rel-RMS {err.max():.3e} over the first {n} blocks")
    assert err.max() <= TOL_F32
    per = gpu_streams_graph(wl, batch=64)
    summed = np.stack([per[0::2].sum(axis=0), per[1::2].sum(axis=0)])
    err2 = rel_rms_per_channel(got, summed)
    log(f"binaural mixdown vs per-channel sum: max rel-RMS {err2.max():.3e}")
    assert err2.max() <= 1e-6
