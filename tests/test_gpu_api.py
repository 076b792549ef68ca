"""GPU tests of the C ABI's failure semantics and of state the API promises
to keep: a rejected call leaves the handle's stream exactly as it was, an
oversized handle fails with ENOMEM and leaves the device usable, a NaN in one
input stays in its own channels and is gone after a reset, and the batched
autotuner keeps the caller's slot selection."""
import ctypes

import numpy as np
import pytest

import synth
from gpu_common import gpu_streams, log, make_convolver, oracle_streams, rel_rms_per_channel

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


def _wl():
    return synth.random_small(seed=61, hop=128, n_channels=6, n_inputs=3, n_samples=128 * 30 + 5,
                              taps_range=(300, 4000), n_slots=3, p_switch=0.5)


def test_rejected_calls_leave_the_stream_unchanged():
    """Every handle-level EINVAL (bad channel, slot or length in set_ir and
    set_irs, a slot out of range in select_ir, n_blocks above max_batch, NULL
    buffers, short strides) issued in the middle of a stream: the outputs stay
    bitwise equal to those of an untouched handle."""
    import torch
    log("EINVAL mid-stream leaves state unchanged")
    wl = _wl()
    ref = gpu_streams(wl, batch=4).astype(np.float32)
    conv = make_convolver(wl)
    lib, h = conv._lib, conv._h
    L, C = wl.hop, wl.n_channels
    x = torch.from_numpy(wl.padded_input()).cuda()
    sched = torch.from_numpy(np.ascontiguousarray(wl.schedule, dtype=np.int32)).cuda()
    out = torch.zeros((C, wl.n_calls * L), device="cuda")
    taps = np.ones(50, np.float32)
    tp = taps.ctypes.data_as(ctypes.c_void_p)
    dev_taps = torch.ones((C, 64), device="cuda")
    bad = np.full(C, 0, np.int32)
    bad[2] = wl.n_slots
    neg = np.full(C, -1, np.int32)
    c = 0
    while c < wl.n_calls:
        n = min(4, wl.n_calls - c)
        if c == 8:
            assert lib.tvolap_set_ir(h, C, 0, tp, 50, 0) == -1                  # channel out of range
            assert lib.tvolap_set_ir(h, -1, 0, tp, 50, 0) == -1
            assert lib.tvolap_set_ir(h, 0, wl.n_slots, tp, 50, 0) == -1         # slot out of range
            assert lib.tvolap_set_ir(h, 0, 0, tp, int(wl.taps_of_channel[0]) + 1, 0) == -1   # too many taps
            assert lib.tvolap_set_ir(h, 0, 0, None, 5, 0) == -1                 # NULL taps
            assert lib.tvolap_set_irs(h, wl.n_slots, ctypes.c_void_p(dev_taps.data_ptr()), 64) == -1
            assert lib.tvolap_set_irs(h, 0, ctypes.c_void_p(dev_taps.data_ptr()), 0) == -1
            assert lib.tvolap_select_ir(h, bad.ctypes.data_as(ctypes.c_void_p)) == -1
            assert lib.tvolap_select_ir(h, neg.ctypes.data_as(ctypes.c_void_p)) == -1
            assert lib.tvolap_process_blocks(h, x.data_ptr(), x.stride(0), conv.max_batch + 1, out.data_ptr(),
                                             out.stride(0), sched.data_ptr(), C) == -1
            assert lib.tvolap_process_blocks(h, x.data_ptr(), x.stride(0), 0, out.data_ptr(), out.stride(0),
                                             sched.data_ptr(), C) == -1
            assert lib.tvolap_process_blocks(h, None, x.stride(0), 2, out.data_ptr(), out.stride(0), None, 0) == -1
            assert lib.tvolap_process_blocks(h, x.data_ptr(), x.stride(0), 2, out.data_ptr(), out.stride(0),
                                             sched.data_ptr(), C - 1) == -1
            assert lib.tvolap_process_block(h, x.data_ptr(), L - 1, out.data_ptr(), out.stride(0), None) == -1
            assert lib.tvolap_process_block(h, x.data_ptr(), x.stride(0), None, out.stride(0), None) == -1
            assert lib.tvolap_configure(h, 3, 0, 0, 0) == -1
            assert lib.tvolap_configure_batch(h, 0, 3, 0, 0, 0, 0) == -1
            msg = lib.tvolap_last_error(h)
            assert msg and msg != b"no error"
        rc = lib.tvolap_process_blocks(h, x.data_ptr() + 4 * L * c, x.stride(0), n, out.data_ptr() + 4 * L * c,
                                       out.stride(0), sched.data_ptr() + 4 * C * c, C)
        assert rc == 0
        c += n
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    conv.close()
    assert np.array_equal(got, ref)


def test_oversized_create_is_enomem_and_device_stays_usable():
    """An IR bank far beyond the device's memory fails with ENOMEM (no handle)
    and the next normal handle works."""
    from paper_2310_00319_amd._lib import TvolapConfig
    import paper_2310_00319_amd as pkg
    log("oversized create")
    lib = pkg.load()
    cfg = TvolapConfig()
    cfg.hop = 256
    cfg.n_channels = 4096
    cfg.n_inputs = 4096
    cfg.max_taps = 2_000_000      # 3907 partitions
    cfg.n_slots = 16
    cfg.spectra_dtype = 0
    cfg.max_batch = 16
    hh = ctypes.c_void_p()
    rc = lib.tvolap_create(ctypes.byref(cfg), ctypes.byref(hh))   # 1 TB of partition spectra
    assert rc == -2, (rc, lib.tvolap_last_error(None))
    assert not hh.value
    wl = _wl()
    got = gpu_streams(wl)
    assert rel_rms_per_channel(got, oracle_streams(wl)).max() <= TOL_F32


@pytest.mark.parametrize("batch", [1, 8])
def test_nan_in_one_input_stays_in_its_channels_and_clears_on_reset(batch):
    import torch
    log(f"NaN isolation, batch {batch}")
    wl = _wl()   # 6 channels on 3 inputs (channel c reads input c mod 3)
    clean = gpu_streams(wl, batch=batch).astype(np.float32)
    conv = make_convolver(wl)
    L = wl.hop
    xp = wl.padded_input().copy()
    xp[1, 10 * L + 7] = np.nan
    x = torch.from_numpy(xp).cuda()
    sched = torch.from_numpy(np.ascontiguousarray(wl.schedule, dtype=np.int32)).cuda()
    got = conv.process(x, sched, batch=batch).cpu().numpy()
    hit = [c for c in range(wl.n_channels) if wl.input_of_channel[c] == 1]
    rest = [c for c in range(wl.n_channels) if c not in hit]
    assert np.array_equal(got[rest], clean[rest])
    for c in hit:
        assert np.all(np.isfinite(got[c, : 10 * L]))          # before the NaN arrives: unchanged
        assert np.array_equal(got[c, : 10 * L], clean[c, : 10 * L])
        assert np.isnan(got[c, 12 * L:]).any()
    conv.reset()
    x = torch.from_numpy(wl.padded_input()).cuda()
    again = conv.process(x, sched, batch=batch).cpu().numpy()
    conv.close()
    assert np.array_equal(again, clean)


def test_batched_autotune_keeps_the_selection():
    """select_ir(s), then the batched autotuner (which times calls with its own
    per-block slots), then calls with no device schedule: they run slot s."""
    import torch
    import oracle as orc
    log("autotune_batch keeps the selection")
    # a shape no other test tunes, so the tuner really runs
    wl = synth.random_small(seed=62, hop=64, n_channels=5, n_inputs=5, n_samples=64 * 40 + 3,
                            taps_range=(700, 2900), n_slots=3, p_switch=0.0)
    conv = make_convolver(wl, max_batch=32)
    sel = np.full(wl.n_channels, 2, np.int32)
    conv.select_ir(sel)
    best = conv.autotune_batch(iters=1)
    assert best > 0, "the tuner took its choice from the cache; pick another shape"
    L = wl.hop
    x = torch.from_numpy(wl.padded_input()).cuda()
    out = conv.process(x, None, batch=8).cpu().numpy().astype(np.float64)
    conv.close()
    xs = wl.padded_input().astype(np.float64)
    for c in range(wl.n_channels):
        H = orc.channel_spectra([t.astype(np.float64) for t in wl.taps[c]], L, int(wl.taps_of_channel[c]))
        ref = orc.tvolap_stream(xs[c], H, np.full(wl.n_calls, 2), L, wl.n_calls)
        assert rel_rms_per_channel(out[c], ref) <= TOL_F32
