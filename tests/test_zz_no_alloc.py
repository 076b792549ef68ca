"""GPU test of the allocation-free offline forward (tvolap_offline_forward_noalloc).

It must give what tvolap_offline_forward gives with a caller workspace, bit for
bit, on two calls in a row (the second with a smaller input, so the static
scratch holds the first call's data when the second starts), and match the
FP64 oracle within 1e-5 relative RMS per channel. The first shape needs several
segments of the 32 MiB scratch; a shape too large for it is refused with EINVAL.
"""
import ctypes

import numpy as np
import pytest

import oracle as orc
from gpu_common import log

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2310_00319_amd as pkg
    pkg.load()
    yield


def _inputs(seed, L, C, K, M, N):
    r = np.random.default_rng(seed)
    x = r.standard_normal((C, N)).astype(np.float32)
    nb = -(-N // L) + 1
    sched = r.integers(0, K, size=(nb, C)).astype(np.int32)
    H = (r.standard_normal((C, K, M, 2 * L + 1)) + 1j * r.standard_normal((C, K, M, 2 * L + 1)))
    H *= np.exp(-np.arange(M) / 4.0)[None, None, :, None]
    return x, H.astype(np.complex64), sched


def _shape(L, C, K, M, N):
    from paper_2310_00319_amd._lib import TvolapOfflineShape
    s = TvolapOfflineShape()
    s.hop, s.n_channels, s.n_slots, s.n_partitions, s.n_samples = L, C, K, M, N
    return s


def _run_both(lib, L, C, K, M, N, seed):
    import torch
    x, H, sched = _inputs(seed, L, C, K, M, N)
    xd = torch.from_numpy(x).cuda()
    Hd = torch.from_numpy(H).cuda()
    sd = torch.from_numpy(sched).cuda()
    s = _shape(L, C, K, M, N)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    y0 = torch.full_like(xd, float("nan"))
    y1 = torch.full_like(xd, float("nan"))
    ws_bytes = lib.tvolap_offline_workspace_bytes(ctypes.byref(s))
    ws = torch.empty(int(ws_bytes), dtype=torch.uint8, device="cuda")
    rc = lib.tvolap_offline_forward(ctypes.byref(s), ctypes.c_void_p(xd.data_ptr()), ctypes.c_void_p(Hd.data_ptr()),
                                    ctypes.c_void_p(sd.data_ptr()), ctypes.c_void_p(y0.data_ptr()),
                                    ctypes.c_void_p(ws.data_ptr()), ws.numel(), st)
    assert rc == 0, lib.tvolap_offline_last_error()
    rc = lib.tvolap_offline_forward_noalloc(ctypes.byref(s), ctypes.c_void_p(xd.data_ptr()),
                                            ctypes.c_void_p(Hd.data_ptr()), ctypes.c_void_p(sd.data_ptr()),
                                            ctypes.c_void_p(y1.data_ptr()), st)
    assert rc == 0, lib.tvolap_offline_last_error()
    torch.cuda.synchronize()
    return x, H, sched, y0.cpu().numpy(), y1.cpu().numpy()


def _check_oracle(x, H, sched, y, L, chans):
    for c in chans:
        ref = orc.tvolap_offline(x[c].astype(np.float64), H[c].astype(np.complex128), sched[:, c], L)
        err = float(np.linalg.norm(y[c] - ref) / np.linalg.norm(ref))
        assert err <= TOL, f"channel {c}: rel-RMS {err:.3e}"


def test_noalloc_forward_two_calls_match_workspace_forward():
    import paper_2310_00319_amd as pkg
    lib = pkg.load()
    # call 1: 32 channels, L = 256, 16 partitions, 2 s: four segments of the scratch
    L, C, K, M, N = 256, 32, 2, 16, 96000
    log(f"noalloc call 1: L={L} C={C} K={K} M={M} N={N}")
    x, H, sched, y0, y1 = _run_both(lib, L, C, K, M, N, seed=11)
    assert np.array_equal(y0, y1), f"max |diff| {np.max(np.abs(y0 - y1)):.3e}"
    _check_oracle(x, H, sched, y1, L, [0, 13, 31])
    # call 2: a smaller shape, one segment, on the same scratch
    L, C, K, M, N = 128, 3, 2, 5, 128 * 40 + 17
    log(f"noalloc call 2: L={L} C={C} K={K} M={M} N={N}")
    x, H, sched, y0, y1 = _run_both(lib, L, C, K, M, N, seed=12)
    assert np.array_equal(y0, y1), f"max |diff| {np.max(np.abs(y0 - y1)):.3e}"
    _check_oracle(x, H, sched, y1, L, range(C))


def test_noalloc_forward_refuses_shape_beyond_scratch():
    import paper_2310_00319_amd as pkg
    lib = pkg.load()
    # C (2M + 8) 16 L = 64 * 520 * 16 * 512 bytes > 32 MiB
    s = _shape(512, 64, 1, 256, 100000)
    dummy = ctypes.c_void_p(16)
    rc = lib.tvolap_offline_forward_noalloc(ctypes.byref(s), dummy, dummy, None, dummy, None)
    assert rc == -1
    assert b"static scratch" in lib.tvolap_offline_last_error()
