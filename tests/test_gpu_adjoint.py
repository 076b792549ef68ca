"""GPU parity of the offline (differentiable) form and its adjoint.

Bars: forward within 1e-5 relative RMS of the FP64 oracle per channel;
gradients (dH, dx) within 1e-5 relative RMS of the oracle's FP64 adjoint per
channel; finite differences of the FP64 oracle loss (exact for the quadratic
MSE loss) agree with the GPU gradient within 1e-4 of the gradient's largest
entry on every checked coordinate.
"""
import numpy as np
import pytest

import oracle as orc
import synth
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


def rel(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _case(seed, L, C, K, M, N, random_H=False):
    r = np.random.default_rng(seed)
    x = r.standard_normal((C, N)).astype(np.float32)
    nb = -(-N // L) + 1
    sched = r.integers(0, K, size=(nb, C)).astype(np.int32)
    H = np.zeros((C, K, M, 2 * L + 1), np.complex64)
    for c in range(C):
        for s in range(K):
            taps = (r.standard_normal(2 * L * M) * np.exp(-np.arange(2 * L * M) / (L * M))).astype(np.float32)
            H[c, s] = orc.partition_spectra(taps.astype(np.float64), L, M).astype(np.complex64)
    if random_H:
        H = H + (0.05 * (r.standard_normal(H.shape) + 1j * r.standard_normal(H.shape))).astype(np.complex64)
    return x, H, sched


CASES = [
    (1, 64, 3, 1, 3, 64 * 20 + 7),
    (2, 128, 2, 2, 5, 128 * 15),
    (3, 256, 2, 3, 4, 256 * 9 + 100),
    (4, 512, 1, 2, 2, 512 * 8 + 1),
    # signals longer than one segment of the workspace forms (1024 hops): the
    # backward runs in segments, the input spectra of the 2(M - 1) blocks
    # before each recomputed and dH summed over the segments
    (5, 64, 2, 2, 4, 64 * 2100 + 33),
    (6, 128, 1, 3, 40, 128 * 1100),
]


@pytest.mark.parametrize("case", CASES, ids=[f"L{c[1]}_K{c[3]}_M{c[4]}_N{c[5]}" for c in CASES])
def test_offline_forward_and_adjoint_match_oracle(case):
    import torch
    from paper_2310_00319_amd import functional as F
    seed, L, C, K, M, N = case
    log(f"offline case {case}")
    x, H, sched = _case(seed, L, C, K, M, N, random_H=True)
    xt = torch.from_numpy(x).cuda().requires_grad_(True)
    Ht = torch.from_numpy(H).cuda().requires_grad_(True)
    st = torch.from_numpy(sched).cuda()
    y = F.tvolap(xt, Ht, L, st)
    r = np.random.default_rng(seed + 100)
    gy = r.standard_normal((C, N)).astype(np.float32)
    y.backward(torch.from_numpy(gy).cuda())
    y_g = y.detach().cpu().numpy()
    dx_g = xt.grad.cpu().numpy()
    dH_g = Ht.grad.cpu().numpy()
    for c in range(C):
        Hc = H[c].astype(np.complex128)
        ref = orc.tvolap_offline(x[c].astype(np.float64), Hc, sched[:, c], L)
        assert rel(y_g[c], ref) <= TOL, ("forward", c, rel(y_g[c], ref))
        dH_ref, dx_ref = orc.tvolap_adjoint(x[c].astype(np.float64), Hc, sched[:, c], L, gy[c].astype(np.float64))
        e_h, e_x = rel(dH_g[c], dH_ref), rel(dx_g[c], dx_ref)
        log(f"  channel {c}: forward {rel(y_g[c], ref):.2e} dH {e_h:.2e} dx {e_x:.2e}")
        assert e_h <= TOL and e_x <= TOL
        assert np.all(dH_g[c][..., 0].imag == 0) and np.all(dH_g[c][..., -1].imag == 0)


def test_offline_equals_streaming_without_delay():
    import torch
    from paper_2310_00319_amd import Convolver
    from paper_2310_00319_amd import functional as F
    log("offline vs streaming")
    L, C, n_taps, N = 128, 3, 1500, 128 * 12 + 33
    wl = synth.random_small(seed=41, hop=L, n_channels=C, n_inputs=C, n_samples=N,
                            taps_range=(n_taps, n_taps), n_slots=2, p_switch=0.5)
    conv = Convolver(hop=L, n_channels=C, max_taps=n_taps, n_slots=2)
    for c in range(C):
        for s in range(2):
            conv.set_ir(c, s, wl.taps[c][s])
    x = torch.from_numpy(wl.padded_input()).cuda()
    sched = torch.from_numpy(wl.schedule.astype(np.int32)).cuda()
    stream = conv.process(x, sched).cpu().numpy()
    conv.close()
    taps = torch.from_numpy(np.stack([np.stack(wl.taps[c]) for c in range(C)])).cuda().contiguous()
    H = F.ir_spectra(taps, L)
    nb = F.n_blocks(N, L)
    y = F.tvolap(torch.from_numpy(wl.x).cuda(), H, L, sched[:nb].contiguous()).cpu().numpy()
    assert rel(y, stream[:, L: L + N]) <= 2e-6


def test_ir_spectra_matches_oracle():
    import torch
    from paper_2310_00319_amd import functional as F
    log("ir spectra")
    r = np.random.default_rng(5)
    for L, M, n in [(64, 3, 300), (256, 4, 2048), (512, 2, 1025)]:
        taps = r.standard_normal((2, 2, n)).astype(np.float32)
        H = F.ir_spectra(torch.from_numpy(taps).cuda(), L, M).cpu().numpy()
        for c in range(2):
            for s in range(2):
                ref = orc.partition_spectra(taps[c, s].astype(np.float64), L, M)
                assert rel(H[c, s], ref) <= 1e-6


def test_gpu_finite_differences_smoke():
    """FP32 central differences of the GPU loss (quadratic, so exact up to
    rounding) against the GPU gradient, to 1e-2."""
    import torch
    from paper_2310_00319_amd import functional as F
    log("gpu finite differences")
    L, C, K, M, N = 64, 2, 1, 4, 64 * 12
    x, H, sched = _case(9, L, C, K, M, N)
    r = np.random.default_rng(10)
    target = torch.from_numpy(r.standard_normal((C, N)).astype(np.float32)).cuda()
    xt = torch.from_numpy(x).cuda().requires_grad_(True)
    Ht = torch.from_numpy(H).cuda().requires_grad_(True)

    def loss(xv, Hv):
        return torch.mean((F.tvolap(xv, Hv, L) - target) ** 2)

    loss(xt, Ht).backward()
    gx, gH = xt.grad.double().cpu().numpy(), Ht.grad.cpu().numpy()
    scale = max(np.abs(gx).max(), np.abs(gH).max())
    with torch.no_grad():
        for (c, t) in [(0, 5), (1, 300), (0, N - 1)]:
            e = 0.05
            xp, xm = xt.detach().clone(), xt.detach().clone()
            xp[c, t] += e
            xm[c, t] -= e
            fd = (loss(xp, Ht).item() - loss(xm, Ht).item()) / (2 * e)
            assert abs(fd - gx[c, t]) <= 1e-2 * scale
        for (c, s, m, k, part) in [(0, 0, 0, 3, 1), (1, 0, 2, 40, 1j), (0, 0, 1, 0, 1)]:
            e = 0.05
            Hp, Hm = Ht.detach().clone(), Ht.detach().clone()
            Hp[c, s, m, k] += e * part
            Hm[c, s, m, k] -= e * part
            fd = (loss(xt, Hp).item() - loss(xt, Hm).item()) / (2 * e)
            an = gH[c, s, m, k].real if part == 1 else gH[c, s, m, k].imag
            assert abs(fd - an) <= 1e-2 * scale


def test_full_autograd_workload_against_fp64_gradient_and_fd():
    """32 channels, L=256, 8192-tap IRs (16 partitions), 96000 samples, MSE
    against a target made by hidden IRs. GPU gradients vs the FP64 oracle
    adjoint on sampled channels, and 64 finite-difference coordinates of the
    FP64 oracle loss (32 on H including Im at DC and Nyquist, 32 on x)."""
    import torch
    from paper_2310_00319_amd import functional as F
    log("full autograd workload")
    wl = synth.autograd()
    C, N, L = wl.n_channels, wl.n_samples, wl.hop
    taps = torch.from_numpy(np.stack([wl.taps[c][0] for c in range(C)])[:, None, :].copy()).cuda()
    H = F.ir_spectra(taps, L)
    M = H.shape[2]
    xt = torch.from_numpy(wl.x).cuda().requires_grad_(True)
    Ht = H.clone().requires_grad_(True)
    target = torch.from_numpy(wl.target).cuda()
    y = F.tvolap(xt, Ht, L)
    loss = torch.mean((y - target) ** 2)
    loss.backward()
    gx = xt.grad.cpu().numpy().astype(np.float64)
    gH = Ht.grad.cpu().numpy().astype(np.complex128)
    Hn = H.cpu().numpy().astype(np.complex128)
    y_g = y.detach().cpu().numpy()
    sched = np.zeros(F.n_blocks(N, L), int)
    x64 = wl.x.astype(np.float64)
    t64 = wl.target.astype(np.float64)
    for c in (0, 17, 31):
        ref_y = orc.tvolap_offline(x64[c], Hn[c], sched, L)
        assert rel(y_g[c], ref_y) <= TOL
        gy = 2.0 * (ref_y - t64[c]) / (C * N)
        dH_ref, dx_ref = orc.tvolap_adjoint(x64[c], Hn[c], sched, L, gy)
        log(f"  channel {c}: dH {rel(gH[c], dH_ref):.2e} dx {rel(gx[c], dx_ref):.2e}")
        assert rel(gH[c], dH_ref) <= TOL and rel(gx[c], dx_ref) <= TOL
    # finite differences of the FP64 loss, one channel at a time (the loss is a
    # sum over channels, so the other channels cancel in the difference)
    r = synth.rng(5, synth.ROLE_FD)
    gmax = max(np.abs(gx).max(), np.abs(gH).max())
    eps = 1e-3

    def chan_loss(c, xc, Hc):
        yv = orc.tvolap_offline(xc, Hc, sched, L)
        return float(np.sum((yv - t64[c]) ** 2) / (C * N))

    coords_h = [(int(r.integers(C)), 0, int(r.integers(M)), int(r.integers(1, 2 * L)), [1, 1j][i % 2])
                for i in range(30)]
    coords_h += [(3, 0, 0, 0, 1j), (4, 0, M - 1, 2 * L, 1j)]          # Im at DC / Nyquist: gradient 0
    for (c, s, m, k, part) in coords_h:
        Hp, Hm = Hn[c].copy(), Hn[c].copy()
        Hp[s, m, k] += eps * part
        Hm[s, m, k] -= eps * part
        fd = (chan_loss(c, x64[c], Hp) - chan_loss(c, x64[c], Hm)) / (2 * eps)
        an = gH[c, s, m, k].real if part == 1 else gH[c, s, m, k].imag
        assert abs(fd - an) <= 1e-4 * gmax, ("H", c, s, m, k, part, fd, an)
    for i in range(32):
        c, t = int(r.integers(C)), int(r.integers(N))
        xp, xm = x64[c].copy(), x64[c].copy()
        xp[t] += eps
        xm[t] -= eps
        fd = (chan_loss(c, xp, Hn[c]) - chan_loss(c, xm, Hn[c])) / (2 * eps)
        assert abs(fd - gx[c, t]) <= 1e-4 * gmax, ("x", c, t, fd, gx[c, t])
