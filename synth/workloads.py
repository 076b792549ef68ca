"""Seeded synthetic multichannel audio workloads.

Every random draw comes from ``numpy.random.default_rng([20231000, cfg, role,
channel, slot])`` so that any array can be regenerated on its own. Signals and
impulse responses are returned as float32 (the precision the GPU path consumes);
the oracle upcasts those same values to float64.

Workload families (shapes follow the paper's use cases: Sec. 3 HRIR switching,
Sec. 4 long binaural room responses, multichannel operation at the end of Sec. 2):

* ``plain``     one channel, white noise, two IRs with a 50 ms exponential decay,
                switched every 50 blocks.
* ``binaural``  S sources x 2 ears, white (even sources) / pink (odd sources)
                noise, K IR slots per ear with RT60 drawn in [0.3, 1.5] s, the
                active slot advancing every block (head tracking).
* ``binaural_fresh`` the same sources with K = 64 response sets per ear and
                block l using set l mod 64: no set recurs within 64 blocks.
* ``uneven``    C channels with their own white-noise input, IR lengths drawn
                log-uniform, two slots per channel, each channel toggling its slot
                with probability 0.1 per block.
* ``autograd``  C channels, white noise, one IR set; a hidden IR gives the target.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_BASE = 20231000
ROLE_INPUT, ROLE_IR, ROLE_SCHED, ROLE_RT60, ROLE_TARGET, ROLE_FD, ROLE_LEN = range(7)

__all__ = [
    "SEED_BASE", "ROLE_INPUT", "ROLE_IR", "ROLE_SCHED", "ROLE_RT60", "ROLE_TARGET",
    "ROLE_FD", "ROLE_LEN", "Workload", "rng", "white_noise", "pink_noise",
    "decaying_ir", "fast_decaying_ir", "n_calls_for", "plain", "binaural", "binaural_fresh", "uneven", "autograd",
    "random_small", "PRESETS",
]


def rng(cfg: int, role: int, channel: int = 0, slot: int = 0) -> np.random.Generator:
    return np.random.default_rng([SEED_BASE, int(cfg), int(role), int(channel), int(slot)])


def white_noise(n: int, r: np.random.Generator) -> np.ndarray:
    return r.standard_normal(n)


def pink_noise(n: int, r: np.random.Generator) -> np.ndarray:
    """White noise shaped by 1/sqrt(f) in the frequency domain, unit RMS."""
    w = r.standard_normal(n)
    spec = np.fft.rfft(w)
    k = np.arange(spec.shape[0], dtype=np.float64)
    scale = np.zeros_like(k)
    scale[1:] = 1.0 / np.sqrt(k[1:])
    p = np.fft.irfft(spec * scale, n)
    return p / np.sqrt(np.mean(p * p))


def decaying_ir(n_taps: int, r: np.random.Generator, fs: float,
                tau: float | None = None, rt60: float | None = None) -> np.ndarray:
    """Gaussian noise under an exponential envelope, normalised to unit L2 norm.

    ``tau``  : envelope exp(-n / (tau*fs)).
    ``rt60`` : envelope 10**(-3 n / (rt60*fs)), i.e. 60 dB of decay after rt60 s.
    """
    n = np.arange(n_taps, dtype=np.float64)
    g = r.standard_normal(n_taps)
    if tau is not None:
        env = np.exp(-n / (tau * fs))
    elif rt60 is not None:
        env = 10.0 ** (-3.0 * n / (rt60 * fs))
    else:
        env = np.ones(n_taps)
    h = g * env
    return h / np.sqrt(np.sum(h * h))


def n_calls_for(n_samples: int, hop: int) -> int:
    """Streaming calls that consume ``n_samples`` plus one flush call of zeros.

    Call c consumes x[cL:(c+1)L] and emits y[(c-1)L:cL], so one extra call is
    needed before the last L input samples appear at the output.
    """
    return -(-n_samples // hop) + 1


@dataclasses.dataclass
class Workload:
    name: str
    cfg: int
    hop: int                       # L (hop size; blocks and partitions are 2L long)
    fs: int
    x: np.ndarray                  # [I][N] float32 input signals
    input_of_channel: np.ndarray   # [C] int32
    taps: list                     # taps[c][s]: float32 IR of channel c in slot s
    taps_of_channel: np.ndarray    # [C] int32 IR length per channel (all slots)
    n_slots: int
    schedule: np.ndarray           # [n_calls][C] int32 slot used by stream call c
    target: np.ndarray | None = None  # [C][N] float32 (autograd family only)
    hidden_taps: list | None = None   # [C] hidden IRs that produced the target

    @property
    def n_channels(self) -> int:
        return int(self.input_of_channel.shape[0])

    @property
    def n_inputs(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_samples(self) -> int:
        return int(self.x.shape[1])

    @property
    def n_calls(self) -> int:
        return int(self.schedule.shape[0])

    def padded_input(self) -> np.ndarray:
        """[I][n_calls*L] float32: the input followed by zeros for the flush call."""
        out = np.zeros((self.n_inputs, self.n_calls * self.hop), dtype=np.float32)
        out[:, : self.n_samples] = self.x
        return out

    def max_taps(self) -> int:
        return int(self.taps_of_channel.max())


def _f32(a: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


def plain(n_samples: int = 480_000, hop: int = 128, n_taps: int = 4096, fs: int = 48_000,
          switch_every: int = 50, cfg: int = 1) -> Workload:
    x = _f32(white_noise(n_samples, rng(cfg, ROLE_INPUT, 0))[None, :])
    taps = [[_f32(decaying_ir(n_taps, rng(cfg, ROLE_IR, 0, s), fs, tau=0.05)) for s in range(2)]]
    n_calls = n_calls_for(n_samples, hop)
    sched = ((np.arange(n_calls) // switch_every) % 2).astype(np.int32)[:, None]
    return Workload("plain", cfg, hop, fs, x, np.zeros(1, np.int32), taps,
                    np.array([n_taps], np.int32), 2, sched)


def binaural(n_sources: int = 64, n_samples: int = 240_000, hop: int = 256,
             n_taps: int = 96_000, n_slots: int = 4, fs: int = 48_000, cfg: int = 2) -> Workload:
    xs = []
    for s in range(n_sources):
        r = rng(cfg, ROLE_INPUT, s)
        xs.append(white_noise(n_samples, r) if s % 2 == 0 else pink_noise(n_samples, r))
    x = _f32(np.stack(xs))
    C = 2 * n_sources
    inp = (np.arange(C) // 2).astype(np.int32)
    taps = []
    for c in range(C):
        row = []
        for k in range(n_slots):
            rt60 = rng(cfg, ROLE_RT60, c, k).uniform(0.3, 1.5)
            row.append(_f32(decaying_ir(n_taps, rng(cfg, ROLE_IR, c, k), fs, rt60=rt60)))
        taps.append(row)
    n_calls = n_calls_for(n_samples, hop)
    sched = np.repeat((np.arange(n_calls) % n_slots).astype(np.int32)[:, None], C, axis=1)
    return Workload("binaural", cfg, hop, fs, x, inp, taps,
                    np.full(C, n_taps, np.int32), n_slots, sched)


def fast_decaying_ir(n_taps: int, r: np.random.Generator, fs: float, rt60: float) -> np.ndarray:
    """float32 Gaussian noise under 10**(-3 n / (rt60 fs)), unit L2 norm: the
    recipe of ``decaying_ir`` drawn in float32, for banks of thousands of
    responses."""
    n = np.arange(n_taps, dtype=np.float32)
    g = r.standard_normal(n_taps, dtype=np.float32)
    h = g * np.exp(n * np.float32(-3.0 * math.log(10.0) / (rt60 * fs)), dtype=np.float32)
    return (h / np.float32(np.sqrt(np.sum(h.astype(np.float64) ** 2)))).astype(np.float32)


def binaural_fresh(n_sources: int = 64, n_samples: int = 240_000, hop: int = 256, n_taps: int = 96_000,
                   n_slots: int = 64, fs: int = 48_000, cfg: int = 6, base: Workload | None = None) -> Workload:
    """Head tracking with a new response set at every block: the binaural
    sources and ears, K = n_slots response sets per ear (RT60 drawn in
    [0.3, 1.5] s per set) and block l using set l mod K for every channel, so
    within K consecutive blocks no set repeats. ``base``: a ``binaural``
    workload of the same sources whose input signals are reused."""
    if base is None:
        base = binaural(n_sources=n_sources, n_samples=n_samples, hop=hop, n_taps=16, n_slots=1, fs=fs)
    from concurrent.futures import ThreadPoolExecutor

    C = 2 * n_sources

    def ear(c):
        return [fast_decaying_ir(n_taps, rng(cfg, ROLE_IR, c, k), fs, rng(cfg, ROLE_RT60, c, k).uniform(0.3, 1.5))
                for k in range(n_slots)]

    with ThreadPoolExecutor(8) as ex:
        taps = list(ex.map(ear, range(C)))
    n_calls = n_calls_for(n_samples, hop)
    sched = np.repeat((np.arange(n_calls) % n_slots).astype(np.int32)[:, None], C, axis=1)
    return Workload("binaural_fresh", cfg, hop, fs, base.x, base.input_of_channel, taps,
                    np.full(C, n_taps, np.int32), n_slots, sched)


def uneven(n_channels: int = 512, n_samples: int = 96_000, hop: int = 128,
           min_taps: int = 4800, max_taps: int = 192_000, p_switch: float = 0.1,
           fs: int = 48_000, cfg: int = 3) -> Workload:
    x = _f32(np.stack([white_noise(n_samples, rng(cfg, ROLE_INPUT, c)) for c in range(n_channels)]))
    lens = np.array([int(round(math.exp(rng(cfg, ROLE_LEN, c).uniform(math.log(min_taps),
                                                                     math.log(max_taps)))))
                     for c in range(n_channels)], dtype=np.int32)
    taps = []
    for c in range(n_channels):
        row = []
        for k in range(2):
            rt60 = rng(cfg, ROLE_RT60, c, k).uniform(0.3, 1.5)
            row.append(_f32(decaying_ir(int(lens[c]), rng(cfg, ROLE_IR, c, k), fs, rt60=rt60)))
        taps.append(row)
    n_calls = n_calls_for(n_samples, hop)
    sched = np.zeros((n_calls, n_channels), np.int32)
    for c in range(n_channels):
        toggles = rng(cfg, ROLE_SCHED, c).random(n_calls) < p_switch
        sched[:, c] = np.cumsum(toggles) % 2
    return Workload("uneven", cfg, hop, fs, x, np.arange(n_channels, dtype=np.int32), taps,
                    lens, 2, sched)


def autograd(n_channels: int = 32, n_samples: int = 96_000, hop: int = 256, n_taps: int = 8192,
             fs: int = 48_000, cfg: int = 5) -> Workload:
    """Time-invariant family with a target signal made by a hidden IR per channel."""
    from scipy.signal import oaconvolve

    x = _f32(np.stack([white_noise(n_samples, rng(cfg, ROLE_INPUT, c)) for c in range(n_channels)]))
    taps = [[_f32(decaying_ir(n_taps, rng(cfg, ROLE_IR, c, 0), fs, rt60=0.5))]
            for c in range(n_channels)]
    hidden = [_f32(decaying_ir(n_taps, rng(cfg, ROLE_TARGET, c), fs, rt60=0.3))
              for c in range(n_channels)]
    target = _f32(np.stack([oaconvolve(x[c].astype(np.float64), hidden[c].astype(np.float64))[:n_samples]
                            for c in range(n_channels)]))
    n_calls = n_calls_for(n_samples, hop)
    sched = np.zeros((n_calls, n_channels), np.int32)
    return Workload("autograd", cfg, hop, fs, x, np.arange(n_channels, dtype=np.int32), taps,
                    np.full(n_channels, n_taps, np.int32), 1, sched, target=target,
                    hidden_taps=hidden)


def random_small(seed: int, hop: int, n_channels: int, n_inputs: int, n_samples: int,
                 taps_range: tuple, n_slots: int, p_switch: float = 0.3, cfg: int = 90) -> Workload:
    """Small mixed workload for parity tests: ragged IR lengths, shared inputs,
    random slot switches. ``seed`` is folded into the cfg field of the seed."""
    c0 = cfg * 1000 + seed
    x = _f32(np.stack([white_noise(n_samples, rng(c0, ROLE_INPUT, i)) for i in range(n_inputs)]))
    inp = (np.arange(n_channels) % n_inputs).astype(np.int32)
    lo, hi = taps_range
    lens = np.array([int(rng(c0, ROLE_LEN, c).integers(lo, hi + 1)) for c in range(n_channels)],
                    dtype=np.int32)
    taps = [[_f32(decaying_ir(int(lens[c]), rng(c0, ROLE_IR, c, k), 48_000, rt60=0.05))
             for k in range(n_slots)] for c in range(n_channels)]
    n_calls = n_calls_for(n_samples, hop)
    sched = np.zeros((n_calls, n_channels), np.int32)
    for c in range(n_channels):
        r = rng(c0, ROLE_SCHED, c)
        cur = 0
        for t in range(n_calls):
            if r.random() < p_switch:
                cur = int(r.integers(0, n_slots))
            sched[t, c] = cur
    return Workload("random_small", c0, hop, 48_000, x, inp, taps, lens, n_slots, sched)


# Full-size workloads, one per benchmark configuration.
PRESETS = {
    "plain": dict(fn=plain, kwargs={}),
    "binaural": dict(fn=binaural, kwargs={}),
    "uneven": dict(fn=uneven, kwargs={}),
    "binaural_bf16": dict(fn=binaural, kwargs={}),
    "autograd": dict(fn=autograd, kwargs={}),
}
