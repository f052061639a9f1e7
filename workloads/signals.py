"""Seeded synthetic signals for the downsampled SST workloads.

Every generator works in float64 with ``numpy.random.default_rng`` streams,
evaluates phases as cycles reduced modulo 1 before multiplying by 2*pi, and
returns the signal rounded to float32.  That float32 array is the single input
fed both to the GPU library and to the float64 CPU oracle.

Each workload also carries its noise-free components (for the output SNR of
Eq. 33) and their closed-form instantaneous frequencies (used to build the
reconstruction zones of Sec. 2.2, Eq. 15 and Sec. 2.3, Eq. 26 as caller-supplied
ridges).

Sigma and window lengths are in samples throughout.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np

TWO_PI = 2.0 * math.pi


@dataclass
class SSTConfig:
    """Transform parameters in the paper's terms (Sec. 2.1, 2.2, 2.4)."""

    fs: float
    win_len: int          # L = 2M + 1 window taps
    sigma: float          # Gaussian width in samples
    hop: int              # H_t
    nfft: int             # N_f
    f_lo: float           # band of interest [f1, f2] in Hz
    f_hi: float
    subdiv: int           # frequency subdivision factor z
    thr_mode: str = "rel"  # "rel": gamma = thr * max|S| ; "abs": gamma = thr
    thr: float = 1e-3
    hw: int = 0           # half-width of the reconstruction zone, destination bins

    @property
    def delta_f(self) -> float:
        return self.fs / self.nfft


@dataclass
class Workload:
    name: str
    x: np.ndarray                      # float32 [N]
    comps: np.ndarray                  # float64 [n_comp, N] noise-free components
    inst_freq: Callable[[np.ndarray], np.ndarray]  # t (s) -> [n_comp, len(t)] Hz
    cfg: SSTConfig
    seed: int
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_frames(self) -> int:
        return -(-self.n // self.cfg.hop)

    def frame_times(self) -> np.ndarray:
        return np.arange(self.n_frames, dtype=np.float64) * self.cfg.hop / self.cfg.fs


def _cos_cycles(cycles: np.ndarray) -> np.ndarray:
    """cos(2*pi*cycles) with the integer part of the cycle count removed first."""
    frac = cycles - np.floor(cycles)
    return np.cos(TWO_PI * frac)


def _white_noise_for(clean: np.ndarray, snr_db: float, rng: np.random.Generator) -> np.ndarray:
    p = float(np.mean(clean * clean))
    return rng.standard_normal(clean.shape[0]) * math.sqrt(p / 10.0 ** (snr_db / 10.0))


def _pink_noise_for(clean: np.ndarray, snr_db: float, rng: np.random.Generator) -> np.ndarray:
    n = clean.shape[0]
    white = rng.standard_normal(n)
    spec = np.fft.rfft(white)
    f = np.arange(spec.shape[0], dtype=np.float64)
    f[0] = 1.0
    spec *= f ** -0.5
    spec[0] = 0.0
    pink = np.fft.irfft(spec, n)
    del spec, white
    p_clean = float(np.mean(clean * clean))
    p_pink = float(np.mean(pink * pink))
    return pink * math.sqrt(p_clean / 10.0 ** (snr_db / 10.0) / p_pink)


def ridge_bins(inst_freq_hz: np.ndarray, fs: float, nfft: int, k1: int, subdiv: int,
               n_dst: int) -> np.ndarray:
    """Destination-bin index nearest to each true IF value (caller-supplied ridge).

    The destination grid is f*_l = (k1 + l/z) * fs/N_f (Eqs. 28-29 with the band
    snapped to source bins).  Frequencies that fall outside the grid map to -1
    ("no ridge in this frame").
    """
    df = fs / nfft
    l = np.floor(subdiv * (np.asarray(inst_freq_hz, dtype=np.float64) / df - k1) + 0.5)
    out = l.astype(np.int64)
    out[(out < 0) | (out >= n_dst)] = -1
    return out.astype(np.int32)


# ---------------------------------------------------------------------------
# Workload c1: plain standard SST, one channel, N = 4096, fs = 1024 Hz
# ---------------------------------------------------------------------------

def make_c1(seed: int = 0, n: int = 4096) -> Workload:
    fs = 1024.0
    nn = np.arange(n, dtype=np.float64)
    t = nn / fs
    x1 = _cos_cycles(50.0 * nn / fs)
    x2 = 0.8 * _cos_cycles(100.0 * t + 75.0 * t * t)
    clean = x1 + x2
    rng = np.random.default_rng(seed)
    x = (clean + _white_noise_for(clean, 20.0, rng)).astype(np.float32)

    def inst_freq(tt):
        tt = np.asarray(tt, dtype=np.float64)
        f2 = 100.0 + 150.0 * tt
        # a real signal above fs/2 shows up folded back into [0, fs/2]
        f2 = np.where(f2 > fs / 2, fs - f2, f2)
        return np.stack([np.full_like(tt, 50.0), f2])

    cfg = SSTConfig(fs=fs, win_len=255, sigma=32.0, hop=1, nfft=4096, f_lo=0.0,
                    f_hi=fs / 2, subdiv=1, thr_mode="rel", thr=1e-6, hw=40)
    return Workload("c1", x, np.stack([x1, x2]), inst_freq, cfg, seed)


# ---------------------------------------------------------------------------
# Workload c2: downsampled SST, one channel, N = 2^20, fs = 25.6 kHz
# ---------------------------------------------------------------------------

C2_F0 = (120.0, 240.0, 600.0)
C2_AMP = (1.0, 0.5, 0.3)


def _amfm_c2_components(nn: np.ndarray, fs: float, f0s, amps, phases=None):
    t = nn / fs
    am = 1.0 + 0.2 * np.sin(TWO_PI * 0.5 * t)
    fm_cycles = (1.0 - np.cos(math.pi * t)) * (0.1 / TWO_PI)
    comps = []
    for i, (f0, a) in enumerate(zip(f0s, amps)):
        ph = 0.0 if phases is None else phases[i] / TWO_PI
        cycles = f0 * nn / fs + f0 * fm_cycles + ph
        comps.append(a * am * _cos_cycles(cycles))
    return np.stack(comps)


def make_c2(seed: int = 0, n: int = 1 << 20) -> Workload:
    fs = 25600.0
    nn = np.arange(n, dtype=np.float64)
    comps = _amfm_c2_components(nn, fs, C2_F0, C2_AMP)
    clean = comps.sum(axis=0)
    rng = np.random.default_rng(seed)
    x = (clean + _white_noise_for(clean, 10.0, rng)).astype(np.float32)

    def inst_freq(tt):
        tt = np.asarray(tt, dtype=np.float64)
        return np.stack([f0 * (1.0 + 0.05 * np.sin(math.pi * tt)) for f0 in C2_F0])

    cfg = SSTConfig(fs=fs, win_len=1023, sigma=128.0, hop=16, nfft=4096, f_lo=0.0,
                    f_hi=6400.0, subdiv=4, thr_mode="rel", thr=1e-3, hw=6)
    return Workload("c2", x, comps, inst_freq, cfg, seed)


# ---------------------------------------------------------------------------
# Workload c3: long run-up, N = 2^26, 8 harmonics of a 50 -> 600 Hz sweep
# ---------------------------------------------------------------------------

def make_c3(seed: int = 0, n: int = 1 << 26, duration: Optional[float] = None) -> Workload:
    fs = 25600.0
    dur = (n / fs) if duration is None else duration  # sweep length in seconds
    rng = np.random.default_rng(seed)
    theta = rng.uniform(0.0, TWO_PI, 8)
    nn = np.arange(n, dtype=np.float64)
    t = nn / fs
    base_cycles = 50.0 * t + 275.0 * t * t / dur
    comps = np.empty((8, n), dtype=np.float64)
    for h in range(1, 9):
        comps[h - 1] = (1.0 / h) * _cos_cycles(h * base_cycles + theta[h - 1] / TWO_PI)
    del base_cycles, t
    clean = comps.sum(axis=0)
    x = (clean + _pink_noise_for(clean, 15.0, rng)).astype(np.float32)
    del clean

    def inst_freq(tt):
        tt = np.asarray(tt, dtype=np.float64)
        f0 = 50.0 + 550.0 * tt / dur
        return np.stack([h * f0 for h in range(1, 9)])

    cfg = SSTConfig(fs=fs, win_len=2047, sigma=256.0, hop=32, nfft=8192, f_lo=0.0,
                    f_hi=5000.0, subdiv=8, thr_mode="rel", thr=1e-3, hw=26)
    return Workload("c3", x, comps, inst_freq, cfg, seed, meta={"duration": dur})


# ---------------------------------------------------------------------------
# Workload c4: many uneven channels with mixed hop / DFT size / subdivision
# ---------------------------------------------------------------------------

def _c4_channel(rng: np.random.Generator, fs: float, n: int):
    n_comp = int(rng.integers(1, 5))
    nn = np.arange(n, dtype=np.float64)
    t = nn / fs
    dur = n / fs
    comps, specs = [], []
    for _ in range(n_comp):
        amp = float(rng.uniform(0.3, 1.0))
        if rng.random() < 0.5:
            fa, fb = (float(v) for v in rng.uniform(100.0, 6000.0, 2))
            cycles = fa * t + 0.5 * (fb - fa) * t * t / dur
            comps.append(amp * _cos_cycles(cycles))
            specs.append(("chirp", fa, fb, dur))
        else:
            f0 = float(rng.uniform(100.0, 6000.0))
            fm_rate = float(rng.uniform(0.1, 1.0))
            am_rate = float(rng.uniform(0.1, 1.0))
            am_depth = float(rng.uniform(0.0, 0.3))
            # f(t) = f0 (1 + 0.05 sin(2 pi fm_rate t))
            cycles = f0 * t + f0 * 0.05 * (1.0 - np.cos(TWO_PI * fm_rate * t)) / (TWO_PI * fm_rate)
            comps.append(amp * (1.0 + am_depth * np.sin(TWO_PI * am_rate * t)) * _cos_cycles(cycles))
            specs.append(("amfm", f0, fm_rate))
    comps = np.stack(comps)
    snr = float(rng.uniform(5.0, 25.0))
    clean = comps.sum(axis=0)
    x = (clean + _white_noise_for(clean, snr, rng)).astype(np.float32)

    def inst_freq(tt, specs=specs):
        tt = np.asarray(tt, dtype=np.float64)
        rows = []
        for s in specs:
            if s[0] == "chirp":
                rows.append(s[1] + (s[2] - s[1]) * tt / s[3])
            else:
                rows.append(s[1] * (1.0 + 0.05 * np.sin(TWO_PI * s[2] * tt)))
        return np.stack(rows)

    return x, comps, inst_freq, snr


def make_c4(seed: int = 0, n_channels: int = 256, log2_min: float = 16.0,
            log2_max: float = 22.0) -> List[Workload]:
    fs = 25600.0
    children = np.random.SeedSequence(seed).spawn(n_channels)
    out = []
    for ci, ss in enumerate(children):
        rng = np.random.default_rng(ss)
        n = int(round(2.0 ** rng.uniform(log2_min, log2_max)))
        hop = int(rng.choice([4, 8, 16, 32]))
        nfft = int(rng.choice([1024, 2048, 4096]))
        z = int(rng.choice([2, 4]))
        x, comps, inst_freq, snr = _c4_channel(rng, fs, n)
        df = fs / nfft
        cfg = SSTConfig(fs=fs, win_len=nfft // 4 - 1, sigma=nfft / 32.0, hop=hop, nfft=nfft,
                        f_lo=0.0, f_hi=6400.0, subdiv=z, thr_mode="rel", thr=1e-3,
                        hw=max(1, int(round(10.0 * z / df))))
        out.append(Workload(f"c4[{ci}]", x, comps, inst_freq, cfg, seed, meta={"snr_db": snr}))
    return out


# ---------------------------------------------------------------------------
# Workload c5: many equal channels, small DFT sizes (precision tier)
# ---------------------------------------------------------------------------

def make_c5(seed: int = 0, n_channels: int = 512, n: int = 1 << 20, nfft: int = 512,
            f_hi: float = 6400.0) -> List[Workload]:
    fs = 25600.0
    rng = np.random.default_rng(seed)
    nn = np.arange(n, dtype=np.float64)
    out = []
    for ci in range(n_channels):
        scale = float(rng.uniform(0.8, 1.25))
        phases = rng.uniform(0.0, TWO_PI, 3)
        f0s = tuple(f * scale for f in C2_F0)
        comps = _amfm_c2_components(nn, fs, f0s, C2_AMP, phases)
        clean = comps.sum(axis=0)
        x = (clean + _white_noise_for(clean, 10.0, rng)).astype(np.float32)

        def inst_freq(tt, f0s=f0s):
            tt = np.asarray(tt, dtype=np.float64)
            return np.stack([f0 * (1.0 + 0.05 * np.sin(math.pi * tt)) for f0 in f0s])

        cfg = SSTConfig(fs=fs, win_len=nfft - 1, sigma=nfft / 8.0, hop=8, nfft=nfft, f_lo=0.0,
                        f_hi=f_hi, subdiv=1, thr_mode="rel", thr=1e-3, hw=1)
        out.append(Workload(f"c5[{ci}]", x, comps, inst_freq, cfg, seed))
    return out


# ---------------------------------------------------------------------------
# The paper's own simulated signal (Sec. 3, Eqs. 30-31)
# ---------------------------------------------------------------------------

def make_paper_eq30(seed: int = 0, snr_db: float = 5.0, n: int = 8192) -> Workload:
    fs = 1024.0
    nn = np.arange(n, dtype=np.float64)
    t = nn / fs
    x1 = (1.0 - 0.1 * np.cos(0.25 * math.pi * t)) * _cos_cycles(50.0 * t)
    # piecewise component: cycles = phase / (2 pi)
    c2a = (500.0 * t - 25.0 * t * t) / 2.0
    c2b = (500.0 * t - 50.0 * t * t + (25.0 / 6.0) * t ** 3 + 4.0 / 3.0) / 2.0
    x2 = np.where(t < 4.0, _cos_cycles(c2a), _cos_cycles(c2b))
    c3 = (740.0 * t + (400.0 / 3.0) * np.sin(0.75 * math.pi * t) / math.pi
          - 200.0 * np.sin(0.5 * math.pi * t) / math.pi) / 2.0
    x3 = (1.0 - 0.2 * np.cos(0.125 * math.pi * t)) * _cos_cycles(c3)
    comps = np.stack([x1, x2, x3])
    clean = comps.sum(axis=0)
    rng = np.random.default_rng(seed)
    x = (clean + _white_noise_for(clean, snr_db, rng)).astype(np.float32)

    def inst_freq(tt):
        tt = np.asarray(tt, dtype=np.float64)
        f1 = np.full_like(tt, 50.0)
        f2 = np.where(tt < 4.0, 250.0 - 25.0 * tt, 250.0 - 50.0 * tt + 6.25 * tt * tt)
        f3 = 370.0 + 50.0 * np.cos(0.75 * math.pi * tt) - 50.0 * np.cos(0.5 * math.pi * tt)
        return np.stack([f1, f2, f3])

    sigma = 0.03 * fs
    L = 2 * int(round(4 * sigma)) + 1
    cfg = SSTConfig(fs=fs, win_len=L, sigma=sigma, hop=1, nfft=n, f_lo=0.0, f_hi=fs / 2,
                    subdiv=1, thr_mode="rel", thr=1e-6, hw=int(round(10.0 * n / fs)))
    return Workload("eq30", x, comps, inst_freq, cfg, seed)


# ---------------------------------------------------------------------------
# Small deterministic signals for pins
# ---------------------------------------------------------------------------

def make_tone(n: int, f0: float, fs: float, amp: float = 1.0, phase: float = 0.0,
              complex_valued: bool = False) -> np.ndarray:
    nn = np.arange(n, dtype=np.float64)
    cyc = f0 * nn / fs + phase / TWO_PI
    frac = cyc - np.floor(cyc)
    if complex_valued:
        return amp * np.exp(1j * TWO_PI * frac)
    return amp * np.cos(TWO_PI * frac)


def make_chirp(n: int, f0: float, rate: float, fs: float, amp: float = 1.0) -> np.ndarray:
    """amp * cos(2 pi (f0 t + rate t^2 / 2)); instantaneous frequency f0 + rate t."""
    t = np.arange(n, dtype=np.float64) / fs
    return amp * _cos_cycles(f0 * t + 0.5 * rate * t * t)
