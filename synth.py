"""Seeded synthetic inputs for the FFA periodicity search.

This module only draws random series and injects pulses; it holds none of the
search's arithmetic. Both the oracle-side tests and the GPU side take their
inputs from here.

Recipe (every generator is numpy ``Generator(Philox(seed))`` with
``seed = 20200407 + 1000 * workload + index``):

* noise: float32 N(0, 1) samples, the model of Sec. 3.1 (uncorrelated Gaussian
  noise of zero mean and unit variance);
* pulse: a periodic von Mises pulse exp(kappa (cos 2 pi (phi - phi0) - 1)) with
  kappa = ln 2 / (1 - cos(pi * duty)) so that its FWHM is duty * period;
  the pulse train is scaled to unit square sum over the whole series and
  multiplied by the amplitude a, so that "S/N a" is the amplitude of Sec. 3.1;
* red noise: a 1/f power spectrum with the DC term removed, scaled to the
  requested standard deviation (left in the series: the search removes it
  with its running-median de-reddening).

Workloads (sizes of the paper's benchmark setting, Sec. 5.8: 2^23 samples of
64 us per DM trial):

1. one 262,144-sample series, tau = 1 (sample units), one pulse of period
   200.37 samples, duty 5 %, amplitude 15; periods [128, 256), bins 128..255,
   widths 1,2,3,4,6,9,13,19,28;
2. one 9,375,000-sample series (600 s at 64 us) with red noise of std 0.1,
   de-reddened in the search by a 5 s running median (78,125 samples), and
   3 pulses of period log-uniform in
   [0.5, 10] s, duty U[1 %, 10 %], amplitude U[8, 20]; periods [0.5, 10) s,
   bins 240..259, widths 1,2,3,5,8,12,19,30,48;
3. 512 series of 2^23 samples at 64 us; a seeded 10 % of them (51) carry one
   pulse with period U[0.5, 10] s, duty U[1 %, 10 %], amplitude U[6, 20];
   same plan as workload 2;
4. workload 3 normalised in FP64 and stored as bfloat16, and as float16;
5. 256 series of floor(2^U) samples, U ~ U[20, 24], tau in {64, 128, 256} us,
   period range 0.1-1 s or 1-30 s; 10 % carry a pulse drawn inside their range.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import numpy as np

SEED_BASE = 20200407

WIDTHS_PAPER = (1, 2, 3, 4, 6, 9, 13, 19, 28)
WIDTHS_DUTY = (1, 2, 3, 5, 8, 12, 19, 30, 48)


def seed(workload: int, index: int) -> int:
    return SEED_BASE + 1000 * workload + index


def rng(workload: int, index: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(seed(workload, index)))


@dataclass
class SearchConfig:
    tsamp: float
    period_min: float
    period_max: float
    bins_min: int
    bins_max: int
    widths: Tuple[int, ...]
    median_window: int = 0   # running-median de-reddening window in samples (0: none)


@dataclass
class Pulse:
    period: float     # in samples
    duty: float
    amplitude: float
    phi0: float


def noise(n: int, g: np.random.Generator) -> np.ndarray:
    return g.standard_normal(n, dtype=np.float32)


def pulse_train(n: int, pulse: Pulse) -> np.ndarray:
    """Unit-square-sum von Mises pulse train, FP64, sampled at t = 0..n-1."""
    kappa = math.log(2.0) / (1.0 - math.cos(math.pi * pulse.duty))
    phase = np.arange(n, dtype=np.float64) / pulse.period - pulse.phi0
    s = np.exp(kappa * (np.cos(2.0 * np.pi * phase) - 1.0))
    s /= np.sqrt(np.dot(s, s))
    return s


def inject(x: np.ndarray, pulse: Pulse) -> np.ndarray:
    out = x.astype(np.float64) + pulse.amplitude * pulse_train(x.size, pulse)
    return out.astype(np.float32)


def red_noise(n: int, std: float, g: np.random.Generator) -> np.ndarray:
    """Gaussian noise with a 1/f power spectrum, DC removed, given std."""
    nf = n // 2 + 1
    f = np.arange(nf, dtype=np.float64)
    amp = np.zeros(nf)
    amp[1:] = 1.0 / np.sqrt(f[1:])
    spec = amp * (g.standard_normal(nf) + 1j * g.standard_normal(nf))
    r = np.fft.irfft(spec, n)
    r -= r.mean()
    r *= std / r.std()
    return r


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------

def workload1() -> Tuple[np.ndarray, SearchConfig, List[Pulse]]:
    g = rng(1, 0)
    n = 262144
    x = noise(n, g)
    p = Pulse(period=200.37, duty=0.05, amplitude=15.0, phi0=float(g.uniform()))
    x = inject(x, p)
    return x, SearchConfig(1.0, 128.0, 256.0, 128, 255, WIDTHS_PAPER), [p]


def config_duty(tsamp: float, pmin: float, pmax: float) -> SearchConfig:
    return SearchConfig(tsamp, pmin, pmax, 240, 259, WIDTHS_DUTY)


def workload2() -> Tuple[np.ndarray, SearchConfig, List[Pulse]]:
    g = rng(2, 0)
    tsamp = 64e-6
    n = 9_375_000
    x = noise(n, g).astype(np.float64) + red_noise(n, 0.1, g)
    pulses = []
    for _ in range(3):
        per_s = math.exp(g.uniform(math.log(0.5), math.log(10.0)))
        pulses.append(Pulse(period=per_s / tsamp, duty=float(g.uniform(0.01, 0.10)),
                            amplitude=float(g.uniform(8.0, 20.0)), phi0=float(g.uniform())))
    for p in pulses:
        x = x + p.amplitude * pulse_train(n, p)
    # de-reddened in the search by a running median of 5 s (78,125 samples)
    cfg = config_duty(tsamp, 0.5, 10.0)
    cfg.median_window = int(round(5.0 / tsamp)) | 1
    return x.astype(np.float32), cfg, pulses


WL3_SERIES = 512
WL3_NSAMP = 1 << 23


def workload3_pulsed(nseries: int = WL3_SERIES) -> np.ndarray:
    """Indices of the seeded 10 % subset of workload-3 series that carry a pulse."""
    g = rng(3, 999_999)
    k = max(1, int(round(0.1 * nseries)))
    return np.sort(g.choice(nseries, size=k, replace=False))


def workload3_series(index: int, nsamp: int = WL3_NSAMP, nseries: int = WL3_SERIES,
                     pulsed: Optional[Sequence[int]] = None) -> Tuple[np.ndarray, Optional[Pulse]]:
    g = rng(3, index)
    x = noise(nsamp, g)
    if pulsed is None:
        pulsed = workload3_pulsed(nseries)
    pulse = None
    if index in set(int(i) for i in pulsed):
        tsamp = 64e-6
        pulse = Pulse(period=float(g.uniform(0.5, 10.0)) / tsamp,
                      duty=float(g.uniform(0.01, 0.10)),
                      amplitude=float(g.uniform(6.0, 20.0)), phi0=float(g.uniform()))
        x = inject(x, pulse)
    return x, pulse


def workload3_config() -> SearchConfig:
    return config_duty(64e-6, 0.5, 10.0)


def to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """float32 -> bfloat16 bit patterns (uint16), round to nearest even."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    rounding = ((u >> 16) & 1) + 0x7FFF
    return ((u + rounding) >> 16).astype(np.uint16)


def from_bf16_bits(b: np.ndarray) -> np.ndarray:
    return (b.astype(np.uint32) << 16).view(np.float32)


def workload5_series(index: int) -> Tuple[np.ndarray, SearchConfig, Optional[Pulse]]:
    g = rng(5, index)
    u = g.uniform(20.0, 24.0)
    n = int(math.floor(2.0 ** u))
    tsamp = float(g.choice([64e-6, 128e-6, 256e-6]))
    lo, hi = (0.1, 1.0) if g.uniform() < 0.5 else (1.0, 30.0)
    x = noise(n, g)
    pulse = None
    if g.uniform() < 0.1:
        pulse = Pulse(period=float(g.uniform(lo, hi)) / tsamp, duty=float(g.uniform(0.01, 0.10)),
                      amplitude=float(g.uniform(6.0, 20.0)), phi0=float(g.uniform()))
        x = inject(x, pulse)
    return x, config_duty(tsamp, lo, hi), pulse
