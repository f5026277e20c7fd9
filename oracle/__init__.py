"""FP64 CPU oracle for the FFA periodicity search of Morello et al. (2020).

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package. The GPU product path
never imports it, and the two share no code: this package has its own period
plan, downsampler, folding transforms and S/N, written from the paper.

Layout:
  * ``ffa_oracle.c`` -- the heavy loops in plain C, double precision
    (path offsets, brute-force fold, depth-first FFA, downsampling, boxcar S/N,
    running median);
  * this module -- the period plan and normalisation (numpy FP64 / Python
    integers) and the ctypes glue.

Readings of the paper used here, where it is silent or ambiguous:
  * plan: first downsampling factor ds0 = P_min / (b_min * tau) and it must be
    >= 1; the factor is multiplied by f = (b_max + 1) / b_min in FP64 from one
    pseudo-octave to the next (Sec. 5.3: always re-downsample the original
    series, never chain), quantised to 32.32 fixed point; a pseudo-octave is
    searched while b_min * tau_k < P_max, and bins p while p * tau_k < P_max;
  * incomplete last rows and the incomplete last downsampling window are
    dropped (Sec. 2.2);
  * transforms with fewer than two rows are skipped (the period of row s
    divides by m - 1, Sec. 2.3);
  * a row is kept when its period P_s < min((p + 1) tau_k, P_max): the paper
    says that the trials past (p + 1) tau overlap the next transform and are
    ignored (Sec. 2.3);
  * the noise variance of a downsampled sample is ds for an integer factor and
    ds - 1/3 otherwise (Sec. 5.3, App. A.4);
  * normalisation uses the population standard deviation of the whole raw
    series (Sec. 5.2);
  * de-reddening (Sec. 5.2) subtracts the running median over an odd window
    centred on each sample, cut at the ends of the series, the median of an
    even count (only at the ends) being the lower of the two middle values.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ffa_oracle.c")
_LIB = os.path.join(_HERE, "_ffa_oracle.so")
_lib = None

TWO32 = 1 << 32


def build(force: bool = True) -> str:
    """Compile the C part of the oracle with gcc (OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    i64, i32, u64, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double
    pd = ctypes.POINTER(ctypes.c_double)
    pi64 = ctypes.POINTER(ctypes.c_int64)
    pi32 = ctypes.POINTER(ctypes.c_int32)
    lib.oracle_path_offset.argtypes = [i64, i64, i64]
    lib.oracle_path_offset.restype = i64
    lib.oracle_path_table.argtypes = [i64, pi64]
    lib.oracle_path_table.restype = None
    lib.oracle_fold_bruteforce.argtypes = [pd, i64, i64, pd]
    lib.oracle_fold_bruteforce.restype = None
    lib.oracle_fold_ffa.argtypes = [pd, i64, i64, pd]
    lib.oracle_fold_ffa.restype = ctypes.c_int
    lib.oracle_downsample.argtypes = [pd, i64, u64, i64, pd]
    lib.oracle_downsample.restype = None
    lib.oracle_boxcar_snr.argtypes = [pd, i64, i64, i64, dbl, pi32, i32, pd]
    lib.oracle_boxcar_snr.restype = None
    lib.oracle_transforms_snr.argtypes = [pd, i64, pi64, pi64, pi64, pd, pi64, pi64, i32, pi32,
                                          i32, pd]
    lib.oracle_transforms_snr.restype = ctypes.c_int
    lib.oracle_running_median.argtypes = [pd, i64, i64, pd, pd]
    lib.oracle_running_median.restype = ctypes.c_int
    _lib = lib
    return lib


def _p(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


# --------------------------------------------------------------------------
# Folding transform (Sec. 2.1, 2.2)
# --------------------------------------------------------------------------

def path_offset(m: int, s: int, r: int) -> int:
    """D_m(s, r): bins by which path s is shifted when it picks up row r."""
    return int(_load().oracle_path_offset(m, s, r))


def path_table(m: int) -> np.ndarray:
    """m x m table D[s, r]."""
    out = np.empty((m, m), dtype=np.int64)
    _load().oracle_path_table(m, _p(out, ctypes.c_int64))
    return out


def fold_bruteforce(X: np.ndarray) -> np.ndarray:
    """Folding transform of an m x p array by brute force, O(p m^2)."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    m, p = X.shape
    F = np.empty_like(X)
    _load().oracle_fold_bruteforce(_p(X, ctypes.c_double), m, p, _p(F, ctypes.c_double))
    return F


def fold_ffa(X: np.ndarray) -> np.ndarray:
    """Folding transform of an m x p array by the depth-first FFA."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    m, p = X.shape
    F = np.empty_like(X)
    if _load().oracle_fold_ffa(_p(X, ctypes.c_double), m, p, _p(F, ctypes.c_double)) != 0:
        raise MemoryError("oracle_fold_ffa")
    return F


# --------------------------------------------------------------------------
# Downsampling, normalisation, S/N (Sec. 5.2 - 5.4, App. A.4)
# --------------------------------------------------------------------------

def downsample(x: np.ndarray, ds_fx: int, nout: int) -> np.ndarray:
    """Overlap-weighted windows of ds_fx / 2^32 samples (32.32 fixed point)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(nout, dtype=np.float64)
    _load().oracle_downsample(_p(x, ctypes.c_double), x.size, ds_fx, nout,
                              _p(y, ctypes.c_double))
    return y


def running_median(x: np.ndarray, window: int):
    """De-reddening by a running median (Sec. 5.2): returns (y, med) with
    med[i] the median of the `window` (odd) samples centred on i, the window
    cut at the ends of the series (the median of n samples being the
    ((n - 1) // 2)-th smallest, 0-based), and y = x - med, in FP64."""
    if window < 1 or window % 2 == 0:
        raise ValueError("window must be odd and positive")
    x = np.ascontiguousarray(x, dtype=np.float64)
    med = np.empty_like(x)
    y = np.empty_like(x)
    if _load().oracle_running_median(_p(x, ctypes.c_double), x.size, window,
                                     _p(med, ctypes.c_double), _p(y, ctypes.c_double)) != 0:
        raise MemoryError("oracle_running_median")
    return y, med


def normalise_stats(x: np.ndarray):
    """Mean and population standard deviation of the whole series, FP64."""
    xd = np.asarray(x, dtype=np.float64)
    mu = xd.sum() / xd.size
    sigma = np.sqrt(((xd - mu) ** 2).sum() / xd.size)
    return float(mu), float(sigma)


def boxcar_snr(F: np.ndarray, m: int, var: float, widths: Sequence[int]) -> np.ndarray:
    """Best circular-boxcar S/N of each row of F (rows x p) for each width."""
    F = np.ascontiguousarray(F, dtype=np.float64)
    rows, p = F.shape
    w = np.ascontiguousarray(widths, dtype=np.int32)
    out = np.empty((rows, w.size), dtype=np.float64)
    _load().oracle_boxcar_snr(_p(F, ctypes.c_double), rows, p, m, var, _p(w, ctypes.c_int32),
                              w.size, _p(out, ctypes.c_double))
    return out


# --------------------------------------------------------------------------
# Period plan (Sec. 2.3, 5.3)
# --------------------------------------------------------------------------

@dataclass
class Transform:
    p: int            # bins per period, base period p * tau_k
    m: int            # rows folded
    keep: int         # rows kept: the first `keep` rows of the transform
    periods: np.ndarray  # FP64 period of each kept row, seconds


@dataclass
class Octave:
    ds: float         # downsampling factor before quantisation
    ds_fx: int        # quantised factor, 32.32 fixed point
    tau: float        # sampling time after downsampling
    nsamp: int        # samples after downsampling
    var: float        # noise variance of one downsampled sample
    transforms: List[Transform] = field(default_factory=list)


class PlanError(ValueError):
    """Raised for parameters the plan cannot serve."""


def trial_period(s, m: int, p: int, tau: float):
    """Period of row s of an m-row transform with base period p * tau (Eq. for P_s, Sec. 2.3)."""
    return tau * p * p / (p - s / (m - 1))


def plan(tsamp: float, period_min: float, period_max: float, bins_min: int, bins_max: int,
         nsamp: int) -> List[Octave]:
    if not (tsamp > 0 and 0 < period_min < period_max and 2 <= bins_min <= bins_max):
        raise PlanError("invalid parameters")
    ds = period_min / (bins_min * tsamp)
    if ds < 1.0:
        raise PlanError("period_min / (bins_min * tsamp) < 1")
    f = (bins_max + 1) / bins_min
    octaves: List[Octave] = []
    while True:
        ds_fx = int(np.floor(ds * TWO32 + 0.5))
        tau = tsamp * (ds_fx / TWO32)
        if bins_min * tau >= period_max:
            break
        nk = (nsamp * TWO32) // ds_fx
        dsq = ds_fx / TWO32
        var = dsq if ds_fx % TWO32 == 0 else dsq - 1.0 / 3.0
        octv = Octave(ds=ds, ds_fx=ds_fx, tau=tau, nsamp=nk, var=var)
        for p in range(bins_min, bins_max + 1):
            if p * tau >= period_max:
                break
            m = nk // p
            if m < 2:
                continue
            s = np.arange(m, dtype=np.float64)
            per = trial_period(s, m, p, tau)
            si = np.arange(m, dtype=np.int64)
            ok = (si * (p + 1) < p * (m - 1)) & (per < period_max)
            keep = int(np.count_nonzero(ok))
            # periods increase with s, so the kept rows are a prefix
            assert ok[:keep].all()
            octv.transforms.append(Transform(p=p, m=m, keep=keep, periods=per[:keep]))
        octaves.append(octv)
        ds = ds * f
    return octaves


def plan_rows(octaves: List[Octave]) -> int:
    return sum(t.keep for o in octaves for t in o.transforms)


# --------------------------------------------------------------------------
# Whole search
# --------------------------------------------------------------------------

@dataclass
class Periodogram:
    periods: np.ndarray   # FP64, one per row
    bins: np.ndarray      # int32 p of the row's transform
    snr: np.ndarray       # FP64, rows x num_widths
    octave: np.ndarray    # int32
    rows_m: np.ndarray    # int32 m of the row's transform
    s: np.ndarray         # int32 row index inside its transform


def search(x: np.ndarray, tsamp: float, period_min: float, period_max: float, bins_min: int,
           bins_max: int, widths: Sequence[int], normalise: bool = True, brute: bool = False,
           octave_subset: Optional[Sequence[int]] = None, median_window: int = 0) -> Periodogram:
    """Periodogram of one series: subtract the running median if a window is
    given, normalise (Sec. 5.2), then for every pseudo-octave downsample the
    original (Sec. 5.3), fold at every p (Sec. 2) and take the boxcar S/N of
    every kept row (Sec. 5.4, 5.5). Rows are in (octave, p, s) order, which is
    ascending period."""
    widths = [int(w) for w in widths]
    if not widths or any(w < 1 for w in widths) or any(b <= a for a, b in zip(widths, widths[1:])):
        raise PlanError("widths must be strictly increasing and >= 1")
    if widths[-1] >= bins_min:
        raise PlanError("widest boxcar must be narrower than bins_min")
    xd = np.asarray(x, dtype=np.float64)
    if median_window:
        xd = running_median(xd, median_window)[0]
    if normalise:
        mu, sigma = normalise_stats(xd)
        if not np.isfinite(sigma) or sigma == 0.0:
            raise PlanError("degenerate series")
        xd = (xd - mu) / sigma
    octaves = plan(tsamp, period_min, period_max, bins_min, bins_max, xd.size)
    w = np.asarray(widths, dtype=np.int32)
    per_l, bins_l, snr_l, oct_l, m_l, s_l = [], [], [], [], [], []
    for k, o in enumerate(octaves):
        if octave_subset is not None and k not in octave_subset:
            continue
        if not o.transforms:
            continue
        y = downsample(xd, o.ds_fx, o.nsamp)
        ntr = len(o.transforms)
        y_off = np.zeros(ntr, dtype=np.int64)
        m = np.array([t.m for t in o.transforms], dtype=np.int64)
        p = np.array([t.p for t in o.transforms], dtype=np.int64)
        var = np.full(ntr, o.var, dtype=np.float64)
        keep = np.array([t.keep for t in o.transforms], dtype=np.int64)
        out_off = np.concatenate([[0], np.cumsum(keep)[:-1]]).astype(np.int64)
        out = np.empty((int(keep.sum()), w.size), dtype=np.float64)
        rc = _load().oracle_transforms_snr(
            _p(y, ctypes.c_double), ntr, _p(y_off, ctypes.c_int64), _p(m, ctypes.c_int64),
            _p(p, ctypes.c_int64), _p(var, ctypes.c_double), _p(keep, ctypes.c_int64),
            _p(out_off, ctypes.c_int64), 1 if brute else 0, _p(w, ctypes.c_int32), w.size,
            _p(out, ctypes.c_double))
        if rc != 0:
            raise MemoryError("oracle_transforms_snr")
        for t in o.transforms:
            per_l.append(t.periods)
            bins_l.append(np.full(t.keep, t.p, dtype=np.int32))
            oct_l.append(np.full(t.keep, k, dtype=np.int32))
            m_l.append(np.full(t.keep, t.m, dtype=np.int32))
            s_l.append(np.arange(t.keep, dtype=np.int32))
        snr_l.append(out)
    cat = lambda l, dt: np.concatenate(l) if l else np.zeros(0, dtype=dt)
    return Periodogram(periods=cat(per_l, np.float64), bins=cat(bins_l, np.int32),
                       snr=np.concatenate(snr_l) if snr_l else np.zeros((0, w.size)),
                       octave=cat(oct_l, np.int32), rows_m=cat(m_l, np.int32),
                       s=cat(s_l, np.int32))


def search_ranges(x: np.ndarray, tsamp: float, ranges, widths: Sequence[int],
                  normalise: bool = True) -> Periodogram:
    """Dynamic duty-cycle resolution (Sec. 5.6): the period range cut into
    consecutive sub-ranges, each searched with its own (period_min,
    period_max, bins_min, bins_max), and the periodograms concatenated in
    range order. `ranges` holds those four values per sub-range, ascending and
    without overlap."""
    parts = []
    for k, (pmin, pmax, bmin, bmax) in enumerate(ranges):
        if k > 0 and ranges[k - 1][1] > pmin:
            raise PlanError("sub-ranges must ascend without overlap")
        parts.append(search(x, tsamp, pmin, pmax, bmin, bmax, widths, normalise=normalise))
    cat = lambda f: np.concatenate([getattr(q, f) for q in parts])
    return Periodogram(periods=cat("periods"), bins=cat("bins"),
                       snr=np.concatenate([q.snr for q in parts]), octave=cat("octave"),
                       rows_m=cat("rows_m"), s=cat("s"))
