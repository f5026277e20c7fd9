"""FP64 CPU reference of the periodogram peak detection (Sec. 5.5 and the
caption of its peak-detection figure).

TEST INFRASTRUCTURE ONLY, like the rest of this package: only the test suite,
the smoke check and the benchmark's CPU-baseline leg may use it. It shares no
code with the library.

What the paper fixes: every width trial of the two-dimensional periodogram is
searched on its own; its S/N, as a function of trial frequency nu = 1 / P, is
cut into equal segments of width dz_seg / T (T the length of the series in
seconds); each segment gives a control point at its centre frequency with
value median + k * sigma, sigma = IQR / 1.349 (k = 6 by default); a polynomial
in log(nu) (degree 2 by default) is fitted to the control points by linear
least squares and is the selection threshold; the points above it are
clustered into peaks.

Readings where the paper is silent (each one is a parameter or a rule here):
  * T = nsamp * tsamp of the raw series;
  * segment i covers [nu_lo + i dnu, nu_lo + (i + 1) dnu), dnu = dz_seg / T,
    nu_lo the lowest trial frequency (1 / the longest trial period); a row's
    segment is floor((nu - nu_lo) / dnu) in FP64; the last segment may be
    partial;
  * median and quartiles: linear interpolation between order statistics at
    position f (n - 1) of the sorted sample (f = 0.25, 0.5, 0.75);
  * a segment with fewer than min_points points, or with a non-finite S/N,
    gives no control point;
  * the fit is unweighted, x = natural log of the centre frequency; with fewer
    than degree + 1 control points the width has no threshold and no peaks;
  * a point is above the threshold when float64(snr) > threshold;
  * clustering: the points above the threshold, in frequency order, form one
    cluster while consecutive members are at most cluster_gap / T apart in
    frequency; a peak is its cluster's brightest member (the first in row
    order on equal S/N), with the member count.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional

import numpy as np

IQR_TO_SIGMA = 1.349


@dataclass
class PeakParams:
    dz_seg: float = 4.0        # segment width in units of 1 / T
    k_sigma: float = 6.0       # threshold = median + k_sigma * IQR / 1.349
    degree: int = 2            # polynomial degree in log(frequency)
    cluster_gap: float = 1.0   # cluster members at most cluster_gap / T apart
    min_points: int = 16       # fewest points of a segment with a control point


@dataclass
class Peak:
    row: int
    width_index: int
    members: int
    snr: float
    threshold: float
    period: float


def quantile_sorted(v: np.ndarray, f: float) -> float:
    """Quantile f of a sorted sample by linear interpolation between the order
    statistics around position f (n - 1)."""
    n = v.size
    pos = f * (n - 1)
    lo = int(np.floor(pos))
    hi = lo + 1 if lo + 1 < n else lo
    t = pos - lo
    a, b = float(v[lo]), float(v[hi])
    return a + (b - a) * t


def segment_index(periods: np.ndarray, T: float, dz_seg: float):
    """Frequency of every row, the lowest trial frequency, the segment width
    and every row's segment."""
    nu = 1.0 / np.asarray(periods, dtype=np.float64)
    nu_lo = float(nu.min())
    dnu = dz_seg / T
    seg = np.floor((nu - nu_lo) / dnu).astype(np.int64)
    return nu, nu_lo, dnu, seg


def control_points(snr_w: np.ndarray, seg: np.ndarray, nu_lo: float, dnu: float,
                   prm: PeakParams):
    """(x, y, segment) of every control point of one width: x = log of the
    segment's centre frequency, y = median + k IQR / 1.349."""
    xs, ys, ids = [], [], []
    for i in np.unique(seg):
        v = np.asarray(snr_w[seg == i], dtype=np.float64)
        if v.size < prm.min_points or not np.all(np.isfinite(v)):
            continue
        v = np.sort(v)
        med = quantile_sorted(v, 0.5)
        iqr = quantile_sorted(v, 0.75) - quantile_sorted(v, 0.25)
        ys.append(med + prm.k_sigma * iqr / IQR_TO_SIGMA)
        xs.append(np.log(nu_lo + (i + 0.5) * dnu))
        ids.append(int(i))
    return np.array(xs), np.array(ys), np.array(ids, dtype=np.int64)


def fit_threshold(xs: np.ndarray, ys: np.ndarray, degree: int) -> Optional[np.ndarray]:
    """Least-squares polynomial coefficients c_0 .. c_d (power basis in x),
    or None with too few control points."""
    if xs.size < degree + 1:
        return None
    V = np.vander(xs, degree + 1, increasing=True)
    c, *_ = np.linalg.lstsq(V, ys, rcond=None)
    return c


def threshold(c: np.ndarray, x: np.ndarray) -> np.ndarray:
    return np.polynomial.polynomial.polyval(x, c)


def cluster(rows: np.ndarray, nu: np.ndarray, snr: np.ndarray, gap: float):
    """Splits rows above the threshold (ascending row = descending
    frequency) into clusters; returns (brightest row, members) per cluster."""
    out = []
    start = 0
    for i in range(1, rows.size + 1):
        if i == rows.size or nu[rows[i - 1]] - nu[rows[i]] > gap:
            r = rows[start:i]
            b = r[int(np.argmax(snr[r]))]  # argmax takes the first of equal values
            out.append((int(b), int(i - start)))
            start = i
    return out


def find_peaks(periods: np.ndarray, snr: np.ndarray, nsamp: int, tsamp: float,
               prm: PeakParams = PeakParams()):
    """Peaks of one periodogram (rows in ascending period, snr rows x widths).
    Returns (peaks ordered by width then row, list of the coefficients or None
    per width, per width the control points (x, y, segment))."""
    T = nsamp * tsamp
    nu, nu_lo, dnu, seg = segment_index(periods, T, prm.dz_seg)
    x = np.log(nu)
    gap = prm.cluster_gap / T
    peaks: List[Peak] = []
    coefs, ctrl = [], []
    for w in range(snr.shape[1]):
        sw = np.asarray(snr[:, w], dtype=np.float64)
        xs, ys, ids = control_points(sw, seg, nu_lo, dnu, prm)
        ctrl.append((xs, ys, ids))
        c = fit_threshold(xs, ys, prm.degree)
        coefs.append(c)
        if c is None:
            continue
        thr = threshold(c, x)
        above = np.flatnonzero(sw > thr)
        for row, members in cluster(above, nu, sw, gap):
            peaks.append(Peak(row=row, width_index=w, members=members, snr=float(sw[row]),
                              threshold=float(thr[row]), period=float(periods[row])))
    return peaks, coefs, ctrl
