"""Pins of the oracle's periodogram peak detection (Sec. 5.5).

Each test checks the oracle against something other than itself: the
constants the paper prints, a library routine the rule reduces to, a
construction whose fitted threshold is known exactly, a statistical law, or
injected peaks whose positions and clusters are known.
"""
import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import peaks as pk
from conftest import golden


def rng(i):
    return np.random.Generator(np.random.Philox(4242 + i))


def small_plan_periods():
    """Trial periods of a one-octave plan in sample units (tau = 1, P in
    [128, 256), 128..255 bins, 2^18 samples): 181,071 rows."""
    octs = oracle.plan(1.0, 128.0, 256.0, 128, 255, 1 << 18)
    return np.concatenate([t.periods for o in octs for t in o.transforms if t.keep])


def test_constants_are_the_papers():
    g = golden("paper_constants.txt")
    assert pk.IQR_TO_SIGMA == float(g["iqr_to_sigma"])
    # the IQR of a unit normal is 2 Phi^-1(3/4) = 1.3490
    assert abs(2 * stats.norm.ppf(0.75) - pk.IQR_TO_SIGMA) < 1e-4
    d = pk.PeakParams()
    assert d.k_sigma == float(g["peak_k_sigma"]) and d.degree == int(g["peak_poly_degree"])


def test_quantiles_are_the_linear_interpolation_rule():
    # the reading reduces to numpy's default ('linear') percentile and median
    for n in list(range(1, 40)) + [255, 256, 1000]:
        v = np.sort(rng(n).standard_normal(n))
        for f in (0.25, 0.5, 0.75):
            ref = np.percentile(v, 100 * f)
            assert abs(pk.quantile_sorted(v, f) - ref) <= 1e-15 * max(1, abs(ref)), (n, f)
        assert abs(pk.quantile_sorted(v, 0.5) - np.median(v)) <= 1e-15


def test_segments_tile_the_frequency_range():
    per = small_plan_periods()
    T = float(1 << 18)
    nu, nu_lo, dnu, seg = pk.segment_index(per, T, 4.0)
    assert nu_lo == 1.0 / per.max()
    # each row lies in its segment's frequency interval
    lo = nu_lo + seg * dnu
    assert np.all(nu >= lo - 1e-15) and np.all(nu < lo + dnu + 1e-15)
    # rows are in ascending period, so segments run down without gaps
    d = np.diff(seg)
    assert np.all((d == 0) | (d == -1))
    assert seg[-1] == 0 and seg[0] == int((nu.max() - nu_lo) // dnu)


def test_threshold_of_an_exact_construction():
    # Every segment holds a linear ramp of n values centred on G(x_c), x_c the
    # log of the segment's centre frequency: median G(x_c), quartiles G -+ 1/2
    # (IQR 1) by the linear rule, so every control point is G(x_c) + k / 1.349
    # and the least-squares fit returns G's coefficients plus that constant.
    per = small_plan_periods()
    T = float(1 << 18)
    prm = pk.PeakParams(dz_seg=4.0, k_sigma=6.0, degree=2, min_points=16)
    nu, nu_lo, dnu, seg = pk.segment_index(per, T, prm.dz_seg)
    G = np.array([1.5, -0.75, 0.125])
    snr = np.empty(per.size)
    for i in np.unique(seg):
        idx = np.flatnonzero(seg == i)
        xc = np.log(nu_lo + (i + 0.5) * dnu)
        ramp = np.linspace(-1.0, 1.0, idx.size)
        snr[idx] = np.polynomial.polynomial.polyval(xc, G) + rng(int(i)).permutation(ramp)
    peaks, coefs, ctrl = pk.find_peaks(per, snr[:, None], 1 << 18, 1.0, prm)
    want = G + np.array([prm.k_sigma / pk.IQR_TO_SIGMA, 0.0, 0.0])
    assert np.allclose(coefs[0], want, rtol=0, atol=1e-8), coefs[0]
    # one control point per segment with at least min_points rows
    counts = np.bincount(seg)
    assert ctrl[0][0].size == int(np.count_nonzero(counts >= prm.min_points))
    # a ramp never exceeds the threshold (max G + 1 < G + 4.45)
    assert peaks == []


def test_gaussian_noise_threshold_is_mean_plus_k_sigma():
    # iid N(mu, s) S/N: median -> mu and IQR / 1.349 -> s, so the fitted
    # threshold is flat at mu + 6 s within the sampling error (about 1 %),
    # and nothing lies that far above the mean in 1.8e5 draws.
    per = small_plan_periods()
    mu, s = 3.0, 0.5
    snr = mu + s * rng(1).standard_normal((per.size, 2))
    peaks, coefs, _ = pk.find_peaks(per, snr, 1 << 18, 1.0)
    x = np.log(1.0 / per)
    for c in coefs:
        thr = pk.threshold(c, x)
        assert np.all(np.abs(thr - (mu + 6 * s)) < 0.06), (thr.min(), thr.max())
    assert peaks == []


def test_injected_peaks_are_found_and_clustered_per_width():
    per = small_plan_periods()
    snr = 3.0 + 0.5 * rng(2).standard_normal((per.size, 3))
    snr[5000:5004, 1] = [12.0, 15.0, 13.0, 11.0]   # one cluster of 4 rows (width 1)
    snr[90000, 1] = 10.0                           # an isolated peak (width 1)
    snr[120000, 2] = 9.5                           # width 2 only
    peaks, _, _ = pk.find_peaks(per, snr, 1 << 18, 1.0)
    got = [(p.width_index, p.row, p.members, p.snr) for p in peaks]
    assert got == [(1, 5001, 4, 15.0), (1, 90000, 1, 10.0), (2, 120000, 1, 9.5)]
    assert all(p.period == per[p.row] for p in peaks)


def test_cluster_gap_rule():
    # rows 0..5 with frequencies 1.0, 0.95, 0.90 (gap 0.05 each) then 0.5 (gap
    # 0.4), 0.49, 0.2 (gap 0.29); with gap 0.1 the clusters are {0,1,2}, {3,4},
    # {5}
    nu = np.array([1.0, 0.95, 0.90, 0.5, 0.49, 0.2])
    snr = np.array([5.0, 7.0, 6.0, 8.0, 8.0, 1.0])
    out = pk.cluster(np.arange(6), nu, snr, 0.1)
    assert out == [(1, 3), (3, 2), (5, 1)]  # equal S/N: the first row
    assert pk.cluster(np.arange(6), nu, snr, 0.3) == [(1, 3), (3, 3)]
    assert pk.cluster(np.arange(6), nu, snr, 0.45) == [(3, 6)]
    assert pk.cluster(np.zeros(0, dtype=np.int64), nu, snr, 0.1) == []
    # a step exactly equal to the gap keeps the cluster together (only a
    # larger step splits it); the frequencies are exact binary fractions
    nu2 = np.array([1.0, 0.75, 0.5, 0.125])
    s2 = np.array([1.0, 3.0, 2.0, 4.0])
    assert pk.cluster(np.arange(4), nu2, s2, 0.25) == [(1, 3), (3, 1)]


def test_small_and_non_finite_segments_give_no_control_point():
    per = small_plan_periods()
    T = float(1 << 18)
    prm = pk.PeakParams()
    nu, nu_lo, dnu, seg = pk.segment_index(per, T, prm.dz_seg)
    snr = 3.0 + 0.5 * rng(3).standard_normal(per.size)
    bad = seg == 7
    snr[np.flatnonzero(bad)[3]] = np.nan
    xs, ys, ids = pk.control_points(snr, seg, nu_lo, dnu, prm)
    assert 7 not in ids and 6 in ids and 8 in ids
    # exactly min_points rows give a control point, one fewer none
    seg2 = np.array([1] * 16 + [0] * 15)
    v2 = np.linspace(0.0, 1.0, seg2.size)
    ids2 = pk.control_points(v2, seg2, 0.1, 0.01, pk.PeakParams(min_points=16))[2]
    assert list(ids2) == [1]
    big = pk.PeakParams(min_points=10 ** 6)
    assert pk.control_points(snr, seg, nu_lo, dnu, big)[0].size == 0
    # no control points: no threshold, no peaks
    peaks, coefs, _ = pk.find_peaks(per, snr[:, None], 1 << 18, 1.0, big)
    assert coefs == [None] and peaks == []
