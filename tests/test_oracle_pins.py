"""Pins of the FP64 oracle to what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a worked
example printed in the paper, a closed form, an invariant, a special case that
reduces to a textbook algorithm written independently here, or a statistical
law. A plausible slip in the oracle (a dropped term, a flipped rotation, a
wrong rounding or split, a missing factor in the S/N) fails at least one.
"""
import math

import numpy as np
import pytest
from scipy import special, stats

import oracle
from conftest import golden


def rng(i):
    return np.random.Generator(np.random.Philox(777 + i))


# --------------------------------------------------------------------------
# Integration paths (Sec. 2.1, 2.2)
# --------------------------------------------------------------------------

def test_path_endpoints_and_unit_steps():
    # A path of total drift s starts at phase 0, ends at phase s and moves by
    # 0 or 1 bin per row: the merge rule only allows a 1-bin jump b in {0, 1}
    # at each head/tail boundary (Sec. 2.2).
    for m in range(1, 200):
        D = oracle.path_table(m)
        assert (D[:, 0] == 0).all()
        assert (D[:, m - 1] == np.arange(m)).all()
        if m > 1:
            steps = np.diff(D, axis=1)
            assert ((steps == 0) | (steps == 1)).all(), m


def test_path_stays_near_the_straight_drift():
    # The path approximates the straight line s * r / (m - 1) (Sec. 2.1); the
    # error grows at most by half a bin per level of the tree.
    for m in [2, 3, 5, 7, 8, 13, 64, 100, 129, 255, 299]:
        D = oracle.path_table(m)
        s = np.arange(m)[:, None]
        r = np.arange(m)[None, :]
        dev = np.abs(D - s * r / max(m - 1, 1))
        assert dev.max() <= 0.5 * math.ceil(math.log2(m)) + 0.5, m


def test_fig1_worked_example():
    g = golden("fig1_folding_transform.txt")
    m, p, phi, s = int(g["m"]), int(g["p"]), int(g["phi"]), int(g["s"])
    X = np.zeros((m, p))
    for r in range(m):
        X[r, (phi + int(round(s * r / (m - 1)))) % p] = 1.0
    for F in (oracle.fold_ffa(X), oracle.fold_bruteforce(X)):
        row, col = np.unravel_index(np.argmax(F), F.shape)
        assert (row, col) == (int(g["peak_row"]), int(g["peak_col"]))
        assert F[row, col] == float(g["peak_value"])
        # the peak is unique: every other cell sums fewer pulses
        assert (F.ravel() == F.max()).sum() == 1


def test_fig2_merge_example():
    # Fig. 2 caption: the fourth output row (s = 3) of an 8-row input is built
    # from one row of the head transform and one of the tail transform. With
    # m_h = m_t = 4: i = nint(3 * 3/7) = 1, j = 1, b = 3 - 2 = 1, so
    # F_3 = H_1 + (T_1 << 2).
    X = rng(1).integers(-5, 6, size=(8, 11)).astype(np.float64)
    H = oracle.fold_ffa(X[:4])
    T = oracle.fold_ffa(X[4:])
    F = oracle.fold_ffa(X)
    assert np.array_equal(F[3], H[1] + np.roll(T[1], -2))


def _staelin_radix2(X):
    """Classic breadth-first FFA for m = 2^k rows (Staelin 1969, as recalled in
    Sec. 2.2): blocks of 2, 4, 8, ... rows; block row s is
    H[s // 2] + roll(T[s // 2], -ceil(s / 2))."""
    m, p = X.shape
    cur = [X[r:r + 1].copy() for r in range(m)]
    while len(cur) > 1:
        nxt = []
        for a in range(0, len(cur), 2):
            H, T = cur[a], cur[a + 1]
            n = 2 * H.shape[0]
            B = np.empty((n, p))
            for s in range(n):
                B[s] = H[s // 2] + np.roll(T[s // 2], -((s + 1) // 2))
            nxt.append(B)
        cur = nxt
    return cur[0]


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6, 7, 8])
def test_power_of_two_reduces_to_staelin(k):
    # The depth-first variant gives results identical to the original FFA (Sec. 2).
    X = rng(k).integers(-8, 9, size=(2 ** k, 17)).astype(np.float64)
    ref = _staelin_radix2(X)
    assert np.array_equal(oracle.fold_ffa(X), ref)
    assert np.array_equal(oracle.fold_bruteforce(X), ref)


def test_ffa_equals_bruteforce_on_random_shapes():
    g = rng(2)
    for trial in range(120):
        m = int(g.integers(1, 300))
        p = int(g.integers(2, 64))
        X = g.integers(-8, 9, size=(m, p)).astype(np.float64)
        assert np.array_equal(oracle.fold_ffa(X), oracle.fold_bruteforce(X)), (m, p)
    for trial in range(20):
        m = int(g.integers(1, 200))
        p = int(g.integers(2, 40))
        X = g.standard_normal((m, p))
        np.testing.assert_allclose(oracle.fold_ffa(X), oracle.fold_bruteforce(X), rtol=0,
                                   atol=1e-11)


def test_transform_invariants():
    g = rng(3)
    for m, p in [(1, 5), (2, 3), (3, 7), (37, 19), (128, 12), (301, 9)]:
        X = g.standard_normal((m, p))
        Y = g.standard_normal((m, p))
        F = oracle.fold_ffa(X)
        # every profile holds every input sample once: the row sums are the total
        np.testing.assert_allclose(F.sum(axis=1), X.sum(), rtol=0, atol=1e-9)
        # s = 0 is the plain fold at period p (Sec. 3.4)
        np.testing.assert_allclose(F[0], X.sum(axis=0), rtol=0, atol=1e-12)
        # s = m - 1 drifts one bin per row
        last = sum(np.roll(X[r], -r) for r in range(m))
        np.testing.assert_allclose(F[m - 1], last, rtol=0, atol=1e-12)
        # linearity
        np.testing.assert_allclose(oracle.fold_ffa(2.5 * X - Y), 2.5 * F - oracle.fold_ffa(Y),
                                   rtol=0, atol=1e-9)


# --------------------------------------------------------------------------
# Boxcar S/N (Sec. 3.3, 3.4, 5.4)
# --------------------------------------------------------------------------

def test_injected_boxcar_along_a_path_returns_its_amplitude():
    # A boxcar pulse that follows path s exactly is a unit-square-sum template
    # times a; the fold plus matched boxcar recovers Z = a (Sec. 3.3, 3.4).
    g = rng(4)
    for (m, p, s, w, phi, a) in [(64, 50, 17, 3, 45, 7.5), (37, 101, 36, 6, 3, 12.0),
                                 (200, 64, 0, 1, 10, 5.0), (129, 33, 128, 9, 30, 20.0)]:
        D = oracle.path_table(m)
        X = np.zeros((m, p))
        h = a / math.sqrt(m * w)
        for r in range(m):
            for u in range(w):
                X[r, (phi + D[s, r] + u) % p] += h
        assert abs(np.sqrt((X ** 2).sum()) - a) < 1e-12
        F = oracle.fold_ffa(X)
        widths = [1, 2, 3, 4, 6, 9]
        snr = oracle.boxcar_snr(F, m, 1.0, widths)
        assert abs(snr[s, widths.index(w)] - a) < 1e-9
        # no other row or width can beat the matched template (Cauchy-Schwarz)
        assert snr.max() <= a + 1e-9


def test_noise_snr_has_the_law_of_the_max_of_p_gaussians():
    # For unit-variance noise, a width-1 boxcar value divided by sqrt(m) is
    # N(0, 1) (Sec. 3.3) and the p phases of one profile are independent, so
    # the width-1 S/N of a profile is the max of p standard normals:
    # P(snr <= x) = Phi(x)^p.
    g = rng(5)
    m, p = 16, 32
    vals = []
    for _ in range(1500):
        X = g.standard_normal((m, p))
        F = oracle.fold_ffa(X)
        vals.append(oracle.boxcar_snr(F[:1], m, 1.0, [1])[0, 0])
    vals = np.array(vals)
    ks = stats.kstest(vals, lambda x: stats.norm.cdf(x) ** p)
    assert ks.pvalue > 1e-3, ks
    # with a wrong variance scale the law fails
    ks_bad = stats.kstest(vals * math.sqrt(2.0), lambda x: stats.norm.cdf(x) ** p)
    assert ks_bad.pvalue < 1e-6


def test_noise_boxcar_values_are_standard_normal():
    # A phase bin summed over m periods and scaled by sqrt(m var) is N(0, 1),
    # also after a non-integer downsampling with var = ds - 1/3 (App. A.4): the
    # samples folded into one bin are p apart, hence uncorrelated (Sec. 5.3).
    # (Adjacent downsampled samples are correlated, so for w > 1 the boxcar
    # variance is slightly above w (ds - 1/3); the paper neglects this.)
    g = rng(6)
    vals = []
    ds = 3.37
    ds_fx = int(round(ds * 2 ** 32))
    var = ds_fx / 2 ** 32 - 1.0 / 3.0
    p, m, w = 40, 12, 1
    n = int(math.ceil((m * p + 2) * ds)) + 2
    for _ in range(2500):
        x = g.standard_normal(n)
        y = oracle.downsample(x, ds_fx, m * p)
        F = oracle.fold_ffa(y.reshape(m, p))
        vals.append(F[0, :w].sum() / math.sqrt(m * w * var))
    vals = np.array(vals)
    assert abs(vals.mean()) < 0.08
    assert abs(vals.std() - 1.0) < 0.05


def test_boxcar_efficiency_against_a_gaussian_pulse():
    # App. A.3: a boxcar of half-width u sigma recovers
    # E(u) = (pi/u^2)^(1/4) erf(u / sqrt 2) of the S/N of a Gaussian pulse;
    # peak 0.943 at u = 1.40 (w = 2.80 sigma). Checked on a finely sampled
    # profile (sigma = 40 bins) through the oracle's boxcar S/N.
    c = golden("paper_constants.txt")
    p, sigma = 4000, 40.0
    phase = np.arange(p) - p / 2 + 0.5
    prof = np.exp(-phase ** 2 / (2 * sigma ** 2))
    prof /= np.sqrt((prof ** 2).sum())          # unit square sum (Sec. 3.1)
    widths = list(range(20, 300, 2))
    snr = oracle.boxcar_snr(prof[None, :], 1, 1.0, widths)[0]
    u = np.array(widths) / (2 * sigma)
    E = (np.pi / u ** 2) ** 0.25 * special.erf(u / np.sqrt(2))
    np.testing.assert_allclose(snr, E, atol=2e-3)
    best = int(np.argmax(snr))
    assert abs(snr[best] - float(c["E_star"])) < 1e-3
    assert abs(widths[best] / sigma - float(c["w_star_over_sigma"])) < 0.06
    # worst case of a factor-2 grid is u* sqrt 2, average over [u*/sqrt2, u* sqrt2]
    ustar = float(c["u_star"])
    Ef = lambda uu: (np.pi / uu ** 2) ** 0.25 * special.erf(uu / np.sqrt(2))
    assert abs(Ef(ustar * math.sqrt(2)) - float(c["E_worst"])) < 1e-3
    uu = np.linspace(ustar / math.sqrt(2), ustar * math.sqrt(2), 20001)
    assert abs(np.trapezoid(Ef(uu), uu) / (uu[-1] - uu[0]) - float(c["E_avg"])) < 1e-3
    assert abs(1.0 / float(c["E_avg"]) - float(c["U_FFA_factor"])) < 1e-3


# --------------------------------------------------------------------------
# Downsampling (Sec. 5.3, App. A.4)
# --------------------------------------------------------------------------

def test_downsample_integer_factor_is_a_block_sum():
    x = rng(7).standard_normal(1000)
    for ds in [1, 2, 3, 7]:
        nout = 1000 // ds
        y = oracle.downsample(x, ds << 32, nout)
        np.testing.assert_allclose(y, x[:nout * ds].reshape(nout, ds).sum(axis=1), atol=1e-12)


def test_downsample_window_weights():
    # every window holds exactly ds samples of weight; windows tile the series
    for ds in [1.0, 1.5, 2.37, 32.552083333, 650.1]:
        ds_fx = int(math.floor(ds * 2 ** 32 + 0.5))
        n = 20000
        nout = (n << 32) // ds_fx
        y = oracle.downsample(np.ones(n), ds_fx, nout)
        np.testing.assert_allclose(y, ds_fx / 2 ** 32, rtol=1e-12)
        # a staircase x_i = i + 1/2 on [i, i+1) checks the overlap weighting:
        # window j is G(b) - G(a) with G(t) the integral of the staircase,
        # G(t) = floor(t)^2 / 2 + frac(t) (floor(t) + 1/2)
        z = oracle.downsample(np.arange(n) + 0.5, ds_fx, nout)
        def G(t_fx):
            fl = t_fx >> 32
            fr = (t_fx & 0xFFFFFFFF) / 2 ** 32
            return fl.astype(np.float64) ** 2 / 2 + fr * (fl + 0.5)
        aa = np.arange(nout, dtype=np.int64) * np.int64(ds_fx)
        np.testing.assert_allclose(z, G(aa + np.int64(ds_fx)) - G(aa), rtol=1e-9)


def test_downsample_variance_is_f_minus_one_third():
    # App. A.4: unit-variance white noise downsampled by a non-integer factor
    # f has sample variance f - 1/3; an integer factor gives f.
    c = golden("paper_constants.txt")
    off = float(c["downsample_var_offset"])
    x = rng(8).standard_normal(4_000_000)
    for f in [1.71, 2.5873, 3.37]:
        ds_fx = int(math.floor(f * 2 ** 32 + 0.5))
        y = oracle.downsample(x, ds_fx, (x.size << 32) // ds_fx)
        se = y.var() * math.sqrt(2.0 / y.size)
        assert abs(y.var() - (f - off)) < 5 * se, (f, y.var())
    y = oracle.downsample(x, 3 << 32, x.size // 3)
    assert abs(y.var() - 3.0) < 5 * 3.0 * math.sqrt(2.0 / y.size)


# --------------------------------------------------------------------------
# Period plan (Sec. 2.3, 5.3)
# --------------------------------------------------------------------------

def test_trial_periods_are_linear_in_frequency():
    # Eqs. for nu_s and P_s (Sec. 2.3): frequency steps are 1 / ((m-1) p^2 tau)
    # and the last trial lies beyond (p + 1) tau.
    for m, p, tau in [(1310, 200, 1.0), (53, 259, 64e-6 * 600.0), (2, 128, 1.0)]:
        s = np.arange(m)
        P = oracle.trial_period(s, m, p, tau)
        nu = 1.0 / P
        np.testing.assert_allclose(np.diff(nu), -1.0 / ((m - 1) * p * p * tau), rtol=1e-9)
        assert P[0] == p * tau
        assert P[-1] > (p + 1) * tau


def test_plan_single_octave_sample_units():
    # periods [128, 256) samples with 128..255 bins: ds0 = 1, f = 2, one octave
    o = oracle.plan(1.0, 128.0, 256.0, 128, 255, 262144)
    assert len(o) == 1
    assert o[0].ds_fx == 1 << 32 and o[0].var == 1.0 and o[0].nsamp == 262144
    assert [t.p for t in o[0].transforms] == list(range(128, 256))
    for t in o[0].transforms:
        assert t.m == 262144 // t.p
        # kept rows: P_s < (p + 1) tau, the rest overlap the next transform
        assert t.keep < t.m
        assert (t.periods < t.p + 1).all()
        assert oracle.trial_period(t.keep, t.m, t.p, 1.0) >= t.p + 1


def test_plan_covers_the_range_once_in_ascending_order():
    tsamp = 64e-6
    for (pmin, pmax, n) in [(0.5, 10.0, 9_375_000), (0.1, 1.0, 1 << 20), (1.0, 30.0, 1 << 22)]:
        octs = oracle.plan(tsamp, pmin, pmax, 240, 259, n)
        f = 260 / 240
        per = np.concatenate([t.periods for o in octs for t in o.transforms])
        assert per[0] == pytest.approx(pmin, rel=1e-9)
        assert (np.diff(per) > 0).all()
        assert per[-1] < pmax
        # octave k downsamples the original by ds0 f^k (Sec. 5.3, never chained)
        for k, o in enumerate(octs):
            assert o.ds == pytest.approx(pmin / (240 * tsamp) * f ** k, rel=1e-12)
            assert o.var == pytest.approx(o.ds_fx / 2 ** 32 - 1 / 3, rel=1e-15)
        # no gap wider than one trial step at the transform joins
        steps = np.diff(per) / per[1:]
        assert steps.max() < 2.5 / min(t.m for o in octs for t in o.transforms)


def test_plan_rejects_bad_parameters():
    with pytest.raises(oracle.PlanError):
        oracle.plan(1.0, 100.0, 256.0, 128, 255, 10000)   # ds0 < 1
    with pytest.raises(oracle.PlanError):
        oracle.plan(1.0, 256.0, 128.0, 128, 255, 10000)   # period_min > period_max
    with pytest.raises(oracle.PlanError):
        oracle.plan(1.0, 128.0, 256.0, 255, 128, 10000)   # bins_min > bins_max


def test_width_recurrence():
    # Sec. 5.4: w0 = 1, w_{k+1} = max(floor(f_sp w_k), w_k + 1), f_sp = 1.5
    c = golden("paper_constants.txt")
    w = [int(c["width_w0"])]
    while len(w) < 9:
        w.append(max(int(math.floor(float(c["width_fsp"]) * w[-1])), w[-1] + 1))
    import synth
    assert tuple(w) == synth.WIDTHS_PAPER


# --------------------------------------------------------------------------
# Whole search
# --------------------------------------------------------------------------

def test_search_finds_a_pulse_at_an_exact_trial_period():
    # Noise-free boxcar pulse train of period exactly p samples: row s = 0 of
    # transform p, S/N = its amplitude at the matched width.
    n, p, w, a = 64 * 150, 150, 3, 9.0
    m = n // p
    x = np.zeros(n)
    h = a / math.sqrt(m * w)
    for r in range(m):
        x[r * p + 40: r * p + 40 + w] = h
    pg = oracle.search(x, 1.0, 100.0, 200.0, 100, 199, [1, 2, 3, 4, 6], normalise=False)
    sel = (pg.bins == p) & (pg.s == 0)
    assert sel.sum() == 1
    assert abs(pg.snr[sel][0, 2] - a) < 1e-9
    assert pg.snr.max() <= a + 1e-9
    assert pg.periods[sel][0] == 150.0


def test_search_bruteforce_and_ffa_agree():
    g = rng(9)
    x = g.standard_normal(6000)
    kw = dict(tsamp=1.0, period_min=40.0, period_max=160.0, bins_min=40, bins_max=47,
              widths=[1, 2, 3, 5])
    a = oracle.search(x, **kw)
    b = oracle.search(x, **kw, brute=True)
    np.testing.assert_allclose(a.snr, b.snr, rtol=0, atol=1e-10)
    assert np.array_equal(a.periods, b.periods)
    assert len(set(a.octave.tolist())) > 2


def test_tie_reading_is_half_up():
    # The paper rounds i and j "to the nearest integer" without a tie rule.
    # This build reads it as half-up (ties are common for odd row counts); no
    # passage decides it, so this test guards the reading rather than pins it.
    # n = 5, s = 2: i = nint(1 * 2 / 4) = nint(0.5) -> 1, j = nint(2 * 2 / 4) = 1,
    # b = 0, so the tail rows are reached after a rotation by s - j = 1.
    assert oracle.path_offset(5, 2, 0) == 0
    assert oracle.path_offset(5, 2, 1) == 1   # head row 1 reached through H_1
    assert oracle.path_offset(5, 2, 2) == 1   # first tail row: rotation s - j = 1


# --------------------------------------------------------------------------
# Dynamic duty-cycle resolution (Sec. 5.6)
# --------------------------------------------------------------------------

def test_sub_ranges_resolve_a_narrow_pulse_better():
    # Sec. 5.6: more phase bins at longer periods raise the duty-cycle
    # resolution there. A 2-sample boxcar pulse at period 700.37 samples is
    # smeared over 4-sample bins with 128..255 bins per profile; a second
    # sub-range [256, 1024) with 256..511 bins has 2-sample bins there, so its
    # best S/N near the pulse period is clearly higher (16.7 against 12.3 for
    # an amplitude of 25; the rest is lost to the 1-bin phase and drift steps).
    n = 1 << 18
    period, a = 700.37, 25.0
    t = np.arange(n, dtype=np.float64)
    ph = np.mod(t / period, 1.0) * period
    s = ((ph >= 100.0) & (ph < 102.0)).astype(np.float64)
    s /= np.sqrt(np.sum(s * s))
    x = a * s + 1e-3 * rng(61).standard_normal(n)
    widths = (1, 2, 3, 4)
    coarse = oracle.search(x, 1.0, 128.0, 1024.0, 128, 255, widths, normalise=False)
    fine = oracle.search_ranges(x, 1.0, [(128.0, 256.0, 128, 255), (256.0, 1024.0, 256, 511)],
                                widths, normalise=False)
    # the concatenation: ascending periods inside [128, 1024), each part its own search
    assert np.all(np.diff(fine.periods) > 0)
    assert fine.periods[0] >= 128.0 and fine.periods[-1] < 1024.0
    first = oracle.search(x, 1.0, 128.0, 256.0, 128, 255, widths, normalise=False)
    k = first.periods.size
    assert np.array_equal(fine.snr[:k], first.snr) and np.all(fine.periods[k:] >= 256.0)
    near = lambda pg: pg.snr[np.abs(pg.periods - period) < 1.0].max()
    assert near(fine) > near(coarse) + 3.0
    assert near(fine) > 0.6 * a
    with pytest.raises(oracle.PlanError):
        oracle.search_ranges(x, 1.0, [(128.0, 300.0, 128, 255), (256.0, 1024.0, 256, 511)],
                             widths, normalise=False)


# --------------------------------------------------------------------------
# Normalisation (Sec. 5.2): zero mean and unit standard deviation of the whole
# raw series, before any downsampling (reading c13: population std, FP64)
# --------------------------------------------------------------------------

def test_normalise_stats_hand_values():
    # [1, 2, 3, 4]: mean 2.5, squared deviations 2.25 + 0.25 + 0.25 + 2.25 = 5,
    # population variance 5 / 4 = 1.25 (the sample variance would be 5 / 3)
    mu, sigma = oracle.normalise_stats(np.array([1.0, 2.0, 3.0, 4.0]))
    assert mu == 2.5
    assert sigma == math.sqrt(1.25)
    # a constant offset and a scale pass straight through
    mu, sigma = oracle.normalise_stats(np.array([-7.0, 13.0]))
    assert (mu, sigma) == (3.0, 10.0)


def test_search_normalise_hand_worked_snr():
    # Raw period of 16 samples: two samples of height h, fourteen of c. Zero
    # mean needs 2h + 14c = 0 (c = -h/7); unit population variance needs
    # (2h^2 + 14c^2)/16 = h^2/7 = 1, so h = sqrt(7). The series given to the
    # search is 5 + 3 z, so normalising must recover z exactly in form.
    # Plan (tsamp 1, P 16..17, 8 bins): ds0 = 16/8 = 2, an integer factor, so
    # the downsampled series is the pair sums [2h, 2c, ..., 2c] with noise
    # variance 2 (App. A.4), and the one transform has p = 8, m = N/16 rows.
    # Row s = 0 does not drift: bin 0 sums to 2hm and the other bins to 2cm.
    #   width 1: 2hm / sqrt(2m) = sqrt(14 m)
    #   width 2: (2h + 2c) m / sqrt(2 * 2m) = (h + c) sqrt(m) = sqrt(36 m / 7)
    # Normalising after downsampling, or by the sample std, gives other values.
    m = 10
    h = math.sqrt(7.0)
    c = -h / 7.0
    period = np.array([h, h] + [c] * 14)
    z = np.tile(period, m)
    x = 5.0 + 3.0 * z
    res = oracle.search(x, 1.0, 16.0, 17.0, 8, 8, (1, 2), normalise=True)
    assert res.periods[0] == 16.0 and res.bins[0] == 8 and res.rows_m[0] == m
    assert res.snr[0, 0] == pytest.approx(math.sqrt(14.0 * m), rel=1e-12)
    assert res.snr[0, 1] == pytest.approx(math.sqrt(36.0 * m / 7.0), rel=1e-12)
    # the same series already normalised gives the same periodogram
    res0 = oracle.search(z, 1.0, 16.0, 17.0, 8, 8, (1, 2), normalise=False)
    assert np.allclose(res.snr, res0.snr, rtol=1e-12, atol=1e-12)
