"""GPU parity of the periodogram peak detection (Sec. 5.5) against the oracle.

Both sides read the same FP32 S/N array. The bar: identical peak lists
(series, width, row, member count, S/N) and thresholds within
1e-9 * max(1, |threshold|) (both FP64; the least-squares solutions differ by
rounding only). Every test input is checked to have no S/N within that band of
the oracle's threshold, so no selection decision is ambiguous.
"""
import numpy as np
import pytest

import oracle
from oracle import peaks as pk
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2004_03701_amd as ffa  # noqa: E402

THR_RTOL = 1e-9


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = ffa.ffa_create(0)
    yield c
    ffa.ffa_destroy(c)


def oracle_periods(prm, nsamp):
    octs = oracle.plan(prm.tsamp, prm.period_min, prm.period_max, prm.bins_min, prm.bins_max,
                       nsamp)
    return np.concatenate([t.periods for o in octs for t in o.transforms if t.keep])


def to_oracle_params(pp):
    return pk.PeakParams(dz_seg=pp.dz_seg, k_sigma=pp.k_sigma, degree=pp.degree,
                         cluster_gap=pp.cluster_gap, min_points=pp.min_points)


def check_against_oracle(got, counts, poly, snr_host, row_offset, prms, nsamps, pp):
    """Runs the oracle on every series' rows of snr_host and compares."""
    for s, (prm, n) in enumerate(zip(prms, nsamps)):
        per = oracle_periods(prm, n)
        rows = per.size
        S = snr_host[row_offset[s]:row_offset[s] + rows].astype(np.float64)
        ref, coefs, _ = pk.find_peaks(per, S, n, prm.tsamp, to_oracle_params(pp))
        x = np.log(1.0 / per)
        for w, c in enumerate(coefs):
            if c is None:
                assert np.all(np.isnan(poly[s, w])), (s, w)
                continue
            thr = pk.threshold(c, x)
            band = THR_RTOL * np.maximum(1.0, np.abs(thr))
            amb = np.abs(S[:, w] - thr) <= band
            assert not amb.any(), f"ambiguous test input: series {s} width {w}"
            thr_gpu = np.polynomial.polynomial.polyval(x, poly[s, w])
            assert np.max(np.abs(thr_gpu - thr) / np.maximum(1.0, np.abs(thr))) < 1e-7, (s, w)
        mine = got[got["series"] == s]
        want = [(p.width_index, p.row, p.members, p.snr) for p in ref]
        have = [(int(q["width_index"]), int(q["row"]), int(q["members"]), float(q["snr"]))
                for q in mine]
        assert have == want, f"series {s}: {have[:5]} vs {want[:5]}"
        assert counts[s] == len(want)
        for q, p in zip(mine, ref):
            assert abs(q["threshold"] - p.threshold) <= THR_RTOL * max(1.0, abs(p.threshold))
            assert q["period"] == p.period
    return True


def small_params():
    return ffa.make_params(1.0, 128.0, 256.0, 128, 255, (1, 2, 3), normalise=False)


def constructed_snr(per, which):
    """S/N of one series on the 2^18-sample single-octave plan: N(3, 0.5) noise
    with injected clusters (which = 0), or every segment an exact ramp around
    a quadratic in log frequency in width 0 and one injected row in width 1
    (which = 1)."""
    g = np.random.Generator(np.random.Philox(9100 + which))
    S = 3.0 + 0.5 * g.standard_normal((per.size, 3))
    if which == 0:
        S[5000:5004, 1] = [12.0, 15.0, 13.0, 11.0]
        S[90000, 1] = 10.0
        S[120000, 2] = 9.5
        S[150000:150002, 0] = [8.0, 8.0]  # equal S/N: the first row is the peak
    else:
        nu, nu_lo, dnu, seg = pk.segment_index(per, float(1 << 18), 4.0)
        G = np.array([1.5, -0.75, 0.125])
        for i in np.unique(seg):
            idx = np.flatnonzero(seg == i)
            xc = np.log(nu_lo + (i + 0.5) * dnu)
            S[idx, 0] = np.polynomial.polynomial.polyval(xc, G) + g.permutation(
                np.linspace(-1.0, 1.0, idx.size))
        S[70000, 1] += 20.0
    return S.astype(np.float32)


def test_peaks_of_constructed_periodograms(ctx):
    print("peaks: constructed periodograms, 2 series, 3 widths", flush=True)
    prm = small_params()
    n = 1 << 18
    per = oracle_periods(prm, n)
    rows = per.size
    row_offset = [0, rows + 7]
    host = np.full((2 * rows + 7, 3), np.nan, dtype=np.float32)
    host[0:rows] = constructed_snr(per, 0)
    host[rows + 7:] = constructed_snr(per, 1)
    snr = torch.from_numpy(host).cuda()
    pp = ffa.make_peak_params()
    got, counts, poly = ffa.ffa_find_peaks_batch(ctx, snr, [prm, prm], [n, n], row_offset, pp)
    check_against_oracle(got, counts, poly, host, row_offset, [prm, prm], [n, n], pp)
    # the injected peaks themselves (independent of the oracle)
    s0 = got[got["series"] == 0]
    assert [(int(q["width_index"]), int(q["row"]), int(q["members"])) for q in s0] == \
        [(0, 150000, 2), (1, 5001, 4), (1, 90000, 1), (2, 120000, 1)]
    s1 = got[got["series"] == 1]
    assert [(int(q["width_index"]), int(q["row"])) for q in s1] == [(1, 70000)]
    # the exact construction's threshold is G + k / 1.349 (up to the FP32
    # rounding of the stored S/N)
    x = np.log(1.0 / per)
    want = np.polynomial.polynomial.polyval(x, [1.5 + 6.0 / 1.349, -0.75, 0.125])
    assert np.max(np.abs(np.polynomial.polynomial.polyval(x, poly[1, 0]) - want)) < 1e-4


@pytest.mark.parametrize("nw", [13, 32])
def test_peaks_with_many_widths(ctx, nw):
    # more than 12 widths: one wave per (segment, width) instead of one
    # workgroup per segment; 32 widths: two load batches in the selection
    prm = ffa.make_params(1.0, 128.0, 256.0, 128, 255, tuple(range(1, nw + 1)), normalise=False)
    n = 1 << 18
    per = oracle_periods(prm, n)
    g = np.random.Generator(np.random.Philox(9300 + nw))
    host = (3.0 + 0.5 * g.standard_normal((per.size, nw))).astype(np.float32)
    host[4000:4003, nw - 1] = [11.0, 14.0, 12.0]
    host[100000, 5] = 10.0
    print(f"peaks: {nw} widths", flush=True)
    snr = torch.from_numpy(host).cuda()
    pp = ffa.make_peak_params()
    got, counts, poly = ffa.ffa_find_peaks_batch(ctx, snr, [prm], [n], [0], pp)
    check_against_oracle(got, counts, poly, host, [0], [prm], [n], pp)
    assert {(int(q["width_index"]), int(q["row"])) for q in got} >= {(nw - 1, 4001), (5, 100000)}


@pytest.mark.parametrize("dz_seg", [6.0, 10.0, 30.0])
def test_peaks_with_larger_segments(ctx, dz_seg):
    # segments of 1025 .. 2048 rows take the two-wave sort, larger ones the
    # workgroup (LDS) sort, smaller ones the one-wave register sort
    prm = small_params()
    n = 1 << 18
    per = oracle_periods(prm, n)
    sizes = np.bincount(pk.segment_index(per, float(n), dz_seg)[3])
    print(f"peaks: dz_seg {dz_seg}, segment rows {sizes.min()}..{sizes.max()}", flush=True)
    assert sizes.max() > 1024 and sizes.max() <= 8192
    host = constructed_snr(per, 0)
    snr = torch.from_numpy(host).cuda()
    pp = ffa.make_peak_params(dz_seg=dz_seg, k_sigma=5.0)
    got, counts, poly = ffa.ffa_find_peaks_batch(ctx, snr, [prm], [n], [0], pp)
    check_against_oracle(got, counts, poly, host, [0], [prm], [n], pp)
    assert counts[0] >= 4


@pytest.mark.parametrize("pp_args", [dict(), dict(dz_seg=2.0, k_sigma=4.0, degree=1,
                                                  min_points=64, cluster_gap=3.0),
                                     dict(degree=4, k_sigma=3.0, cluster_gap=0.0)])
def test_peaks_of_searched_periodograms(ctx, pp_args):
    # periodograms written by the GPU search: two pulsed workload-3 series
    # and a noise series of 2^22 samples, and one of 2^21 (a second plan)
    cfg = synth.workload3_config()
    pulsed = synth.workload3_pulsed()
    quiet = next(i for i in range(synth.WL3_SERIES) if i not in set(pulsed.tolist()))
    idx = [int(pulsed[0]), int(pulsed[1]), quiet, int(pulsed[2])]
    nsamps = [1 << 22, 1 << 22, 1 << 22, 1 << 21]
    print(f"peaks: searched periodograms {idx} {pp_args}", flush=True)
    xs = [synth.workload3_series(i, nsamp=n, pulsed=pulsed)[0] for i, n in zip(idx, nsamps)]
    prms = [ffa.make_params(cfg.tsamp, cfg.period_min, cfg.period_max, cfg.bins_min,
                            cfg.bins_max, cfg.widths) for _ in xs]
    series = [torch.from_numpy(x.astype(np.float32)).cuda() for x in xs]
    snr, row_offset = ffa.ffa_search_batch(ctx, series, prms)
    pp = ffa.make_peak_params(**pp_args)
    got, counts, poly = ffa.ffa_find_peaks_batch(ctx, snr, prms, nsamps, row_offset, pp)
    host = snr.cpu().numpy()
    print(f"peaks per series {counts.tolist()}", flush=True)
    check_against_oracle(got, counts, poly, host, row_offset, prms, nsamps, pp)


def test_peaks_full_size_batch(ctx):
    # the bench's shape: full 2^23-sample workload-3 series in one batch
    # (here 8, two of them pulsed), default peak parameters; three series
    # checked against the oracle
    cfg = synth.workload3_config()
    pulsed = synth.workload3_pulsed()
    quiet = [i for i in range(synth.WL3_SERIES) if i not in set(pulsed.tolist())][:6]
    idx = [int(pulsed[3]), quiet[0], int(pulsed[4])] + quiet[1:6]
    print(f"peaks: full-size batch {idx}", flush=True)
    xs = [synth.workload3_series(i, pulsed=pulsed)[0] for i in idx]
    prms = [ffa.make_params(cfg.tsamp, cfg.period_min, cfg.period_max, cfg.bins_min,
                            cfg.bins_max, cfg.widths) for _ in xs]
    series = [torch.from_numpy(x.astype(np.float32)).cuda() for x in xs]
    n = synth.WL3_NSAMP
    snr, row_offset = ffa.ffa_search_batch(ctx, series, prms)
    pp = ffa.make_peak_params()
    got, counts, poly = ffa.ffa_find_peaks_batch(ctx, snr, prms, [n] * len(xs), row_offset, pp)
    host = snr.cpu().numpy()
    print(f"peaks per series {counts.tolist()}", flush=True)
    pick = [0, 1, 2]
    sub = got[np.isin(got["series"], pick)]
    check_against_oracle(sub, counts[pick], poly[pick], host, [row_offset[i] for i in pick],
                         [prms[i] for i in pick], [n] * len(pick), pp)


def test_peak_capacity_degenerate_and_errors(ctx):
    print("peaks: capacity, NaN periodogram, argument errors", flush=True)
    prm = small_params()
    n = 1 << 18
    per = oracle_periods(prm, n)
    rows = per.size
    host = np.concatenate([constructed_snr(per, 0), np.full((rows, 3), np.nan, np.float32)])
    snr = torch.from_numpy(host).cuda()
    ro = [0, rows]
    got, counts, poly = ffa.ffa_find_peaks_batch(ctx, snr, [prm, prm], [n, n], ro)
    assert counts[1] == 0 and np.all(np.isnan(poly[1]))   # no control point anywhere
    assert counts[0] == 4
    # too small a buffer: the error, with the counts still reported
    with pytest.raises(ffa.FFAError) as e:
        ffa.ffa_find_peaks_batch(ctx, snr, [prm, prm], [n, n], ro, capacity=3)
    assert e.value.status == ffa.FFA_ERR_BUFFER_TOO_SMALL
    # segments larger than the LDS sort holds, a bad degree, rows past the array
    for bad in (dict(dz_seg=100.0), dict(degree=5), dict(min_points=0), dict(dz_seg=0.0)):
        with pytest.raises(ffa.FFAError) as e:
            ffa.ffa_find_peaks_batch(ctx, snr, [prm], [n], [0], ffa.make_peak_params(**bad))
        assert e.value.status == ffa.FFA_ERR_INVALID_ARG, bad
    with pytest.raises(ffa.FFAError) as e:
        ffa.ffa_find_peaks_batch(ctx, snr, [prm], [n], [rows + 1])
    assert e.value.status == ffa.FFA_ERR_INVALID_ARG
    # too few control points for the degree: no threshold, no peaks
    got, counts, poly = ffa.ffa_find_peaks_batch(ctx, snr, [prm], [n], [0],
                                                 ffa.make_peak_params(min_points=10 ** 6))
    assert counts[0] == 0 and np.all(np.isnan(poly))


def test_multi_dm_chain_on_search_output(ctx):
    # Sec. 5.7 end to end: one pulsar seen in 8 DM trials with an S/N that
    # peaks at the right DM; the periodograms' peaks of all trials are
    # clustered in frequency and the clusters flagged as harmonics. The
    # brightest cluster is the pulsar's frequency, its brightest member comes
    # from the brightest trial, and the flags satisfy their definition on the
    # clusters the chain produced.
    n, tsamp = 1 << 20, 64e-6
    T = n * tsamp
    period_s = 0.7131
    amps = [4.0, 8.0, 12.0, 16.0, 20.0, 16.0, 12.0, 8.0]
    xs = []
    for i, a in enumerate(amps):
        g = synth.rng(23, i)
        pu = synth.Pulse(period=period_s / tsamp, duty=0.03, amplitude=a, phi0=0.25)
        xs.append(torch.from_numpy(synth.inject(synth.noise(n, g), pu)).cuda())
    prm = [ffa.make_params(tsamp, 0.2, 2.0, 240, 259, synth.WIDTHS_DUTY) for _ in amps]
    snr, offs = ffa.ffa_search_batch(ctx, xs, prm)
    torch.cuda.synchronize()
    peaks, counts, _ = ffa.ffa_find_peaks_batch(ctx, snr, prm, [n] * len(amps), offs)
    assert counts.sum() > 0
    freq = 1.0 / peaks["period"]
    tol = 1.0 / T
    cl, br, mb = ffa.ffa_cluster_frequencies(freq, peaks["snr"], tol)
    cf, cs = freq[br], peaks["snr"][br]
    top = int(np.argmax(cs))
    assert abs(cf[top] - 1.0 / period_s) <= 2 * tol
    assert peaks["series"][br[top]] == int(np.argmax(amps))
    par, num, den = ffa.ffa_flag_harmonics(cf, cs, tol, 8)
    assert par[top] == -1
    for j in range(len(cf)):
        if par[j] < 0:
            continue
        i, a, b = int(par[j]), int(num[j]), int(den[j])
        assert cs[i] > cs[j] or (cs[i] == cs[j] and i < j)
        assert abs(cf[j] - a / b * cf[i]) <= tol * (1 + a / b)
    # the pulsar's harmonics that the search found are flagged against it
    for j in range(len(cf)):
        for a in (2, 3):
            if j != top and abs(cf[j] - a * cf[top]) <= tol * (1 + a) and cs[j] < cs[top]:
                assert par[j] >= 0
