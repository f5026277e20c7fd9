"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bars: the folding transform is bit-exact on integer-valued inputs (every FP32
partial sum is then an exact integer); S/N agrees within
1e-4 * max(1, |oracle|) in FP32; statistics and downsampling within stated
FP32/FP64 rounding bounds.
"""
import math

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2004_03701_amd as ffa  # noqa: E402

SNR_RTOL = 1e-4


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = ffa.ffa_create(0)
    yield c
    ffa.ffa_destroy(c)


def dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def snr_close(gpu, ref, rtol=SNR_RTOL):
    gpu = np.asarray(gpu, dtype=np.float64)
    err = np.abs(gpu - ref) / np.maximum(1.0, np.abs(ref))
    return float(err.max()) if err.size else 0.0


# ---------------------------------------------------------------------------
# Folding transform, bit-exact on integers
# ---------------------------------------------------------------------------

TRANSFORM_SHAPES = [
    (1, 7), (2, 2), (2, 3), (3, 5), (5, 17), (8, 6), (37, 128), (64, 255), (100, 259),
    (129, 259), (130, 259), (131, 259), (257, 240), (1000, 251), (1073, 259), (1310, 200),
    (2048, 128), (3001, 97), (12000, 33), (500, 1000), (300, 1280), (41, 2),
    # wide rows whose tiles hold few rows: the range passes take fewer levels
    (200, 1280), (500, 600), (497, 519),
]


@pytest.mark.parametrize("m,p", TRANSFORM_SHAPES)
def test_transform_bit_exact_on_integers(ctx, m, p):
    print(f"transform m={m} p={p}", flush=True)
    g = np.random.default_rng(1000 * m + p)
    X = g.integers(-8, 9, size=(m, p)).astype(np.float64)
    ref = oracle.fold_ffa(X)
    out = ffa.ffa_transform(ctx, dev(X))
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().astype(np.float64), ref)


@pytest.mark.parametrize("lds_rows,levels,waves", [(16, 1, 16), (16, 2, 16), (24, 3, 16),
                                                   (40, 4, 16), (0, 2, 16), (0, 4, 8),
                                                   (16, 1, 8), (16, 5, 8), (0, 5, 16)])
def test_transform_tilings_agree(ctx, lds_rows, levels, waves):
    m, p = 1500, 61
    g = np.random.default_rng(7)
    X = g.integers(-8, 9, size=(m, p)).astype(np.float64)
    ref = oracle.fold_ffa(X)
    ffa.ffa_set_tiling(ctx, lds_rows, levels, waves_per_group=waves)
    try:
        out = ffa.ffa_transform(ctx, dev(X))
        torch.cuda.synchronize()
    finally:
        ffa.ffa_set_tiling(ctx)
    assert np.array_equal(out.cpu().numpy().astype(np.float64), ref)


def test_transform_noise_fp32(ctx):
    m, p = 1073, 259
    X = np.random.default_rng(3).standard_normal((m, p)).astype(np.float32)
    ref = oracle.fold_ffa(X.astype(np.float64))
    out = ffa.ffa_transform(ctx, dev(X)).cpu().numpy()
    # 11 FP32 additions per output: relative error well under 1e-5 of sqrt(m)
    assert np.abs(out - ref).max() < 1e-5 * math.sqrt(m) * 4


# ---------------------------------------------------------------------------
# Statistics and downsampling
# ---------------------------------------------------------------------------

def test_series_stats(ctx):
    x = (np.random.default_rng(4).standard_normal(1_000_003) * 3.0 + 17.0).astype(np.float32)
    st = ffa.ffa_series_stats(ctx, dev(x)).cpu().numpy()
    mu, sd = oracle.normalise_stats(x)
    assert abs(st[0] - mu) < 1e-12 * abs(mu) + 1e-12
    assert abs(st[1] - sd) < 1e-11 * sd


def check_downsampled(y, xn, ds_fx, ref, out_ulp):
    """Downsampled output against the oracle, to a bound taken from the FP32
    arithmetic of the prefix-sum method.

    A block keeps the exclusive prefix sum P of its stretch (at most 32768
    samples) in FP32; every P carries at most ~40 roundings, each no larger than
    half an ulp of the largest |P| of the block, and an output combines four P
    values with weights of at most 2. |P| is bounded by the range of the
    series' cumulative sum within 32768 samples either side of the window.
    Element by element the error stays within that worst case; its RMS must
    stay near the few roundings of a typical P, which the bound exceeds
    fifty-fold, so an accumulation without the per-block restart would fail.
    The output is then rounded to its storage type (out_ulp: half an ulp,
    relative).
    """
    from scipy.ndimage import maximum_filter1d, minimum_filter1d
    span = 32768
    cs = np.concatenate([[0.0], np.cumsum(xn)])
    rng = maximum_filter1d(cs, 2 * span + 1) - minimum_filter1d(cs, 2 * span + 1)
    start = (np.arange(len(ref), dtype=np.float64) * (ds_fx / 2.0 ** 32)).astype(np.int64)
    prange = rng[np.minimum(start, len(cs) - 1)]
    err = np.abs(y - ref)
    worst = 256 * 2.0 ** -24 * prange + out_ulp * np.abs(ref) + 1e-7
    assert np.all(err <= worst), (err - worst).max()
    rms_allow = 5 * 2.0 ** -24 * np.sqrt(np.mean(prange ** 2)) + out_ulp * np.sqrt(np.mean(ref ** 2))
    assert np.sqrt(np.mean(err ** 2)) <= rms_allow


@pytest.mark.parametrize("ds", [1.0, 3.0, 1.37, 32.552083333333336, 651.04, 2000.3, 5000.3, 16000.3])
def test_downsample(ctx, ds):
    n = 300_001
    x = (np.random.default_rng(5).standard_normal(n) + 0.3).astype(np.float32)
    ds_fx = int(math.floor(ds * 2 ** 32 + 0.5))
    nout = (n << 32) // ds_fx
    xd = dev(x)
    st = ffa.ffa_series_stats(ctx, xd)
    y = ffa.ffa_downsample(ctx, xd, ds_fx, nout, stats=st).cpu().numpy().astype(np.float64)
    mu, sd = oracle.normalise_stats(x)
    xn = (x.astype(np.float64) - mu) / sd
    check_downsampled(y, xn, ds_fx, oracle.downsample(xn, ds_fx, nout), 0.0)


@pytest.mark.parametrize("ds", [651.04, 5000.3, 16000.3])
def test_downsample_large_mean(ctx, ds):
    # a series far from zero mean: the FP32 mean the samples are shifted by
    # is off by up to half its ulp, which would bias every window by that
    # times its length; the kernel drops the residual per window, so the
    # outputs meet the same bound as a zero-mean series
    n = 300_001
    x = (1000.0 + np.random.default_rng(6).standard_normal(n)).astype(np.float32)
    ds_fx = int(math.floor(ds * 2 ** 32 + 0.5))
    nout = (n << 32) // ds_fx
    xd = dev(x)
    st = ffa.ffa_series_stats(ctx, xd)
    y = ffa.ffa_downsample(ctx, xd, ds_fx, nout, stats=st).cpu().numpy().astype(np.float64)
    mu, sd = oracle.normalise_stats(x)
    assert abs(float(np.float32(mu)) - mu) * ds / sd > 1e-3  # the residual the kernel corrects
    xn = (x.astype(np.float64) - mu) / sd
    check_downsampled(y, xn, ds_fx, oracle.downsample(xn, ds_fx, nout), 0.0)


@pytest.mark.parametrize("tdt,dt", [(torch.float32, ffa.FFA_F32), (torch.bfloat16, ffa.FFA_BF16),
                                     (torch.float16, ffa.FFA_F16)])
@pytest.mark.parametrize("offset", [0, 1, 3])
@pytest.mark.parametrize("ds", [1.0, 2.7, 651.04, 5000.3])
def test_downsample_storage_types_and_alignment(ctx, tdt, dt, offset, ds):
    # 16-byte loads take aligned series; a series that starts off a 16-byte
    # boundary (offset > 0), or a ragged end, loads per sample
    n = 200_003
    base = torch.from_numpy(np.random.default_rng(9).standard_normal(n + offset).astype(np.float32))
    xs = base.to(tdt)
    x = xs.float().numpy()[offset:].astype(np.float64)
    xd = xs.cuda()[offset:]
    ds_fx = int(math.floor(ds * 2 ** 32 + 0.5))
    nout = (n << 32) // ds_fx
    st = ffa.ffa_series_stats(ctx, xd, dtype=dt)
    y = ffa.ffa_downsample(ctx, xd, ds_fx, nout, stats=st, dtype=dt).float().cpu().numpy()
    mu, sd = oracle.normalise_stats(x)
    xn = (x - mu) / sd
    ulp = {torch.float32: 0.0, torch.bfloat16: 2.0 ** -8, torch.float16: 2.0 ** -11}[tdt]
    check_downsampled(y.astype(np.float64), xn, ds_fx, oracle.downsample(xn, ds_fx, nout), ulp)


def test_downsample_unaligned_output_is_refused(ctx):
    n = 10_000
    xd = dev(np.random.default_rng(2).standard_normal(n).astype(np.float32))
    out = torch.empty(n, dtype=torch.float32, device="cuda")
    st = ffa.lib().ffa_downsample(ctx, xd.data_ptr(), n, ffa.FFA_F32, None, 1 << 32, 100,
                                  out.data_ptr() + 4, None)
    assert st == ffa.FFA_ERR_INVALID_ARG


def test_downsample_factor_beyond_block_is_refused(ctx):
    # a window longer than a downsampling block can hold is an argument error
    n = 100_000
    xd = dev(np.random.default_rng(2).standard_normal(n).astype(np.float32))
    ds_fx = 20_000 << 32
    with pytest.raises(RuntimeError):
        ffa.ffa_downsample(ctx, xd, ds_fx, n // 20_000)


def test_downsample_widest_window_boundary(ctx):
    # the halo, floor(ds) + 2 samples padded to 8, and the block must fill at
    # most two LDS rounds of 16,384 samples with the block at least as long as
    # the halo: floor(ds) = 16,382 is the widest accepted, and its outputs
    # still match the oracle; 16,383 is refused
    n = 200_000
    x = np.random.default_rng(4).standard_normal(n).astype(np.float32)
    xd = dev(x)
    ds_fx = (16_382 << 32) + (1 << 31)
    nout = (n << 32) // ds_fx
    y = ffa.ffa_downsample(ctx, xd, ds_fx, nout).cpu().numpy().astype(np.float64)
    xn = x.astype(np.float64)
    check_downsampled(y, xn, ds_fx, oracle.downsample(xn, ds_fx, nout), 0.0)
    with pytest.raises(RuntimeError):
        ffa.ffa_downsample(ctx, xd, 16_383 << 32, n // 16_383)


# ---------------------------------------------------------------------------
# Whole search
# ---------------------------------------------------------------------------

def run_search(ctx, x, cfg, normalise=True, dtype=ffa.FFA_F32, tdtype=torch.float32):
    prm = ffa.make_params(cfg.tsamp, cfg.period_min, cfg.period_max, cfg.bins_min, cfg.bins_max,
                          cfg.widths, normalise=normalise, dtype=dtype,
                          median_window=cfg.median_window)
    per, bins, snr = ffa.ffa_search(ctx, dev(x, tdtype), prm)
    torch.cuda.synchronize()
    return per, bins, snr.cpu().numpy()


def test_search_small_multi_octave(ctx):
    x = np.random.default_rng(6).standard_normal(20_000).astype(np.float32)
    cfg = synth.SearchConfig(1.0, 40.0, 400.0, 40, 47, (1, 2, 3, 5, 8))
    per, bins, snr = run_search(ctx, x, cfg)
    ref = oracle.search(x, 1.0, 40.0, 400.0, 40, 47, cfg.widths)
    assert np.array_equal(per, ref.periods) and np.array_equal(bins, ref.bins)
    assert snr_close(snr, ref.snr) < SNR_RTOL


# Each S/N form against the oracle: the compiled width grids in their
# register-window form (p large enough), in their ring form (short rows), and
# general widths; with a pulse so that the maxima are not all noise.
@pytest.mark.parametrize("widths,bmin,bmax,pmin", [
    ((1, 2, 3, 4, 6, 9, 13, 19, 28), 40, 47, 40.0),     # paper grid, ring form
    ((1, 2, 3, 4, 6, 9, 13, 19, 28), 96, 103, 96.0),    # paper grid, register windows
    ((1, 2, 3, 5, 8, 12, 19, 30, 48), 60, 67, 60.0),    # duty grid, ring form
    ((1, 2, 3, 5, 8, 12, 19, 30, 48), 120, 127, 120.0),  # duty grid, register windows
    ((1, 2, 5, 7, 11), 100, 107, 100.0),                 # general widths
])
def test_snr_forms_match_oracle(ctx, widths, bmin, bmax, pmin):
    g = synth.rng(11, bmin)
    x = synth.inject(synth.noise(60_000, g),
                     synth.Pulse(period=pmin * 1.37, duty=0.05, amplitude=12.0, phi0=0.3))
    cfg = synth.SearchConfig(1.0, pmin, pmin * 4.0, bmin, bmax, widths)
    per, bins, snr = run_search(ctx, x, cfg)
    ref = oracle.search(x, 1.0, pmin, pmin * 4.0, bmin, bmax, widths)
    assert np.array_equal(per, ref.periods) and np.array_equal(bins, ref.bins)
    assert snr_close(snr, ref.snr) < SNR_RTOL
    assert float(np.max(ref.snr)) > 8.0  # the pulse is found


def test_search_integer_series_matches_closely(ctx):
    # integer samples, ds = 1, no normalisation: boxcar sums are exact
    x = np.random.default_rng(8).integers(-8, 9, size=40_000).astype(np.float32)
    cfg = synth.SearchConfig(1.0, 64.0, 128.0, 64, 127, (1, 2, 3, 4, 6, 9))
    per, bins, snr = run_search(ctx, x, cfg, normalise=False)
    ref = oracle.search(x, 1.0, 64.0, 128.0, 64, 127, cfg.widths, normalise=False)
    assert snr_close(snr, ref.snr) < 1e-6


def test_search_workload1_full(ctx):
    x, cfg, pulses = synth.workload1()
    per, bins, snr = run_search(ctx, x, cfg)
    ref = oracle.search(x, cfg.tsamp, cfg.period_min, cfg.period_max, cfg.bins_min,
                        cfg.bins_max, cfg.widths)
    assert np.array_equal(per, ref.periods)
    assert snr_close(snr, ref.snr) < SNR_RTOL
    # the injected pulse (period 200.37 samples, S/N 15) is the top peak
    best = np.unravel_index(np.argmax(snr), snr.shape)
    assert abs(per[best[0]] - pulses[0].period) < 0.01
    assert snr.max() > 11.0


def test_degenerate_series_sets_status(ctx):
    x = np.full(20_000, 3.0, dtype=np.float32)
    cfg = synth.SearchConfig(1.0, 40.0, 400.0, 40, 47, (1, 2))
    _, _, snr = run_search(ctx, x, cfg)
    assert np.isnan(snr).all()
    assert ffa.ffa_sync_status(ctx) == ffa.FFA_ERR_DEGENERATE
    assert ffa.ffa_sync_status(ctx) == ffa.FFA_OK


def test_fresh_context_reports_ok_status():
    # the status word of a new context starts cleared (its memory may hold
    # anything before the first search writes it)
    junk = torch.full((1 << 20,), -1, dtype=torch.int32, device="cuda")
    del junk
    c = ffa.ffa_create(0)
    try:
        x = np.random.default_rng(12).standard_normal(20_000).astype(np.float32)
        prm = ffa.make_params(1.0, 40.0, 400.0, 40, 47, (1, 2))
        ffa.ffa_search(c, dev(x), prm)
        assert ffa.ffa_sync_status(c) == ffa.FFA_OK
    finally:
        ffa.ffa_destroy(c)


def test_invalid_arguments_do_no_device_work(ctx):
    x = dev(np.zeros(1000, np.float32))
    prm = ffa.make_params(1.0, 40.0, 400.0, 40, 47, (1, 2))
    snr = torch.zeros((3, 2), device="cuda")
    with pytest.raises(ffa.FFAError) as e:
        ffa.ffa_search(ctx, x, prm, snr=snr)
    assert e.value.status == ffa.FFA_ERR_BUFFER_TOO_SMALL
    assert "small" in ffa.ffa_last_error(ctx)
    assert (snr == 0).all()


def test_search_window_wider_than_a_downsampling_block_is_refused(ctx):
    # the first factor P_min / (b_min tau) = 16,500 already leaves no room for a
    # downsampling block (floor(ds) <= 16,382): an argument error, no device work
    x = dev(np.zeros(1 << 23, np.float32))
    prm = ffa.make_params(1.0, 240 * 16_500.0, 5.0e6, 240, 259, (1, 2))
    assert ffa.ffa_plan_rows(prm, 1 << 23) > 0
    snr = torch.zeros((ffa.ffa_plan_rows(prm, 1 << 23), 2), device="cuda")
    with pytest.raises(ffa.FFAError) as e:
        ffa.ffa_search(ctx, x, prm, snr=snr)
    assert e.value.status == ffa.FFA_ERR_INVALID_ARG
    assert "downsampling block" in ffa.ffa_last_error(ctx)
    assert (snr == 0).all()


def test_search_duty_width_grid(ctx):
    g = synth.rng(9, 0)
    x = synth.inject(synth.noise(1 << 21, g),
                     synth.Pulse(period=1.234 / 64e-6, duty=0.04, amplitude=18.0, phi0=0.7))
    cfg = synth.config_duty(64e-6, 0.5, 4.0)
    per, bins, snr = run_search(ctx, x, cfg)
    ref = oracle.search(x, cfg.tsamp, cfg.period_min, cfg.period_max, cfg.bins_min,
                        cfg.bins_max, cfg.widths)
    assert np.array_equal(per, ref.periods)
    assert snr_close(snr, ref.snr) < SNR_RTOL
    best = np.unravel_index(np.argmax(snr), snr.shape)
    assert abs(per[best[0]] - 1.234) < 1e-3


def test_search_workload2_full(ctx):
    # red noise de-reddened in the search by the running median of 5 s
    # (Sec. 5.2), then normalised and searched
    x, cfg, pulses = synth.workload2()
    assert cfg.median_window == 78125
    per, bins, snr = run_search(ctx, x, cfg)
    ref = oracle.search(x, cfg.tsamp, cfg.period_min, cfg.period_max, cfg.bins_min,
                        cfg.bins_max, cfg.widths, median_window=cfg.median_window)
    assert np.array_equal(per, ref.periods)
    assert snr_close(snr, ref.snr) < SNR_RTOL
    # the brightest injected pulse stands out of the de-reddened periodogram
    top = max(pulses, key=lambda q: q.amplitude)
    near = np.abs(per / (top.period * cfg.tsamp) - 1.0) < 0.01
    assert snr[near].max() > 7.0


def test_batch_with_and_without_de_reddening(ctx):
    # a batch mixing series with and without the running median (different
    # windows), eager and replayed, and the single-series no-allocation search
    # of one of them, against the oracle
    g = synth.rng(21, 0)
    n = 600_000
    base = [synth.noise(n, g).astype(np.float64) + synth.red_noise(n, 0.3, g) for _ in range(3)]
    xs = [b.astype(np.float32) for b in base]
    windows = [0, 15625, 4001]
    tsamp = 64e-6
    params = [ffa.make_params(tsamp, 0.1, 2.0, 240, 259, synth.WIDTHS_DUTY, median_window=w)
              for w in windows]
    dev_x = [dev(x) for x in xs]
    refs = [oracle.search(x, tsamp, 0.1, 2.0, 240, 259, synth.WIDTHS_DUTY, median_window=w)
            for x, w in zip(xs, windows)]
    snr, offs = ffa.ffa_search_batch(ctx, dev_x, params)
    torch.cuda.synchronize()
    got = snr.cpu().numpy()
    for i, r in enumerate(refs):
        assert snr_close(got[offs[i]:offs[i] + r.snr.shape[0]], r.snr) < SNR_RTOL, i
    out = torch.full(snr.shape, -1.0, device="cuda")
    for rep in range(2):
        out.fill_(-1.0)
        ffa.ffa_search_batch(ctx, dev_x, params, snr=out, row_offset=offs, use_graph=True)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), got), rep
        ffa.ffa_search_batch(ctx, dev_x[:1], params[:1])
        torch.cuda.synchronize()
    one = torch.full((refs[1].snr.shape[0], 9), -1.0, device="cuda")
    ffa.ffa_search_noalloc(ctx, dev_x[1], params[1], one)
    torch.cuda.synchronize()
    assert np.array_equal(one.cpu().numpy(), got[offs[1]:offs[1] + refs[1].snr.shape[0]])
    tm_before = ffa.ffa_read_timing(ctx, reset=False)
    assert "median_ms" in tm_before


@pytest.mark.parametrize("tdt,dt,bmax,bmed", [(torch.bfloat16, ffa.FFA_BF16, 0.1, 0.01),
                                              (torch.float16, ffa.FFA_F16, 0.01, 1e-3)])
def test_low_precision_search_with_de_reddening(ctx, tdt, dt, bmax, bmed):
    # 16-bit storage with the running median: the de-reddened series and the
    # downsampled series are kept in the storage type; against the oracle on
    # the stored (dequantised) samples
    g = synth.rng(22, 0)
    n = 400_000
    x = (synth.noise(n, g).astype(np.float64) + synth.red_noise(n, 0.3, g)).astype(np.float32)
    xq = torch.from_numpy(x).to(tdt)
    xdq = xq.float().numpy()
    prm = ffa.make_params(64e-6, 0.1, 2.0, 240, 259, synth.WIDTHS_DUTY, dtype=dt,
                          median_window=4001)
    _, _, snr = ffa.ffa_search(ctx, xq.cuda(), prm)
    torch.cuda.synchronize()
    assert ffa.ffa_sync_status(ctx) == ffa.FFA_OK
    ref = oracle.search(xdq, 64e-6, 0.1, 2.0, 240, 259, synth.WIDTHS_DUTY, median_window=4001)
    err = np.abs(snr.cpu().numpy() - ref.snr)
    print(f"{tdt} de-reddened: max |dS/N| {err.max():.3e} median {np.median(err):.3e}")
    assert err.max() < bmax and np.median(err) < bmed


def batch_inputs(n):
    xs, prms = [], []
    for i in range(n):
        g = synth.rng(7, i)
        ns = int(g.integers(300_000, 900_000))
        x = synth.noise(ns, g)
        tsamp = [64e-6, 128e-6, 256e-6][i % 3]
        lo, hi = [(0.1, 1.0), (0.2, 3.0), (1.0, 30.0)][i % 3]
        xs.append(x)
        prms.append((tsamp, lo, hi))
    return xs, prms


def test_batch_equals_single_series_bit_for_bit(ctx):
    xs, cfgs = batch_inputs(7)
    dev_x = [dev(x) for x in xs]
    params = [ffa.make_params(t, lo, hi, 240, 259, synth.WIDTHS_DUTY) for t, lo, hi in cfgs]
    snr_b, offs = ffa.ffa_search_batch(ctx, dev_x, params)
    torch.cuda.synchronize()
    snr_b = snr_b.cpu().numpy()
    for i in range(len(xs)):
        _, _, s1 = ffa.ffa_search(ctx, dev_x[i], params[i])
        torch.cuda.synchronize()
        s1 = s1.cpu().numpy()
        assert np.array_equal(snr_b[offs[i]:offs[i] + s1.shape[0]], s1)
    # spot check one series against the oracle
    t, lo, hi = cfgs[2]
    ref = oracle.search(xs[2], t, lo, hi, 240, 259, synth.WIDTHS_DUTY)
    assert snr_close(snr_b[offs[2]:offs[2] + ref.snr.shape[0]], ref.snr) < SNR_RTOL


@pytest.mark.parametrize("tdt,dt", [(torch.float32, ffa.FFA_F32), (torch.bfloat16, ffa.FFA_BF16)])
def test_batch_with_unaligned_series(ctx, tdt, dt):
    # series that start off a 16-byte boundary (views at odd offsets) take
    # the per-sample loads of the statistics and the downsampler; in a batch
    # with aligned series of other plans (other block lengths), each must
    # equal its own single-series search bit for bit, and the oracle
    xs, cfgs = batch_inputs(4)
    views = []
    for i, x in enumerate(xs):
        off = (0, 1, 3, 0)[i]
        buf = torch.zeros(x.size + off, dtype=tdt, device="cuda")
        buf[off:] = torch.from_numpy(x).to(tdt)
        views.append(buf[off:])
    params = [ffa.make_params(t, lo, hi, 240, 259, synth.WIDTHS_DUTY, dtype=dt) for t, lo, hi in cfgs]
    snr_b, offs = ffa.ffa_search_batch(ctx, views, params)
    torch.cuda.synchronize()
    assert ffa.ffa_sync_status(ctx) == ffa.FFA_OK
    snr_b = snr_b.cpu().numpy()
    for i, v in enumerate(views):
        _, _, s1 = ffa.ffa_search(ctx, v, params[i])
        torch.cuda.synchronize()
        assert np.array_equal(snr_b[offs[i]:offs[i] + s1.shape[0]], s1.cpu().numpy()), i
    if dt == ffa.FFA_F32:
        t, lo, hi = cfgs[1]
        ref = oracle.search(xs[1], t, lo, hi, 240, 259, synth.WIDTHS_DUTY)
        assert snr_close(snr_b[offs[1]:offs[1] + ref.snr.shape[0]], ref.snr) < SNR_RTOL


def test_graph_replay_matches_eager(ctx):
    xs, cfgs = batch_inputs(4)
    dev_x = [dev(x) for x in xs]
    params = [ffa.make_params(t, lo, hi, 240, 259, synth.WIDTHS_DUTY) for t, lo, hi in cfgs]
    eager, offs = ffa.ffa_search_batch(ctx, dev_x, params)
    torch.cuda.synchronize()
    eager = eager.cpu().numpy()
    out = torch.full((eager.shape[0], eager.shape[1]), -1.0, device="cuda")
    for rep in range(4):
        out.fill_(-1.0)
        ffa.ffa_search_batch(ctx, dev_x, params, snr=out, row_offset=offs, use_graph=True)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), eager), rep
        # eager work of the program between replays
        ffa.ffa_search_batch(ctx, dev_x[:1], params[:1])
        torch.cuda.synchronize()


@pytest.mark.parametrize("dt,tdt,bound", [(ffa.FFA_BF16, torch.bfloat16, 0.02),
                                         (ffa.FFA_F16, torch.float16, 2e-3)])
def test_low_precision_storage(ctx, dt, tdt, bound):
    g = synth.rng(9, 1)
    x = synth.noise(1 << 21, g)
    xq = torch.from_numpy(x).to(tdt)
    xdq = xq.to(torch.float32).numpy()       # what the kernels actually read
    cfg = synth.config_duty(64e-6, 0.5, 4.0)
    prm = ffa.make_params(cfg.tsamp, cfg.period_min, cfg.period_max, cfg.bins_min,
                          cfg.bins_max, cfg.widths, dtype=dt)
    _, _, snr = ffa.ffa_search(ctx, xq.cuda(), prm)
    torch.cuda.synchronize()
    snr = snr.cpu().numpy()
    ref = oracle.search(x, cfg.tsamp, cfg.period_min, cfg.period_max, cfg.bins_min,
                        cfg.bins_max, cfg.widths)
    ref_dq = oracle.search(xdq, cfg.tsamp, cfg.period_min, cfg.period_max, cfg.bins_min,
                           cfg.bins_max, cfg.widths)
    err = np.abs(snr - ref.snr)
    err_dq = np.abs(snr - ref_dq.snr)
    print(f"dtype {dt}: vs FP32 input max {err.max():.3e} median {np.median(err):.3e}; "
          f"vs dequantised input max {err_dq.max():.3e} median {np.median(err_dq):.3e}")
    assert err.max() < bound * 8 and np.median(err) < bound
    assert err_dq.max() < bound * 8


# Workload 3 at full size (2^23 samples at 64 us) in the batch call with the
# default tiling (the configuration the benchmark times): every periodogram row
# of four series (two with a pulse) against the oracle in FP32; then the same
# series normalised in FP64 and stored as BF16 and as FP16 (workload 4): S/N
# error against the oracle on the FP32 series and detection agreement at
# S/N >= 7, per (row, width) and per injected pulse.
def test_workload3_full_size_batch_and_low_precision(ctx):
    cfg = synth.workload3_config()
    pulsed = synth.workload3_pulsed()
    idx = [int(pulsed[0]), int(pulsed[1]), 1, 3]
    xs, pulses = zip(*[synth.workload3_series(i, pulsed=pulsed) for i in idx])
    refs = [oracle.search(x, cfg.tsamp, cfg.period_min, cfg.period_max, cfg.bins_min,
                          cfg.bins_max, cfg.widths) for x in xs]
    ref_all = np.concatenate([r.snr for r in refs])

    def run(arrs, dt):
        series = [dev(a) if dt == ffa.FFA_F32 else a for a in arrs]
        prm = [ffa.make_params(cfg.tsamp, cfg.period_min, cfg.period_max, cfg.bins_min,
                               cfg.bins_max, cfg.widths, dtype=dt) for _ in arrs]
        snr, _ = ffa.ffa_search_batch(ctx, series, prm)
        torch.cuda.synchronize()
        assert ffa.ffa_sync_status(ctx) == ffa.FFA_OK
        return snr.cpu().numpy().astype(np.float64)

    snr32 = run(xs, ffa.FFA_F32)
    assert snr32.shape == ref_all.shape
    assert snr_close(snr32, ref_all) < SNR_RTOL
    rows = [r.snr.shape[0] for r in refs]
    starts = np.cumsum([0] + rows)
    for tdt, dt, bound_max, bound_med in ((torch.bfloat16, ffa.FFA_BF16, 0.1, 0.01),
                                          (torch.float16, ffa.FFA_F16, 0.01, 1e-3)):
        lowp = []
        for x in xs:
            xd = x.astype(np.float64)
            xn = (xd - xd.mean()) / np.sqrt(((xd - xd.mean()) ** 2).mean())
            lowp.append(torch.from_numpy(xn.astype(np.float32)).to(tdt).cuda())
        snr = run(lowp, dt)
        err = np.abs(snr - ref_all)
        det_g, det_r = snr >= 7.0, ref_all >= 7.0
        agree = float(np.mean(det_g == det_r))
        found = []
        for k, (pu, r) in enumerate(zip(pulses, refs)):
            if pu is None:
                continue
            period_s = pu.period * cfg.tsamp
            near = np.abs(r.periods / period_s - 1.0) < 0.02
            blk = snr[starts[k]:starts[k + 1]]
            found.append((bool(blk[near].max() >= 7.0), bool(r.snr[near].max() >= 7.0)))
        print(f"{tdt}: max |dS/N| {err.max():.3e} median {np.median(err):.3e}; "
              f"detections (S/N >= 7) gpu {int(det_g.sum())} oracle {int(det_r.sum())}, "
              f"agreement per (row, width) {agree:.6f}; pulses found gpu/oracle {found}")
        assert err.max() < bound_max and np.median(err) < bound_med
        assert all(a == b for a, b in found)


def test_workload3_batch_spanning_two_scratch_groups(ctx):
    # 72 full-size workload-3 series need two scratch groups (two launches per
    # group, the benchmark's grouping); series from both groups against the oracle
    cfg = synth.workload3_config()
    pulsed = synth.workload3_pulsed()
    n = 72
    print(f"two scratch groups: {n} series of 2^23", flush=True)
    xs = [synth.workload3_series(i, pulsed=pulsed)[0] for i in range(n)]
    series = [dev(x) for x in xs]
    prm = [ffa.make_params(cfg.tsamp, cfg.period_min, cfg.period_max, cfg.bins_min, cfg.bins_max,
                           cfg.widths) for _ in xs]
    ffa.ffa_set_timing(ctx, True)
    ffa.ffa_read_timing(ctx, reset=True)
    snr, offs = ffa.ffa_search_batch(ctx, series, prm)
    torch.cuda.synchronize()
    tm = ffa.ffa_read_timing(ctx, reset=True)
    ffa.ffa_set_timing(ctx, False)
    assert ffa.ffa_sync_status(ctx) == ffa.FFA_OK
    assert tm["fold_launches"] == 4, tm["fold_launches"]
    host = snr.cpu().numpy().astype(np.float64)
    for i in (0, 40, n - 1):
        ref = oracle.search(xs[i], cfg.tsamp, cfg.period_min, cfg.period_max, cfg.bins_min,
                            cfg.bins_max, cfg.widths)
        got = host[offs[i]:offs[i] + ref.snr.shape[0]]
        assert snr_close(got, ref.snr) < SNR_RTOL, i


def test_smaller_scratch_groups_when_memory_is_short():
    # a fresh context on a device with only 6 GB free: the 20-series batch's
    # scratch (two buffers of 5 GB) does not fit, the call lowers the scratch
    # budget until it does (groups of 4 series) and still returns the right
    # periodogram
    cfg = synth.workload3_config()
    pulsed = synth.workload3_pulsed()
    n = 20
    xs = [synth.workload3_series(i, pulsed=pulsed)[0] for i in range(n)]
    series = [dev(x) for x in xs]
    prm = [ffa.make_params(cfg.tsamp, cfg.period_min, cfg.period_max, cfg.bins_min, cfg.bins_max,
                           cfg.widths) for _ in xs]
    rows = [ffa.ffa_plan_rows(q, x.size) for q, x in zip(prm, xs)]
    snr = torch.empty((sum(rows), len(cfg.widths)), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    free, _ = torch.cuda.mem_get_info()
    fill = free - (6 << 30)
    print(f"short memory: {free / 2**30:.1f} GiB free, holding {fill / 2**30:.1f} GiB", flush=True)
    filler = torch.empty(max(fill, 0), dtype=torch.uint8, device="cuda")
    c = ffa.ffa_create(0)
    try:
        ffa.ffa_set_timing(c, True)
        got, offs = ffa.ffa_search_batch(c, series, prm, snr=snr)
        torch.cuda.synchronize()
        tm = ffa.ffa_read_timing(c, reset=True)
        assert ffa.ffa_sync_status(c) == ffa.FFA_OK
    finally:
        ffa.ffa_destroy(c)
        del filler
        torch.cuda.empty_cache()
    assert tm["fold_launches"] == 10, tm["fold_launches"]  # 5 groups of 4 series, 2 passes
    host = got.cpu().numpy().astype(np.float64)
    for i in (0, n - 1):
        ref = oracle.search(xs[i], cfg.tsamp, cfg.period_min, cfg.period_max, cfg.bins_min,
                            cfg.bins_max, cfg.widths)
        assert snr_close(host[offs[i]:offs[i] + ref.snr.shape[0]], ref.snr) < SNR_RTOL, i


def test_persistent_launch_equals_pass_launches(ctx):
    # same tiles either way: the periodograms are bit-identical (the
    # persistent launch runs the general kernel, the per-pass launches the
    # kernels compiled for full-tile and range-tile passes)
    xs, cfgs = batch_inputs(5)
    dev_x = [dev(x) for x in xs]
    params = [ffa.make_params(t, lo, hi, 240, 259, synth.WIDTHS_DUTY) for t, lo, hi in cfgs]
    ffa.ffa_set_tiling(ctx, 0, 4, persistent=True)
    try:
        a, offs = ffa.ffa_search_batch(ctx, dev_x, params)
        torch.cuda.synchronize()
    finally:
        ffa.ffa_set_tiling(ctx)
    b, _ = ffa.ffa_search_batch(ctx, dev_x, params)
    torch.cuda.synchronize()
    assert ffa.ffa_sync_status(ctx) == ffa.FFA_OK
    assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())


@pytest.mark.parametrize("lds_rows,levels,persistent,waves", [
    (32, 2, True, 16), (64, 3, False, 16), (48, 1, True, 16), (0, 2, True, 16),
    (0, 4, False, 8), (0, 3, True, 8), (40, 2, False, 8), (0, 5, False, 8), (24, 5, True, 8)])
def test_search_tilings_agree(ctx, lds_rows, levels, persistent, waves):
    # the FFA addition tree does not depend on the tiling; the boxcar prefix
    # sums start at the segment a wave takes, so S/N agrees to FP32 rounding
    x = synth.noise(1 << 21, synth.rng(9, 2))
    cfg = synth.config_duty(64e-6, 0.5, 4.0)
    ref = run_search(ctx, x, cfg)[2]
    ffa.ffa_set_tiling(ctx, lds_rows, levels, persistent=persistent, waves_per_group=waves)
    try:
        got = run_search(ctx, x, cfg)[2]
    finally:
        ffa.ffa_set_tiling(ctx)
    assert ffa.ffa_sync_status(ctx) == ffa.FFA_OK
    assert snr_close(got, ref.astype(np.float64)) < 2e-6


def test_workload5_full_uneven_batch(ctx):
    # the uneven batch at its full size, as the benchmark runs it: 256 series
    # of 2^20..2^24 samples, three sampling times and two period ranges in one
    # batched call with the default tiling (transforms of up to ~21,000 rows,
    # three passes); the shortest and longest series and one of every
    # (sampling time, period range) pair against the oracle
    xs, cfgs, keys = [], [], []
    for i in range(256):
        x, cfg, _ = synth.workload5_series(i)
        xs.append(x)
        cfgs.append(cfg)
        keys.append((cfg.tsamp, cfg.period_min))
        if (i + 1) % 64 == 0:
            print(f"uneven batch: generated {i + 1}/256 series", flush=True)
    dev_x = [dev(x) for x in xs]
    params = [ffa.make_params(c.tsamp, c.period_min, c.period_max, c.bins_min, c.bins_max,
                              c.widths) for c in cfgs]
    ffa.ffa_set_tiling(ctx)
    snr, offs = ffa.ffa_search_batch(ctx, dev_x, params)
    torch.cuda.synchronize()
    assert ffa.ffa_sync_status(ctx) == ffa.FFA_OK
    host = snr.cpu().numpy()
    del dev_x, snr
    sizes = [x.size for x in xs]
    pick = {int(np.argmin(sizes)), int(np.argmax(sizes))}
    for k in sorted(set(keys)):
        pick.add(keys.index(k))
    assert len(pick) >= 6
    for i in sorted(pick):
        c = cfgs[i]
        print(f"uneven batch: series {i}, {xs[i].size} samples, tsamp {c.tsamp}, "
              f"periods {c.period_min}-{c.period_max} s", flush=True)
        ref = oracle.search(xs[i], c.tsamp, c.period_min, c.period_max, c.bins_min, c.bins_max,
                            c.widths)
        got = host[offs[i]:offs[i] + ref.snr.shape[0]]
        assert snr_close(got, ref.snr) < SNR_RTOL, i


def test_autotune_uneven_batch_and_cache(ctx, tmp_path):
    # uneven lengths, sampling times and period ranges (the uneven-batch
    # workload, scaled down); the tuned tiling gives the same periodogram to
    # FP32 rounding and is read back from the cache file
    xs, cfgs = [], []
    for i in range(6):
        x, cfg, _ = synth.workload5_series(i)
        xs.append(x[: min(x.size, 1 << 21)])
        cfgs.append(cfg)
    dev_x = [dev(x) for x in xs]
    params = [ffa.make_params(c.tsamp, c.period_min, c.period_max, c.bins_min, c.bins_max,
                              c.widths) for c in cfgs]
    ref, offs = ffa.ffa_search_batch(ctx, dev_x, params)
    torch.cuda.synchronize()
    cache = str(tmp_path / "tiles.txt")
    try:
        best = ffa.ffa_autotune(ctx, dev_x, params, cache_path=cache)
        assert best.waves_per_group in (8, 16) and 1 <= best.levels_per_pass <= 5
        assert best.lds_rows in (0, 40)
        got, _ = ffa.ffa_search_batch(ctx, dev_x, params)
        torch.cuda.synchronize()
        assert snr_close(got.cpu().numpy(), ref.cpu().numpy().astype(np.float64)) < 2e-6
        again = ffa.ffa_autotune(ctx, dev_x, params, cache_path=cache)
        assert (again.waves_per_group, again.levels_per_pass, again.persistent,
                again.lds_rows) == (best.waves_per_group, best.levels_per_pass,
                                    best.persistent, best.lds_rows)
        assert len(open(cache).read().strip().splitlines()) == 1
    finally:
        ffa.ffa_set_tiling(ctx)
    i = 3
    ref_o = oracle.search(xs[i], cfgs[i].tsamp, cfgs[i].period_min, cfgs[i].period_max,
                          cfgs[i].bins_min, cfgs[i].bins_max, cfgs[i].widths)
    assert snr_close(got.cpu().numpy()[offs[i]:offs[i] + ref_o.snr.shape[0]], ref_o.snr) < SNR_RTOL


# ---------------------------------------------------------------------------
# The forms that run in the benchmark, against the oracle
# ---------------------------------------------------------------------------

def test_pair_kernels_integer_search_bit_exact(ctx):
    # The kernels compiled for the pair-merge forms and the register-window S/N
    # (every p >= 160, the duty-cycle width grid): ds = 1 (P_min = 240 tau,
    # one pseudo-octave: P_max = 259.5 tau stops the search before the second,
    # whose factor 260/240 is not an integer), no normalisation, integer samples with
    # |x| <= 8, so every merge and prefix sum is an exact FP32 integer
    # (m (p + 48) 8 < 2^24). Transforms of 772..833 rows take a full-tile pass
    # and a range pass. The S/N is then the exact best boxcar sum times the
    # FP32 scale 1/sqrt(m w), rounded once.
    n = 200_000
    x = np.random.default_rng(31).integers(-8, 9, size=n).astype(np.float32)
    widths = synth.WIDTHS_DUTY
    prm = ffa.make_params(1.0, 240.0, 259.5, 240, 259, widths, normalise=False)
    per, bins, snr = ffa.ffa_search(ctx, dev(x), prm)
    torch.cuda.synchronize()
    got = snr.cpu().numpy()
    ref = oracle.search(x, 1.0, 240.0, 259.5, 240, 259, widths, normalise=False)
    assert np.array_equal(per, ref.periods) and np.array_equal(bins, ref.bins)
    assert (ref.octave == 0).all() and ref.rows_m.min() > 64 and ref.rows_m.max() * (259 + 48) * 8 < 2 ** 24
    w = np.asarray(widths, dtype=np.float64)[None, :]
    mw = ref.rows_m.astype(np.float64)[:, None] * w
    best = np.rint(ref.snr * np.sqrt(mw))
    assert np.allclose(best, ref.snr * np.sqrt(mw), rtol=0, atol=1e-6)
    scale = (1.0 / np.sqrt(mw)).astype(np.float32)
    want = best.astype(np.float32) * scale
    assert want.dtype == np.float32
    assert np.array_equal(got, want)


def _workload3_pair():
    cfg = synth.workload3_config()
    pulsed = synth.workload3_pulsed()
    idx = [int(pulsed[0]), 2]
    xs = [synth.workload3_series(i, pulsed=pulsed)[0] for i in idx]
    refs = [oracle.search(x, cfg.tsamp, cfg.period_min, cfg.period_max, cfg.bins_min,
                          cfg.bins_max, cfg.widths) for x in xs]
    prm = [ffa.make_params(cfg.tsamp, cfg.period_min, cfg.period_max, cfg.bins_min,
                           cfg.bins_max, cfg.widths) for _ in xs]
    return xs, prm, np.concatenate([r.snr for r in refs])


def test_persistent_and_graph_forms_match_oracle(ctx):
    # two full-size workload-3 series, every row against the oracle: one
    # persistent launch per group, eager and replayed from a hipGraph, and the
    # per-pass launches replayed from a hipGraph
    xs, prm, ref = _workload3_pair()
    series = [dev(x) for x in xs]
    for persistent in (True, False):
        ffa.ffa_set_tiling(ctx, 0, 5, persistent=persistent)
        try:
            if persistent:
                print("persistent launch, eager", flush=True)
                got, offs = ffa.ffa_search_batch(ctx, series, prm)
                torch.cuda.synchronize()
                assert ffa.ffa_sync_status(ctx) == ffa.FFA_OK
                assert snr_close(got.cpu().numpy(), ref) < SNR_RTOL
            print(f"graph replays, persistent={persistent}", flush=True)
            offs = [0, int(ffa.ffa_plan_rows(prm[0], xs[0].size))]
            out = torch.full((ref.shape[0], ref.shape[1]), -1.0, device="cuda")
            for rep in range(3):
                out.fill_(-1.0)
                ffa.ffa_search_batch(ctx, series, prm, snr=out, row_offset=offs, use_graph=True)
                torch.cuda.synchronize()
                assert ffa.ffa_sync_status(ctx) == ffa.FFA_OK
                assert snr_close(out.cpu().numpy(), ref) < SNR_RTOL, rep
                # eager work of the program between replays
                ffa.ffa_search_batch(ctx, series[:1], prm[:1])
                torch.cuda.synchronize()
        finally:
            ffa.ffa_set_tiling(ctx)


def test_graph_replay_after_context_buffers_move(ctx):
    # a replayed graph must not keep the addresses of context buffers that a
    # later call has reallocated (a raw transform growing the scratch, an
    # autotune dropping the cached tables)
    xs, cfgs = batch_inputs(3)
    dev_x = [dev(x) for x in xs]
    params = [ffa.make_params(t, lo, hi, 240, 259, synth.WIDTHS_DUTY) for t, lo, hi in cfgs]
    eager, offs = ffa.ffa_search_batch(ctx, dev_x, params)
    torch.cuda.synchronize()
    eager = eager.cpu().numpy()
    out = torch.full(eager.shape, -1.0, device="cuda")
    ffa.ffa_search_batch(ctx, dev_x, params, snr=out, row_offset=offs, use_graph=True)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), eager)
    # a raw transform far larger than the batch's scratch: the scratch moves
    X = np.random.default_rng(5).integers(-8, 9, size=(20000, 259)).astype(np.float32)
    big = ffa.ffa_transform(ctx, dev(X))
    torch.cuda.synchronize()
    del big
    out.fill_(-1.0)
    ffa.ffa_search_batch(ctx, dev_x, params, snr=out, row_offset=offs, use_graph=True)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), eager)
    # the job tables are dropped and rebuilt by an autotune
    try:
        ffa.ffa_autotune(ctx, dev_x[:1], params[:1])
    finally:
        ffa.ffa_set_tiling(ctx)
    out.fill_(-1.0)
    ffa.ffa_search_batch(ctx, dev_x, params, snr=out, row_offset=offs, use_graph=True)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), eager)
