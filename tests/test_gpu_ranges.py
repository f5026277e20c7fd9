"""GPU parity of the dynamic duty-cycle search (Sec. 5.6): one series over
consecutive period sub-ranges with their own phase-bin ranges, against the
oracle's concatenated searches. Bars as for the plain search: periods and bins
identical, S/N within 1e-4 * max(1, |oracle|) in FP32."""
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


def run_and_compare(ctx, x, tsamp, ranges, widths, normalise):
    prms = [ffa.make_params(tsamp, pmin, pmax, bmin, bmax, widths, normalise=normalise)
            for pmin, pmax, bmin, bmax in ranges]
    per, bins, snr, row0 = ffa.ffa_search_ranges(ctx, torch.from_numpy(x.astype(np.float32)).cuda(),
                                                 prms)
    torch.cuda.synchronize()
    ref = oracle.search_ranges(x.astype(np.float32).astype(np.float64), tsamp, ranges, widths,
                               normalise=normalise)
    assert np.array_equal(per, ref.periods) and np.array_equal(bins, ref.bins)
    assert row0[-1] == ref.periods.size and row0[0] == 0
    for k, r in enumerate(ranges):
        # the 32.32 quantisation of the downsampling factor may put the first
        # period a few 1e-10 below period_min
        part = per[row0[k]:row0[k + 1]]
        assert np.all(part >= r[0] * (1 - 1e-9)) and np.all(part < r[1])
    got = snr.cpu().numpy().astype(np.float64)
    err = np.abs(got - ref.snr) / np.maximum(1.0, np.abs(ref.snr))
    print(f"ranges {ranges}: rows {per.size}, max rel err {err.max():.2e}", flush=True)
    assert err.max() < SNR_RTOL
    return per, got


def test_sub_ranges_sample_units(ctx):
    n = 1 << 18
    g = np.random.Generator(np.random.Philox(5600))
    t = np.arange(n, dtype=np.float64)
    ph = np.mod(t / 700.37, 1.0) * 700.37
    x = g.standard_normal(n) + 3.0 * ((ph >= 100.0) & (ph < 102.0))
    ranges = [(128.0, 256.0, 128, 255), (256.0, 1024.0, 256, 511)]
    per, snr = run_and_compare(ctx, x, 1.0, ranges, (1, 2, 3, 4), False)
    # three sub-ranges with a gap between the second and the third
    run_and_compare(ctx, x, 1.0, [(128.0, 200.0, 128, 150), (200.0, 400.0, 200, 260),
                                  (500.0, 1000.0, 300, 331)], (1, 2, 3, 4), True)


def test_sub_ranges_workload_series(ctx):
    # a pulsed workload-3 series of 2^22 samples: 0.5-2 s at 240..259 bins,
    # 2-10 s at twice the duty-cycle resolution
    cfg = synth.workload3_config()
    pulsed = synth.workload3_pulsed()
    x, _ = synth.workload3_series(int(pulsed[0]), nsamp=1 << 22, pulsed=pulsed)
    run_and_compare(ctx, x, cfg.tsamp, [(0.5, 2.0, 240, 259), (2.0, 10.0, 480, 519)],
                    cfg.widths, True)


def test_sub_range_errors(ctx):
    x = torch.zeros(1 << 16, device="cuda")
    mk = lambda pmin, pmax, bmin, bmax, tsamp=1.0: ffa.make_params(tsamp, pmin, pmax, bmin, bmax,
                                                                 (1, 2), normalise=False)
    for bad in ([mk(128.0, 300.0, 128, 255), mk(256.0, 1024.0, 256, 511)],      # overlap
                [mk(128.0, 256.0, 128, 255), mk(256.0, 1024.0, 128, 255, 2.0)]):  # tsamp
        with pytest.raises(ffa.FFAError) as e:
            ffa.ffa_search_ranges(ctx, x, bad)
        assert e.value.status == ffa.FFA_ERR_INVALID_ARG
    good = [mk(128.0, 256.0, 128, 255), mk(256.0, 1024.0, 256, 511)]
    small = torch.empty((10, 2), device="cuda")
    with pytest.raises(ffa.FFAError) as e:
        ffa.ffa_search_ranges(ctx, x, good, snr=small)
    assert e.value.status == ffa.FFA_ERR_BUFFER_TOO_SMALL


def test_sub_ranges_with_about_a_thousand_bins(ctx):
    # long periods at about 1000 bins on a full-length series: transforms of
    # a few hundred rows of ~1000 bins, whose tiles hold only 14 rows, so the
    # range passes are capped at 3 levels (a 5-level tile would need 32 rows)
    cfg = synth.workload3_config()
    pulsed = synth.workload3_pulsed()
    x, _ = synth.workload3_series(int(pulsed[1]), pulsed=pulsed)
    per, _ = run_and_compare(ctx, x, cfg.tsamp, [(0.5, 2.0, 240, 259), (2.0, 10.0, 960, 1039)],
                             cfg.widths, True)
    assert per.size > 0
