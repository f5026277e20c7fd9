"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point of include/ffa.h, validates arguments, and its period plan
equals the oracle's, row for row."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_2004_03701_amd as ffa
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "ffa.h")).read()
    return sorted(set(re.findall(r"^\s*(?:ffa_status|const char\*)\s+(ffa_\w+)\s*\(", text,
                                 flags=re.M)))


def test_library_exports_every_declared_entry_point():
    L = ffa.lib()
    names = header_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(ffa.EXPORTED)


def test_status_strings():
    for st in range(-7, 1):
        assert ffa.status_string(st)
    assert ffa.status_string(-99) == "unknown status"


CONFIGS = [
    (1.0, 128.0, 256.0, 128, 255, synth.WIDTHS_PAPER, 262144),
    (64e-6, 0.5, 10.0, 240, 259, synth.WIDTHS_DUTY, 9_375_000),
    (64e-6, 0.5, 10.0, 240, 259, synth.WIDTHS_DUTY, 1 << 23),
    (1.0, 40.0, 160.0, 40, 47, (1, 2, 3, 5), 6000),
    (0.37, 3.1, 50.0, 7, 9, (1, 2), 20000),
]


@pytest.mark.parametrize("cfg", CONFIGS)
def test_plan_equals_oracle_plan(cfg):
    ts, pmin, pmax, bmin, bmax, w, n = cfg
    octs = oracle.plan(ts, pmin, pmax, bmin, bmax, n)
    prm = ffa.make_params(ts, pmin, pmax, bmin, bmax, w)
    ex = ffa.ffa_plan_export(prm, n)
    per = np.concatenate([t.periods for o in octs for t in o.transforms if t.keep])
    bins = np.concatenate([np.full(t.keep, t.p) for o in octs for t in o.transforms if t.keep])
    ms = np.concatenate([np.full(t.keep, t.m) for o in octs for t in o.transforms if t.keep])
    ok = np.concatenate([np.full(t.keep, k) for k, o in enumerate(octs) for t in o.transforms
                         if t.keep])
    dsfx = np.concatenate([np.full(t.keep, o.ds_fx, dtype=np.uint64) for o in octs
                           for t in o.transforms if t.keep])
    assert ffa.ffa_plan_rows(prm, n) == per.size
    assert np.array_equal(ex["period"], per)   # bit-identical FP64 labels
    assert np.array_equal(ex["bins"], bins)
    assert np.array_equal(ex["m"], ms)
    assert np.array_equal(ex["octave"], ok)
    assert np.array_equal(ex["ds_fx"], dsfx)


def test_plan_equals_oracle_on_uneven_workload_draws():
    for i in range(12):
        g = synth.rng(5, i)
        u = g.uniform(20.0, 24.0)
        n = int(2 ** u)
        tsamp = float(g.choice([64e-6, 128e-6, 256e-6]))
        lo, hi = (0.1, 1.0) if g.uniform() < 0.5 else (1.0, 30.0)
        octs = oracle.plan(tsamp, lo, hi, 240, 259, n)
        prm = ffa.make_params(tsamp, lo, hi, 240, 259, synth.WIDTHS_DUTY)
        per = np.concatenate([t.periods for o in octs for t in o.transforms if t.keep])
        assert np.array_equal(ffa.ffa_plan_export(prm, n)["period"], per)


def status_of(fn):
    try:
        fn()
    except ffa.FFAError as e:
        return e.status
    return ffa.FFA_OK


def test_parameter_validation():
    good = dict(tsamp=1.0, period_min=128.0, period_max=256.0, bins_min=128, bins_max=255,
                widths=(1, 2, 3))
    def rows(**kw):
        d = dict(good)
        d.update(kw)
        return lambda: ffa.ffa_plan_rows(ffa.make_params(**d), 262144)
    assert status_of(rows()) == ffa.FFA_OK
    assert status_of(rows(tsamp=0.0)) == ffa.FFA_ERR_INVALID_ARG
    assert status_of(rows(tsamp=float("nan"))) == ffa.FFA_ERR_INVALID_ARG
    assert status_of(rows(period_max=100.0)) == ffa.FFA_ERR_INVALID_ARG
    assert status_of(rows(bins_min=1)) == ffa.FFA_ERR_INVALID_ARG
    assert status_of(rows(bins_max=100)) == ffa.FFA_ERR_INVALID_ARG
    assert status_of(rows(bins_max=5000)) == ffa.FFA_ERR_INVALID_ARG
    assert status_of(rows(widths=())) == ffa.FFA_ERR_INVALID_ARG
    assert status_of(rows(widths=(2, 2))) == ffa.FFA_ERR_INVALID_ARG
    assert status_of(rows(widths=(0, 1))) == ffa.FFA_ERR_INVALID_ARG
    assert status_of(rows(widths=(1, 128))) == ffa.FFA_ERR_INVALID_ARG  # w >= bins_min
    assert status_of(rows(widths=tuple(range(1, 34)))) == ffa.FFA_ERR_INVALID_ARG
    assert status_of(rows(period_min=100.0)) == ffa.FFA_ERR_RANGE       # ds0 < 1
    # too short for any transform with two rows
    assert status_of(lambda: ffa.ffa_plan_rows(ffa.make_params(**good), 250)) == ffa.FFA_ERR_RANGE
    assert status_of(lambda: ffa.ffa_plan_rows(ffa.make_params(**good), 0)) == ffa.FFA_ERR_INVALID_ARG
    p = ffa.make_params(**good)
    p.normalise = 2
    assert status_of(lambda: ffa.ffa_plan_rows(p, 262144)) == ffa.FFA_ERR_INVALID_ARG
    p = ffa.make_params(**good)
    p.dtype = 7
    assert status_of(lambda: ffa.ffa_plan_rows(p, 262144)) == ffa.FFA_ERR_INVALID_ARG
    # the running-median window (Sec. 5.2) is 0 (none) or odd
    assert status_of(rows(median_window=1001)) == ffa.FFA_OK
    assert status_of(rows(median_window=1000)) == ffa.FFA_ERR_INVALID_ARG
    assert status_of(rows(median_window=-1)) == ffa.FFA_ERR_INVALID_ARG


def test_plan_export_capacity():
    prm = ffa.make_params(1.0, 128.0, 256.0, 128, 255, synth.WIDTHS_PAPER)
    n = ffa.ffa_plan_rows(prm, 262144)
    buf = np.empty(n - 1)
    st = ffa.lib().ffa_plan_export(ctypes.byref(prm), 262144, buf.ctypes.data, None, None, None,
                                   None, None, n - 1)
    assert st == ffa.FFA_ERR_BUFFER_TOO_SMALL
    assert ffa.lib().ffa_plan_rows(None, 10, None) == ffa.FFA_ERR_INVALID_ARG


def test_null_context_is_rejected_without_device_work():
    L = ffa.lib()
    prm = ffa.make_params(1.0, 128.0, 256.0, 128, 255, (1, 2))
    assert L.ffa_search(None, None, 10, ctypes.byref(prm), None, None, None, 0, None) == \
        ffa.FFA_ERR_INVALID_ARG
    assert L.ffa_transform(None, None, 4, 4, None, None) == ffa.FFA_ERR_INVALID_ARG
    pk = ffa.make_peak_params()
    n = ctypes.c_int64(0)
    assert L.ffa_find_peaks_batch(None, 1, ctypes.byref(ctypes.c_int64(10)), ctypes.byref(prm),
                                  ctypes.byref(ctypes.c_int64(0)), None, 0, ctypes.byref(pk),
                                  None, 0, ctypes.byref(n), None, None) == ffa.FFA_ERR_INVALID_ARG
    assert L.ffa_search_ranges(None, None, 10, ctypes.byref(prm), 1, None, None, None, None, 0,
                               None) == ffa.FFA_ERR_INVALID_ARG
    assert L.ffa_destroy(None) == ffa.FFA_OK
    assert L.ffa_create(0, None) == ffa.FFA_ERR_INVALID_ARG
