"""Python binding of the MI355X FFA periodicity-search library.

Argument marshalling only: every step of the search runs in the HIP kernels
of ``libffa_mi355x.so`` behind the C ABI declared in ``include/ffa.h``; the
functions below carry the same names as the C entry points. PyTorch is used
only for device memory and streams.

The library must have been built (``python -m paper_2004_03701_amd.build``);
importing the raw entry points without it raises immediately, there is no
fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libffa_mi355x.so")

FFA_OK = 0
FFA_ERR_INVALID_ARG = -1
FFA_ERR_RANGE = -2
FFA_ERR_BUFFER_TOO_SMALL = -3
FFA_ERR_NOMEM = -4
FFA_ERR_DEVICE = -5
FFA_ERR_DEGENERATE = -6
FFA_ERR_NOT_IMPLEMENTED = -7

FFA_F32, FFA_BF16, FFA_F16 = 0, 1, 2

EXPORTED = (
    "ffa_create", "ffa_destroy", "ffa_status_string", "ffa_last_error", "ffa_plan_rows",
    "ffa_plan_export", "ffa_search", "ffa_search_batch", "ffa_transform", "ffa_series_stats",
    "ffa_downsample", "ffa_sync_status", "ffa_get_tiling", "ffa_set_tiling", "ffa_autotune",
    "ffa_set_timing", "ffa_read_timing", "ffa_find_peaks_batch", "ffa_search_ranges",
    "ffa_search_noalloc", "ffa_running_median", "ffa_select_dm_trials", "ffa_cluster_frequencies",
    "ffa_flag_harmonics",
)

FFA_NOALLOC_WORKSPACE_BYTES = 128 << 20


class ffa_search_params(ctypes.Structure):
    _fields_ = [
        ("tsamp", ctypes.c_double),
        ("period_min", ctypes.c_double),
        ("period_max", ctypes.c_double),
        ("bins_min", ctypes.c_int32),
        ("bins_max", ctypes.c_int32),
        ("widths", ctypes.POINTER(ctypes.c_int32)),
        ("num_widths", ctypes.c_int32),
        ("normalise", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("median_window", ctypes.c_int32),
    ]


class ffa_tiling(ctypes.Structure):
    _fields_ = [("lds_rows", ctypes.c_int32), ("levels_per_pass", ctypes.c_int32),
                ("persistent", ctypes.c_int32), ("waves_per_group", ctypes.c_int32),
                ("range_waves_per_group", ctypes.c_int32)]


class ffa_kernel_times(ctypes.Structure):
    _fields_ = [
        ("stats_ms", ctypes.c_double),
        ("downsample_ms", ctypes.c_double),
        ("fold_ms", ctypes.c_double),
        ("stats_launches", ctypes.c_int64),
        ("downsample_launches", ctypes.c_int64),
        ("fold_launches", ctypes.c_int64),
        ("profiles", ctypes.c_int64),
        ("folded_cells", ctypes.c_int64),
        ("input_samples", ctypes.c_int64),
        ("downsampled_samples", ctypes.c_int64),
        ("peaks_ms", ctypes.c_double),
        ("peaks_launches", ctypes.c_int64),
        ("median_ms", ctypes.c_double),
        ("median_launches", ctypes.c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ffa_peak_params(ctypes.Structure):
    _fields_ = [("dz_seg", ctypes.c_double), ("k_sigma", ctypes.c_double),
                ("degree", ctypes.c_int32), ("min_points", ctypes.c_int32),
                ("cluster_gap", ctypes.c_double)]


class ffa_peak(ctypes.Structure):
    _fields_ = [("row", ctypes.c_int64), ("period", ctypes.c_double),
                ("threshold", ctypes.c_double), ("snr", ctypes.c_float),
                ("series", ctypes.c_int32), ("width_index", ctypes.c_int32),
                ("members", ctypes.c_int32)]


PEAK_DTYPE = np.dtype([("row", np.int64), ("period", np.float64), ("threshold", np.float64),
                       ("snr", np.float32), ("series", np.int32), ("width_index", np.int32),
                       ("members", np.int32)], align=True)
assert PEAK_DTYPE.itemsize == ctypes.sizeof(ffa_peak)


class FFAError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{message} (status {status})")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2004_03701_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    P = ctypes.POINTER
    pp = P(ffa_search_params)
    sig = {
        "ffa_create": ([ctypes.c_int, P(vp)], i32),
        "ffa_destroy": ([vp], i32),
        "ffa_status_string": ([i32], ctypes.c_char_p),
        "ffa_last_error": ([vp], ctypes.c_char_p),
        "ffa_plan_rows": ([pp, i64, P(i64)], i32),
        "ffa_plan_export": ([pp, i64, vp, vp, vp, vp, vp, vp, i64], i32),
        "ffa_search": ([vp, vp, i64, pp, vp, vp, vp, i64, vp], i32),
        "ffa_search_noalloc": ([vp, vp, i64, pp, vp, vp, vp, i64, vp], i32),
        "ffa_running_median": ([vp, vp, i64, i32, i32, vp, i32, vp], i32),
        "ffa_search_batch": ([vp, i32, P(vp), P(i64), pp, P(i64), vp, i64, i32, vp], i32),
        "ffa_transform": ([vp, vp, i32, i32, vp, vp], i32),
        "ffa_series_stats": ([vp, vp, i64, i32, vp, vp], i32),
        "ffa_downsample": ([vp, vp, i64, i32, vp, u64, i64, vp, vp], i32),
        "ffa_sync_status": ([vp, vp], i32),
        "ffa_get_tiling": ([vp, P(ffa_tiling)], i32),
        "ffa_set_tiling": ([vp, P(ffa_tiling)], i32),
        "ffa_autotune": ([vp, i32, P(vp), P(i64), pp, ctypes.c_char_p, P(ffa_tiling), vp], i32),
        "ffa_set_timing": ([vp, i32], i32),
        "ffa_read_timing": ([vp, P(ffa_kernel_times), i32], i32),
        "ffa_search_ranges": ([vp, vp, i64, pp, i32, vp, vp, vp, vp, i64, vp], i32),
        "ffa_find_peaks_batch": ([vp, i32, P(i64), pp, P(i64), vp, i64, P(ffa_peak_params), vp,
                                  i64, P(i64), vp, vp], i32),
        "ffa_select_dm_trials": ([vp, i32, ctypes.c_double, ctypes.c_double, ctypes.c_double, vp,
                                  P(i32)], i32),
        "ffa_cluster_frequencies": ([vp, vp, i32, ctypes.c_double, vp, vp, vp, P(i32)], i32),
        "ffa_flag_harmonics": ([vp, vp, i32, ctypes.c_double, i32, vp, vp, vp], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def status_string(st: int) -> str:
    return lib().ffa_status_string(st).decode()


def _check(st: int, ctx=None):
    if st != FFA_OK:
        msg = ""
        if ctx is not None:
            msg = lib().ffa_last_error(ctx).decode()
        raise FFAError(st, msg or status_string(st))


def make_params(tsamp: float, period_min: float, period_max: float, bins_min: int,
                bins_max: int, widths: Sequence[int], normalise: bool = True,
                dtype: int = FFA_F32, median_window: int = 0) -> ffa_search_params:
    """Parameter struct; keeps its widths array alive as an attribute."""
    w = (ctypes.c_int32 * len(widths))(*[int(v) for v in widths])
    prm = ffa_search_params(float(tsamp), float(period_min), float(period_max), int(bins_min),
                            int(bins_max), ctypes.cast(w, ctypes.POINTER(ctypes.c_int32)),
                            len(widths), 1 if normalise else 0, int(dtype), int(median_window))
    prm._widths_keepalive = w
    return prm


def _ptr(t) -> int:
    return t.data_ptr() if t is not None else None


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return stream


# ---------------------------------------------------------------------------
# Entry points, same names as the C ABI
# ---------------------------------------------------------------------------

def ffa_create(device: int = 0):
    h = ctypes.c_void_p()
    _check(lib().ffa_create(device, ctypes.byref(h)))
    return h


def ffa_destroy(ctx) -> None:
    _check(lib().ffa_destroy(ctx))


def ffa_last_error(ctx) -> str:
    return lib().ffa_last_error(ctx).decode()


def ffa_plan_rows(params: ffa_search_params, nsamp: int) -> int:
    rows = ctypes.c_int64()
    _check(lib().ffa_plan_rows(ctypes.byref(params), nsamp, ctypes.byref(rows)))
    return rows.value


def ffa_plan_export(params: ffa_search_params, nsamp: int) -> dict:
    n = ffa_plan_rows(params, nsamp)
    out = dict(period=np.empty(n, np.float64), bins=np.empty(n, np.int32),
               m=np.empty(n, np.int32), s=np.empty(n, np.int32),
               octave=np.empty(n, np.int32), ds_fx=np.empty(n, np.uint64))
    a = [out[k].ctypes.data for k in ("period", "bins", "m", "s", "octave", "ds_fx")]
    _check(lib().ffa_plan_export(ctypes.byref(params), nsamp, *a, n))
    return out


def ffa_search(ctx, series, params: ffa_search_params, snr=None, stream=None,
               want_labels: bool = True):
    """Periodogram of one device series (torch tensor). Returns
    (periods, bins, snr) with periods/bins as numpy arrays (None unless
    want_labels) and snr a device tensor rows x num_widths."""
    import torch
    nsamp = series.numel()
    rows = ffa_plan_rows(params, nsamp)
    if snr is None:
        snr = torch.empty((rows, params.num_widths), dtype=torch.float32, device=series.device)
    per = np.empty(rows, np.float64) if want_labels else None
    bins = np.empty(rows, np.int32) if want_labels else None
    st = lib().ffa_search(ctx, series.data_ptr(), nsamp, ctypes.byref(params),
                          per.ctypes.data if want_labels else None,
                          bins.ctypes.data if want_labels else None,
                          snr.data_ptr(), snr.shape[0], _stream(stream))
    _check(st, ctx)
    return per, bins, snr


def ffa_search_noalloc(ctx, series, params: ffa_search_params, snr, stream=None,
                       want_labels: bool = True):
    """ffa_search in the library's static device workspace: no device memory
    is allocated by the call. `snr` (a device tensor rows x num_widths, float32)
    is required. Returns (periods, bins, snr)."""
    nsamp = series.numel()
    per = bins = None
    if want_labels:
        rows = ffa_plan_rows(params, nsamp)
        per = np.empty(rows, np.float64)
        bins = np.empty(rows, np.int32)
    st = lib().ffa_search_noalloc(ctx, series.data_ptr(), nsamp, ctypes.byref(params),
                                  per.ctypes.data if want_labels else None,
                                  bins.ctypes.data if want_labels else None,
                                  snr.data_ptr(), snr.shape[0], _stream(stream))
    _check(st, ctx)
    return per, bins, snr


def ffa_running_median(ctx, series, window: int, out=None, out_dtype: int = FFA_F32,
                       stream=None):
    """De-reddened copy of a device series (torch tensor of float32, bfloat16
    or float16): series minus its running median over `window` samples."""
    import torch
    dt = {torch.float32: FFA_F32, torch.bfloat16: FFA_BF16, torch.float16: FFA_F16}[series.dtype]
    tdt = {FFA_F32: torch.float32, FFA_BF16: torch.bfloat16, FFA_F16: torch.float16}[out_dtype]
    if out is None:
        out = torch.empty(series.numel(), dtype=tdt, device=series.device)
    _check(lib().ffa_running_median(ctx, series.data_ptr(), series.numel(), dt, window,
                                    out.data_ptr(), out_dtype, _stream(stream)), ctx)
    return out


def ffa_search_batch(ctx, series: Sequence, params: Sequence[ffa_search_params], snr=None,
                     row_offset: Optional[Sequence[int]] = None, use_graph: bool = False,
                     stream=None):
    """Periodograms of several device series (torch tensors, uneven lengths).
    Returns (snr, row_offset)."""
    import torch
    n = len(series)
    nsamp = [int(s.numel()) for s in series]
    if row_offset is None:
        rows = [ffa_plan_rows(p, ns) for p, ns in zip(params, nsamp)]
        row_offset = np.concatenate([[0], np.cumsum(rows)[:-1]]).astype(np.int64)
        total = int(sum(rows))
    else:
        total = None
    if snr is None:
        if total is None:
            rows = [ffa_plan_rows(p, ns) for p, ns in zip(params, nsamp)]
            total = int(max(o + r for o, r in zip(row_offset, rows)))
        snr = torch.empty((total, params[0].num_widths), dtype=torch.float32,
                          device=series[0].device)
    ptrs = (ctypes.c_void_p * n)(*[s.data_ptr() for s in series])
    ns = (ctypes.c_int64 * n)(*nsamp)
    prm = (ffa_search_params * n)(*params)
    ro = (ctypes.c_int64 * n)(*[int(v) for v in row_offset])
    st = lib().ffa_search_batch(ctx, n, ptrs, ns, prm, ro, snr.data_ptr(), snr.shape[0],
                                1 if use_graph else 0, _stream(stream))
    _check(st, ctx)
    return snr, np.asarray(row_offset, dtype=np.int64)


def ffa_search_ranges(ctx, series, ranges: Sequence[ffa_search_params], snr=None, stream=None):
    """Periodogram of one device series over consecutive period sub-ranges,
    each with its own parameters. Returns (periods, bins, snr, range_row0)."""
    import torch
    n = len(ranges)
    nsamp = int(series.numel())
    rows = [ffa_plan_rows(r, nsamp) for r in ranges]
    total = int(sum(rows))
    if snr is None:
        snr = torch.empty((total, ranges[0].num_widths), dtype=torch.float32, device=series.device)
    per = np.zeros(total, dtype=np.float64)
    bins = np.zeros(total, dtype=np.int32)
    row0 = np.zeros(n + 1, dtype=np.int64)
    prm = (ffa_search_params * n)(*ranges)
    st = lib().ffa_search_ranges(ctx, series.data_ptr(), nsamp, prm, n, per.ctypes.data,
                                 bins.ctypes.data, row0.ctypes.data, snr.data_ptr(),
                                 snr.shape[0], _stream(stream))
    _check(st, ctx)
    return per, bins, snr, row0


def ffa_transform(ctx, x, out=None, stream=None):
    """Folding transform of a device m x p float32 tensor."""
    import torch
    m, p = x.shape
    if out is None:
        out = torch.empty_like(x)
    _check(lib().ffa_transform(ctx, x.data_ptr(), m, p, out.data_ptr(), _stream(stream)), ctx)
    return out


def ffa_series_stats(ctx, series, dtype: int = FFA_F32, stream=None):
    import torch
    st = torch.empty(2, dtype=torch.float64, device=series.device)
    _check(lib().ffa_series_stats(ctx, series.data_ptr(), series.numel(), dtype, st.data_ptr(),
                                  _stream(stream)), ctx)
    return st


def ffa_downsample(ctx, series, ds_fx: int, nout: int, stats=None, dtype: int = FFA_F32,
                   stream=None):
    import torch
    tdt = {FFA_F32: torch.float32, FFA_BF16: torch.bfloat16, FFA_F16: torch.float16}[dtype]
    out = torch.empty(nout, dtype=tdt, device=series.device)
    _check(lib().ffa_downsample(ctx, series.data_ptr(), series.numel(), dtype,
                                _ptr(stats), ds_fx, nout, out.data_ptr(), _stream(stream)), ctx)
    return out


def ffa_sync_status(ctx, stream=None) -> int:
    return lib().ffa_sync_status(ctx, _stream(stream))


def ffa_get_tiling(ctx) -> ffa_tiling:
    t = ffa_tiling()
    _check(lib().ffa_get_tiling(ctx, ctypes.byref(t)), ctx)
    return t


def ffa_set_tiling(ctx, lds_rows: int = 0, levels_per_pass: int = 5,
                   persistent: bool = False, waves_per_group: int = 8,
                   range_waves_per_group: int = 0) -> None:
    t = ffa_tiling(lds_rows, levels_per_pass, 1 if persistent else 0, waves_per_group,
                   range_waves_per_group)
    _check(lib().ffa_set_tiling(ctx, ctypes.byref(t)), ctx)


def ffa_autotune(ctx, series: Sequence, params: Sequence[ffa_search_params],
                 cache_path: Optional[str] = None, stream=None) -> ffa_tiling:
    n = len(series)
    ptrs = (ctypes.c_void_p * n)(*[s.data_ptr() for s in series])
    ns = (ctypes.c_int64 * n)(*[int(s.numel()) for s in series])
    prm = (ffa_search_params * n)(*params)
    best = ffa_tiling()
    _check(lib().ffa_autotune(ctx, n, ptrs, ns, prm,
                              cache_path.encode() if cache_path else None, ctypes.byref(best),
                              _stream(stream)), ctx)
    return best


def ffa_set_timing(ctx, enable: bool) -> None:
    _check(lib().ffa_set_timing(ctx, 1 if enable else 0), ctx)


def ffa_read_timing(ctx, reset: bool = True) -> dict:
    t = ffa_kernel_times()
    _check(lib().ffa_read_timing(ctx, ctypes.byref(t), 1 if reset else 0), ctx)
    return t.as_dict()


def make_peak_params(dz_seg: float = 4.0, k_sigma: float = 6.0, degree: int = 2,
                     min_points: int = 16, cluster_gap: float = 1.0) -> ffa_peak_params:
    return ffa_peak_params(float(dz_seg), float(k_sigma), int(degree), int(min_points),
                           float(cluster_gap))


def ffa_find_peaks_batch(ctx, snr, params: Sequence[ffa_search_params], nsamp: Sequence[int],
                         row_offset: Sequence[int], peak_params: Optional[ffa_peak_params] = None,
                         capacity: int = 1 << 16, stream=None):
    """Peaks of the periodograms in `snr` (a device tensor written by
    ffa_search_batch). Returns (peaks: structured array of PEAK_DTYPE ordered
    by series, width and row; counts per series; threshold coefficients,
    series x widths x (degree + 1)). Raises FFAError with status
    FFA_ERR_BUFFER_TOO_SMALL when more than `capacity` peaks are found."""
    if peak_params is None:
        peak_params = make_peak_params()
    n = len(params)
    ns = (ctypes.c_int64 * n)(*[int(v) for v in nsamp])
    prm = (ffa_search_params * n)(*params)
    ro = (ctypes.c_int64 * n)(*[int(v) for v in row_offset])
    out = np.zeros(max(int(capacity), 1), dtype=PEAK_DTYPE)
    counts = np.zeros(n, dtype=np.int64)
    nw = params[0].num_widths
    poly = np.zeros((n, nw, peak_params.degree + 1), dtype=np.float64)
    st = lib().ffa_find_peaks_batch(
        ctx, n, ns, prm, ro, snr.data_ptr(), snr.shape[0], ctypes.byref(peak_params),
        out.ctypes.data, int(capacity), counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
        poly.ctypes.data, _stream(stream))
    if st == FFA_ERR_BUFFER_TOO_SMALL:
        raise FFAError(st, f"{int(counts.sum())} peaks found, capacity {capacity}")
    _check(st, ctx)
    return out[:int(counts.sum())].copy(), counts, poly


# ---------------------------------------------------------------------------
# Multi-DM pipeline pieces (Sec. 5.7): host computations, no context needed.
# ---------------------------------------------------------------------------

def _host_array(v, dtype):
    import numpy as np
    return np.ascontiguousarray(np.asarray(v, dtype=dtype))


def ffa_select_dm_trials(dms, f_lo_mhz: float, f_hi_mhz: float, max_smear_s: float):
    """Indices (ascending) of the DM trials to search."""
    import numpy as np
    d = _host_array(dms, np.float64)
    keep = np.empty(max(1, d.size), dtype=np.int32)
    nk = ctypes.c_int32(0)
    _check(lib().ffa_select_dm_trials(d.ctypes.data, d.size, float(f_lo_mhz), float(f_hi_mhz),
                                      float(max_smear_s), keep.ctypes.data, ctypes.byref(nk)))
    return keep[:nk.value].copy()


def ffa_cluster_frequencies(freq, snr, tol_hz: float):
    """(cluster of each peak, brightest peak of each cluster, member counts)."""
    import numpy as np
    f = _host_array(freq, np.float64)
    s = _host_array(snr, np.float32)
    if s.size != f.size:
        raise ValueError("freq and snr differ in length")
    n = f.size
    cl = np.empty(max(1, n), dtype=np.int32)
    br = np.empty(max(1, n), dtype=np.int32)
    mb = np.empty(max(1, n), dtype=np.int32)
    nc = ctypes.c_int32(0)
    _check(lib().ffa_cluster_frequencies(f.ctypes.data, s.ctypes.data, n, float(tol_hz),
                                         cl.ctypes.data, br.ctypes.data, mb.ctypes.data,
                                         ctypes.byref(nc)))
    return cl[:n].copy(), br[:nc.value].copy(), mb[:nc.value].copy()


def ffa_flag_harmonics(freq, snr, tol_hz: float, max_order: int = 8):
    """(parent or -1, ratio numerator, ratio denominator) of every entry."""
    import numpy as np
    f = _host_array(freq, np.float64)
    s = _host_array(snr, np.float32)
    if s.size != f.size:
        raise ValueError("freq and snr differ in length")
    n = f.size
    par = np.empty(max(1, n), dtype=np.int32)
    num = np.empty(max(1, n), dtype=np.int32)
    den = np.empty(max(1, n), dtype=np.int32)
    _check(lib().ffa_flag_harmonics(f.ctypes.data, s.ctypes.data, n, float(tol_hz), int(max_order),
                                    par.ctypes.data, num.ctypes.data, den.ctypes.data))
    return par[:n].copy(), num[:n].copy(), den[:n].copy()
