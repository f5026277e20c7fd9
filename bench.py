"""Benchmark of the FFA + boxcar S/N search on one MI355X.

One step = the whole hot path over one batch: FP64 statistics of every
series, every pseudo-octave downsampled, every FFA transform folded and every
kept profile's boxcar S/N written (the periodogram). Inputs are resident in
HBM before the timed region starts.

Workload (default): 512 series of 2^23 samples at 64 us (the paper's
benchmark shape, Sec. 5.8), N(0,1) noise with 10 % of the series carrying a
pulse; periods 0.5-10 s, 240-259 bins, 9 boxcar widths (1..48 bins). It is
run with the series stored as bfloat16 (normalised in FP64 beforehand), the
headline, and as plain float32 for comparison.

Each variant is timed twice over the same steps: with eager launches, each
bracketed by HIP events (the per-kernel times behind the roofline), and as
replays of the step captured in one hipGraph (the headline value).

Prints one JSON line (rank 0).
"""
import argparse
import concurrent.futures as cf
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP32 vector issue of the chip without packed FP32 (the kernels are built
# with packed FP32 disabled): 256 CUs x 64 lanes x 2.4 GHz, one op per lane
# and cycle, in 10^12 op/s
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--series", type=int, default=512)
    ap.add_argument("--log2n", type=int, default=23)
    ap.add_argument("--variants", default="bf16,f32,f16")
    ap.add_argument("--graph", type=int, default=1,
                    help="1: after the per-kernel timed steps, time the same steps again as "
                         "hipGraph replays (the headline value); 0: eager launches only")
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--ranges", type=int, default=64,
                    help="series of the dynamic duty-cycle leg (Sec. 5.6): 0.5-2 s at 240-259 "
                         "bins and 2-10 s at 480-519 bins, FP32; 0 skips it")
    ap.add_argument("--peaks", type=int, default=1,
                    help="1: also time peak detection (Sec. 5.5) on the headline variant's "
                         "periodograms, reported apart from the step")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--median", type=int, default=1,
                    help="1: also time the running-median de-reddening (Sec. 5.2) of the "
                         "workload-2 series, reported apart from the step")
    ap.add_argument("--workload", default="batch", choices=["batch", "uneven", "single"])
    ap.add_argument("--autotune", type=int, default=0,
                    help="autotune the tiling on --tune-series series first (the default tiling "
                         "is what the tuner picks for the batch workload)")
    ap.add_argument("--tune-series", type=int, default=16)
    ap.add_argument("--waves", type=int, default=8,
                    help="waves per workgroup of the first fold pass (8 or 16)")
    ap.add_argument("--range-waves", type=int, default=0,
                    help="waves per workgroup of the later fold passes (0: as --waves)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one device copy of this size first (counter calibration)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_inputs(torch, nseries, nsamp):
    import synth
    x = torch.empty((nseries, nsamp), dtype=torch.float32, device="cuda")
    pulsed = synth.workload3_pulsed(nseries)
    def gen(i):
        s, _ = synth.workload3_series(i, nsamp=nsamp, nseries=nseries, pulsed=pulsed)
        return i, s
    with cf.ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 4)) as ex:
        for i, s in ex.map(gen, range(nseries)):
            x[i].copy_(torch.from_numpy(s))
            if (i + 1) % 64 == 0:
                log(f"generated {i + 1}/{nseries} series")
    torch.cuda.synchronize()
    return x


def lowp(torch, x, dt):
    # normalised in FP64 per series, then rounded to the storage type (RNE)
    out = torch.empty(x.shape, dtype=dt, device=x.device)
    for i in range(x.shape[0]):
        xd = x[i].double()
        mu = xd.mean()
        sd = torch.sqrt(((xd - mu) ** 2).mean())
        out[i].copy_(((xd - mu) / sd).to(dt))
    torch.cuda.synchronize()
    return out


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("ffa_kernels.hip", "ffa_internal.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2004_03701_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def committed_traffic(workload, storage):
    """HBM bytes per step of the fold kernel from the committed rocprofv3
    counter summary, if it was taken on the kernel source as it is now."""
    path = os.path.join(ROOT, "profiles", "fold_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_src_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_step", {}).get(f"{workload}:{storage}")


def merge_rows(n, memo={}):
    """Rows produced by the merges of an n-row FFA tree (head floor(n/2),
    tail the rest, Sec. 2.2); each produced row costs p additions."""
    if n <= 1:
        return 0
    if n not in memo:
        memo[n] = n + merge_rows(n // 2) + merge_rows(n - n // 2)
    return memo[n]


def alg_ops_per_series(plan, num_widths):
    """Algorithmic FP32 operations of the fold kernel for one series: the
    merge additions of every transform plus, per kept profile, the prefix
    (p additions) and per width one subtraction and one maximum per phase."""
    xf = {}
    for k, p, m in zip(plan["octave"], plan["bins"], plan["m"]):
        xf[(int(k), int(p))] = int(m)
    merges = sum(p * merge_rows(m) for (_, p), m in xf.items())
    snr = int(plan["bins"].astype(np.int64).sum()) * (1 + 2 * num_widths)
    return merges + snr


def copy_ceiling(torch, mib=1024, reps=10):
    """GB/s of a plain device-to-device copy (read + write bytes), the
    practical ceiling of an HBM-bound kernel."""
    src = torch.ones(mib << 18, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * src.numel() * 4 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def bench_peaks(ffa, ctx, snr, prm, nsamp, rows1, a):
    """Peak detection of every series' periodogram, timed with HIP events
    around its three steps (control points, fit, selection and clustering)
    and by wall clock (the call includes its host work and the copy of the
    peaks to the host)."""
    import torch
    n = len(prm)
    ro = [i * rows1 for i in range(n)]
    ns = [nsamp] * n
    pp = ffa.make_peak_params()
    ffa.ffa_find_peaks_batch(ctx, snr, prm, ns, ro, pp, capacity=1 << 22)
    torch.cuda.synchronize()
    ffa.ffa_set_timing(ctx, True)
    ffa.ffa_read_timing(ctx, reset=True)
    t0 = time.perf_counter()
    for _ in range(a.steps):
        got, counts, _ = ffa.ffa_find_peaks_batch(ctx, snr, prm, ns, ro, pp, capacity=1 << 22)
    wall = (time.perf_counter() - t0) / a.steps
    tm = ffa.ffa_read_timing(ctx, reset=True)
    ffa.ffa_set_timing(ctx, False)
    kms = tm["peaks_ms"] / a.steps
    # the S/N array is read twice (control points, then the scan); the
    # frequency tables (16 B per row of the shared plan) once
    alg = 2 * snr.shape[0] * snr.shape[1] * 4 + 16 * rows1
    gbs = alg / (kms * 1e-3) / 1e9
    return {"ms_per_call": 1e3 * wall, "kernel_ms": kms,
            "timed_steps_per_call": tm["peaks_launches"] / a.steps, "alg_bytes": alg,
            "alg_GBps": gbs, "frac_of_hbm": gbs / HBM_PEAK_GBS, "peaks_found": int(counts.sum()),
            "params": {"dz_seg": pp.dz_seg, "k_sigma": pp.k_sigma, "degree": pp.degree,
                       "min_points": pp.min_points, "cluster_gap": pp.cluster_gap}}


def bench_ranges(ffa, ctx, x32, nsamp, cfg, a):
    """Dynamic duty-cycle resolution (Sec. 5.6) on the first a.ranges series:
    every series searched over two sub-ranges in one batch (each series an
    entry per sub-range), against the same series searched over 0.5-10 s at
    240-259 bins."""
    import torch
    n = min(a.ranges, x32.shape[0])
    series = [x32[i] for i in range(n)]
    sub = [(0.5, 2.0, 240, 259), (2.0, 10.0, 480, 519)]
    out = {"series": n, "ranges_s_bins": [list(r) for r in sub]}
    for name, rng in (("sub_ranges", sub), ("single_range", [(0.5, 10.0, 240, 259)])):
        prm = [ffa.make_params(cfg.tsamp, lo, hi, bmin, bmax, cfg.widths)
               for _ in range(n) for (lo, hi, bmin, bmax) in rng]
        ser = [x for x in series for _ in rng]
        snr, _ = ffa.ffa_search_batch(ctx, ser, prm)
        torch.cuda.synchronize()
        ffa.ffa_set_timing(ctx, True)
        ffa.ffa_read_timing(ctx, reset=True)
        t0 = time.perf_counter()
        for _ in range(a.steps):
            ffa.ffa_search_batch(ctx, ser, prm, snr=snr)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / a.steps
        tm = ffa.ffa_read_timing(ctx, reset=True)
        ffa.ffa_set_timing(ctx, False)
        rows = snr.shape[0]
        out[name] = {"ms_per_step": 1e3 * wall, "profiles": rows,
                     "profiles_per_s": rows / wall, "fold_ms": tm["fold_ms"] / a.steps}
        del snr
    return out


def cpu_baseline(seconds, nsamp):
    """The FP64 oracle, as it stands, on whole series of the same workload
    until `seconds` have passed (at least one series)."""
    import oracle
    import synth
    cfg = synth.workload3_config()
    pulsed = synth.workload3_pulsed()
    rows = 0
    done = 0
    t0 = time.perf_counter()
    while True:
        x, _ = synth.workload3_series(done, nsamp=nsamp, pulsed=pulsed)
        pg = oracle.search(x, cfg.tsamp, cfg.period_min, cfg.period_max, cfg.bins_min,
                           cfg.bins_max, cfg.widths)
        rows += pg.snr.shape[0]
        done += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": rows / dt, "unit": "profiles/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"{done} whole series of 2^{int(math.log2(nsamp))} samples, full plan "
                      f"({rows} profiles x 9 widths) in {dt:.1f} s, FP64 depth-first FFA"}


def cpu_model():
    """The host CPU's model name (lscpu, else /proc/cpuinfo)."""
    import subprocess
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in txt.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def main_uneven(a):
    """The uneven batch (256 series of 2^20..2^24 samples, three sampling
    times, two period ranges): tiling autotuned on the first 4 x --tune-series
    series against the fixed default, both timed on the whole batch."""
    import torch
    import paper_2004_03701_amd as ffa
    import synth
    nser = a.series if a.series != 512 else 256
    xs, prm = [], []
    for i in range(nser):
        x, cfg, _ = synth.workload5_series(i)
        xs.append(torch.from_numpy(x).cuda())
        prm.append(ffa.make_params(cfg.tsamp, cfg.period_min, cfg.period_max, cfg.bins_min,
                                   cfg.bins_max, cfg.widths))
        if (i + 1) % 64 == 0:
            log(f"generated {i + 1}/{nser} series")
    rows = [ffa.ffa_plan_rows(p, x.numel()) for p, x in zip(prm, xs)]
    ctx = ffa.ffa_create(0)
    snr = torch.empty((sum(rows), 9), dtype=torch.float32, device="cuda")
    out = {}
    for name in ("default", "autotuned"):
        ffa.ffa_set_tiling(ctx)
        if name == "autotuned":
            k = min(len(xs), 4 * a.tune_series)  # a representative share of the batch
            t = ffa.ffa_autotune(ctx, xs[:k], prm[:k])
            log(f"autotuned on {k} series")
            out["tiling"] = {"waves_per_group": t.waves_per_group,
                             "levels_per_pass": t.levels_per_pass, "persistent": t.persistent,
                             "lds_rows": t.lds_rows}
        for _ in range(a.warmup):
            ffa.ffa_search_batch(ctx, xs, prm, snr=snr)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            ffa.ffa_search_batch(ctx, xs, prm, snr=snr)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / a.steps
        out[name] = {"ms_per_step": ms, "profiles_per_s": sum(rows) / (ms * 1e-3)}
        log(f"{name}: {ms:.2f} ms/step")
    ffa.ffa_destroy(ctx)
    r = out["autotuned"]
    print(json.dumps({
        "metric": "trial profiles/sec (FFA+S/N), uneven batch, autotuned vs default tiling, 1 GPU",
        "value": r["profiles_per_s"], "unit": "profiles/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{nser} series of 2^20-2^24 samples, tsamp 64/128/256 us, "
                               "periods 0.1-1 s or 1-30 s, bins 240-259, 9 widths"},
        "speedup_vs_default": out["default"]["ms_per_step"] / r["ms_per_step"],
        "variants": out}), flush=True)


def bench_median(ffa, ctx, torch, a):
    """Running-median de-reddening (Sec. 5.2) of the workload-2 series
    (9,375,000 samples, 78,125-sample window), apart from the step: kernel
    time from HIP events, algorithmic bytes (one read and one write of the
    series, FP32) against 8 TB/s, and the oracle on the same series."""
    import synth
    x, cfg, _ = synth.workload2()
    dev = torch.from_numpy(x).cuda()
    out = torch.empty_like(dev)
    for _ in range(2):
        ffa.ffa_running_median(ctx, dev, cfg.median_window, out=out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    e0.record()
    for _ in range(reps):
        ffa.ffa_running_median(ctx, dev, cfg.median_window, out=out)
    e1.record()
    torch.cuda.synchronize()
    assert ffa.ffa_sync_status(ctx) == ffa.FFA_OK
    ms = e0.elapsed_time(e1) / reps
    alg = 8 * x.size
    res = {"samples": int(x.size), "window": cfg.median_window, "ms_per_call": ms,
           "samples_per_s": x.size / (ms * 1e-3), "alg_bytes": alg,
           "alg_GBps": alg / (ms * 1e-3) / 1e9, "frac_of_hbm": alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    if a.cpu_baseline:
        import oracle
        t0 = time.perf_counter()
        oracle.running_median(x, cfg.median_window)
        res["cpu_oracle_ms"] = 1e3 * (time.perf_counter() - t0)
    log(f"running median: {ms:.3f} ms per call")
    del dev, out
    return res


def main_single(a):
    """Single series (workloads 1 and 2): launch- and latency-bound searches,
    timed as eager per-pass launches, as hipGraph replays, and as graph
    replays of one persistent launch, next to the oracle on the same series."""
    import torch
    import paper_2004_03701_amd as ffa
    import oracle
    import synth
    ctx = ffa.ffa_create(0)
    out = {}
    for wl, make in (("workload1", synth.workload1), ("workload2", synth.workload2)):
        x, cfg, _ = make()
        dev = torch.from_numpy(x.astype(np.float32)).cuda()
        prm = ffa.make_params(cfg.tsamp, cfg.period_min, cfg.period_max, cfg.bins_min,
                              cfg.bins_max, cfg.widths, median_window=cfg.median_window)
        rows = ffa.ffa_plan_rows(prm, dev.numel())
        snr = torch.empty((rows, len(cfg.widths)), dtype=torch.float32, device="cuda")
        res = {"samples": int(dev.numel()), "profiles": rows, "median_window": cfg.median_window}
        for name, persistent, graph in (("eager", 0, False), ("graph", 0, True),
                                        ("persistent_graph", 1, True)):
            ffa.ffa_set_tiling(ctx, persistent=persistent)
            for _ in range(max(a.warmup, 1)):
                ffa.ffa_search_batch(ctx, [dev], [prm], snr=snr, use_graph=graph)
            torch.cuda.synchronize()
            reps = 10 * a.steps
            t0 = time.perf_counter()
            for _ in range(reps):
                ffa.ffa_search_batch(ctx, [dev], [prm], snr=snr, use_graph=graph)
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0) / reps
            res[name] = {"ms_per_search": ms, "profiles_per_s": rows / (ms * 1e-3)}
            log(f"{wl} {name}: {ms:.3f} ms")
        ffa.ffa_set_tiling(ctx)
        if a.cpu_baseline:
            t0 = time.perf_counter()
            oracle.search(x, cfg.tsamp, cfg.period_min, cfg.period_max, cfg.bins_min,
                          cfg.bins_max, cfg.widths, median_window=cfg.median_window)
            dt = time.perf_counter() - t0
            res["cpu_oracle"] = {"ms_per_search": 1e3 * dt, "profiles_per_s": rows / dt,
                                 "cores": int(os.environ.get("OMP_NUM_THREADS",
                                                             os.cpu_count() or 1))}
        out[wl] = res
        del dev, snr
    ffa.ffa_destroy(ctx)
    best = max(out["workload2"][k]["profiles_per_s"] for k in ("eager", "graph",
                                                                 "persistent_graph"))
    r2 = out["workload2"]
    print(json.dumps({
        "metric": "trial profiles/sec (FFA+S/N), one series, 1 GPU",
        "value": best, "unit": "profiles/s", "n_gpus": 1, "steps": 10 * a.steps,
        "warmup": a.warmup, "ms_per_step": min(r2[k]["ms_per_search"] for k in
                                               ("eager", "graph", "persistent_graph")),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "workload 2: 9,375,000 samples at 64 us, periods 0.5-10 s, "
                               "bins 240-259, 9 widths (workload 1: 2^18 samples, periods "
                               "128-256 samples, bins 128-255, also reported)"},
        "variants": out}), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "the benchmark measures one GPU (series shard across GPUs with no exchange: run one process per GPU on its share); --gpus must be 1"}))
        sys.exit(2)
    if a.workload == "uneven":
        return main_uneven(a)
    if a.workload == "single":
        return main_single(a)
    import torch
    import paper_2004_03701_amd as ffa
    import synth

    if a.calib_copy_mib:
        src = torch.empty(a.calib_copy_mib << 18, dtype=torch.float32, device="cuda")
        src.fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy of {a.calib_copy_mib} MiB done")
        del src, dst
    copy_gbs = copy_ceiling(torch)
    log(f"device copy: {copy_gbs:.0f} GB/s")
    nsamp = 1 << a.log2n
    cfg = synth.workload3_config()
    x32 = make_inputs(torch, a.series, nsamp)
    variants = [v for v in a.variants.split(",") if v]
    store = {"f32": (ffa.FFA_F32, None), "bf16": (ffa.FFA_BF16, torch.bfloat16),
             "f16": (ffa.FFA_F16, torch.float16)}
    ctx = ffa.ffa_create(0)
    results = {}
    for v in variants:
        log(f"variant {v}")
        dt_code, tdt = store[v]
        xs = x32 if tdt is None else lowp(torch, x32, tdt)
        series = [xs[i] for i in range(a.series)]
        prm = [ffa.make_params(cfg.tsamp, cfg.period_min, cfg.period_max, cfg.bins_min,
                               cfg.bins_max, cfg.widths, normalise=True, dtype=dt_code)
               for _ in range(a.series)]
        rows1 = ffa.ffa_plan_rows(prm[0], nsamp)
        plan = ffa.ffa_plan_export(prm[0], nsamp)
        bins = plan["bins"].astype(np.int64)
        alg_ops = a.series * alg_ops_per_series(plan, len(cfg.widths))
        snr = torch.empty((rows1 * a.series, len(cfg.widths)), dtype=torch.float32,
                          device="cuda")
        ffa.ffa_set_tiling(ctx, waves_per_group=a.waves, range_waves_per_group=a.range_waves)
        tiling = {"waves_per_group": a.waves, "range_waves_per_group": a.range_waves}
        if a.autotune:
            k = min(a.tune_series, a.series)
            t = ffa.ffa_autotune(ctx, series[:k], prm[:k])
            tiling = {"waves_per_group": t.waves_per_group, "levels_per_pass": t.levels_per_pass,
                      "persistent": t.persistent, "lds_rows": t.lds_rows,
                      "range_waves_per_group": t.range_waves_per_group}
            log(f"variant {v}: autotuned on {k} series -> {tiling}")
        for _ in range(a.warmup):
            ffa.ffa_search_batch(ctx, series, prm, snr=snr)
        torch.cuda.synchronize()
        log(f"variant {v}: warm-up done, timing {a.steps} steps (per-kernel HIP events)")
        # eager launches, each bracketed by HIP events on its stream
        ffa.ffa_set_timing(ctx, True)
        ffa.ffa_read_timing(ctx, reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            ffa.ffa_search_batch(ctx, series, prm, snr=snr)
        torch.cuda.synchronize()
        wall_eager = time.perf_counter() - t0
        tm = ffa.ffa_read_timing(ctx, reset=True)
        ffa.ffa_set_timing(ctx, False)
        assert ffa.ffa_sync_status(ctx) == ffa.FFA_OK
        wall = wall_eager
        graph_ms = None
        if a.graph:
            # the same steps as replays of one captured hipGraph
            ffa.ffa_search_batch(ctx, series, prm, snr=snr, use_graph=True)  # capture
            torch.cuda.synchronize()
            log(f"variant {v}: timing {a.steps} graph replays")
            t0 = time.perf_counter()
            for _ in range(a.steps):
                ffa.ffa_search_batch(ctx, series, prm, snr=snr, use_graph=True)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            graph_ms = 1e3 * wall / a.steps
            assert ffa.ffa_sync_status(ctx) == ffa.FFA_OK
        ffa.ffa_set_tiling(ctx)
        ms = 1e3 * wall / a.steps
        profiles = rows1 * a.series
        esize = 4 if tdt is None else 2  # the folded (downsampled) series: the storage type
        alg_bytes = a.series * (int(bins.sum()) * esize + rows1 * len(cfg.widths) * 4)
        alg_bytes_f32 = a.series * (int(bins.sum()) * 4 + rows1 * len(cfg.widths) * 4)
        fold_ms = tm["fold_ms"] / a.steps if tm["fold_launches"] else None
        res = {"ms_per_step": ms, "profiles_per_s": profiles / (ms * 1e-3),
               "profiles": profiles, "alg_bytes_fold": alg_bytes,
               "alg_bytes_fold_f32": alg_bytes_f32, "alg_ops_fold": alg_ops,
               "timing": tm,
               "tiling": tiling, "eager_ms_per_step": 1e3 * wall_eager / a.steps,
               "graph_ms_per_step": graph_ms}
        if fold_ms:
            res["fold_ms_per_step"] = fold_ms
            res["fold_launches_per_step"] = tm["fold_launches"] / a.steps
            res["fold_alg_GBps"] = alg_bytes / (fold_ms * 1e-3) / 1e9
            res["fold_alg_Tops"] = alg_ops / (fold_ms * 1e-3) / 1e12
            res["stats_ms_per_step"] = tm["stats_ms"] / a.steps
            res["downsample_ms_per_step"] = tm["downsample_ms"] / a.steps
        if a.peaks and v == variants[0]:
            res["peaks"] = bench_peaks(ffa, ctx, snr, prm, nsamp, rows1, a)
        results[v] = res
        del series, xs, snr
        torch.cuda.empty_cache()
    ranges_res = bench_ranges(ffa, ctx, x32, nsamp, cfg, a) if a.ranges else None
    del x32
    torch.cuda.empty_cache()
    median_res = bench_median(ffa, ctx, torch, a) if a.median else None
    head = variants[0]
    r = results[head]
    out = {
        "metric": "trial profiles/sec and HBM GB/s (FFA+S/N), batched BF16 vs plain FP32, 1 GPU",
        "value": r["profiles_per_s"],
        "unit": "profiles/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{a.series} series x 2^{a.log2n} samples at 64 us, periods "
                               f"0.5-10 s, bins 240-259, widths 1-48 (9), storage {head}",
                   "storage": head, "series": a.series, "nsamp": nsamp,
                   "graph": bool(a.graph)},
    }
    if "fold_alg_GBps" in r:
        ach = r["fold_alg_GBps"]
        tb = committed_traffic("batch", head)
        out["roofline"] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": ach / HBM_PEAK_GBS,
                           "traffic": (tb / (r["fold_ms_per_step"] * 1e-3) / 1e9) if tb else None,
                           "kernel": "k_ffa_pass (all fold launches of a step)",
                           "bytes_per_input_sample": 4 if head == "f32" else 2,
                           "frac_at_fp32_bytes": (r["alg_bytes_fold_f32"] /
                                                  (r["fold_ms_per_step"] * 1e-3) / 1e9 /
                                                  HBM_PEAK_GBS),
                           "fold_ms_per_step": r["fold_ms_per_step"],
                           "copy_GBps": copy_gbs, "frac_of_copy": ach / copy_gbs,
                           "alu": {"achieved": r["fold_alg_Tops"], "peak": VALU_PEAK_TOPS,
                                   "unit": "Top/s",
                                   "frac": r["fold_alg_Tops"] / VALU_PEAK_TOPS}}
    if "peaks" in r:
        out["peaks"] = r["peaks"]
    if ranges_res:
        out["ranges"] = ranges_res
    if median_res:
        out["median"] = median_res
    out["variants"] = {k: {kk: vv for kk, vv in v.items() if kk not in ("timing", "peaks")}
                       for k, v in results.items()}
    if "f32" in results and head != "f32":
        out["speedup_vs_f32"] = results[head]["profiles_per_s"] / results["f32"]["profiles_per_s"]
    if a.cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(a.cpu_seconds, nsamp)
    ffa.ffa_destroy(ctx)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
