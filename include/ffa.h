/*
 * ffa.h -- C ABI of the MI355X FFA periodicity search.
 *
 * The library computes the hot path of the search described by Morello,
 * Barr, Stappers, Keane & Lyne (2020), "Optimal periodicity searching:
 * revisiting the Fast Folding Algorithm for large-scale pulsar surveys":
 * normalise a time series (Sec. 5.2), downsample it for every pseudo-octave
 * of a period range (Sec. 5.3), fold it at every trial period with the FFA
 * (Sec. 2), and evaluate the boxcar matched-filter S/N of every folded
 * profile (Sec. 5.4), giving the two-dimensional periodogram of Sec. 5.5.
 *
 * Conventions shared by every call:
 *   - Every call returns an ffa_status: FFA_OK (0) or a negative error code.
 *     No C++ exception crosses the ABI.
 *   - Arguments are validated before any device work is queued; on error
 *     nothing is written except the context's last-error message.
 *   - Pointers documented as DEVICE point to memory on the context's GPU
 *     (for instance torch tensor storage); HOST pointers point to host memory.
 *     The caller owns every buffer passed in; the context owns its workspace.
 *   - `stream` is a hipStream_t (NULL = the default stream). Device work is
 *     queued on it asynchronously: device outputs are valid once the stream
 *     has synchronised. Host outputs are written before the call returns.
 *   - A context is used by one host thread at a time.
 */
#ifndef FFA_MI355X_H
#define FFA_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FFA_OK = 0,
  FFA_ERR_INVALID_ARG = -1,      /* a null pointer, a size or a parameter out of its domain */
  FFA_ERR_RANGE = -2,            /* period_min / (bins_min * tsamp) < 1, or no transform with m >= 2 */
  FFA_ERR_BUFFER_TOO_SMALL = -3, /* capacity below the number of periodogram rows */
  FFA_ERR_NOMEM = -4,            /* device or host allocation failed */
  FFA_ERR_DEVICE = -5,           /* a HIP runtime call failed */
  FFA_ERR_DEGENERATE = -6,       /* zero or non-finite variance of a series to normalise */
  FFA_ERR_NOT_IMPLEMENTED = -7
} ffa_status;

/* Storage type of an input series (and of its downsampled series). Arithmetic
 * is FP32 (FP64 for the normalisation statistics and the S/N noise constants)
 * whatever the storage. */
typedef enum { FFA_F32 = 0, FFA_BF16 = 1, FFA_F16 = 2 } ffa_dtype;

typedef struct ffa_ctx ffa_ctx;

/* The search of one series (Sec. 5.3 - 5.5).
 *   tsamp        sampling time tau of the series, seconds, > 0.
 *   period_min   P_min, seconds; period_max P_max > period_min. The first
 *                downsampling factor is ds0 = P_min / (bins_min * tsamp) and
 *                must be >= 1 (FFA_ERR_RANGE otherwise).
 *   bins_min, bins_max
 *                number of phase bins per folded profile, 2 <= min <= max.
 *                Pseudo-octave k downsamples the original series by
 *                ds0 * f^k, f = (bins_max + 1) / bins_min (Sec. 5.3).
 *   widths       HOST array of num_widths boxcar widths in bins, strictly
 *                increasing, 1 <= w < bins_min (Sec. 5.4), at most 32 widths.
 *   normalise    1: subtract the mean and divide by the population standard
 *                deviation of the whole series, both computed in FP64 on the
 *                device (Sec. 5.2); 0: the series is used as given (it should
 *                then have zero mean and unit variance).
 *   dtype        ffa_dtype of the series. The statistics and the
 *                downsampler read it in this type, and the downsampled
 *                series are stored in it too (a BF16 or FP16 search reads
 *                half the bytes of an FP32 one); the fold converts them on
 *                load, and every sum from there on is FP32. With FP16 storage
 *                the downsampled samples must fit FP16 (as they do for a
 *                normalised series).
 *   median_window  0: no de-reddening; otherwise an odd number of samples:
 *                the running median over that window is subtracted from the
 *                series first (Sec. 5.2; see ffa_running_median), the result
 *                kept in the storage type, and normalisation (if asked) and
 *                everything after it use the de-reddened series. */
typedef struct {
  double tsamp;
  double period_min;
  double period_max;
  int32_t bins_min;
  int32_t bins_max;
  const int32_t* widths;
  int32_t num_widths;
  int32_t normalise;
  int32_t dtype;
  int32_t median_window;
} ffa_search_params;

/* Creates a context on HIP device `device`. *out receives the handle. */
ffa_status ffa_create(int device, ffa_ctx** out);

/* Waits for the context's work, frees its workspace and the handle. NULL is a no-op. */
ffa_status ffa_destroy(ffa_ctx* ctx);

/* Static English text of a status code. */
const char* ffa_status_string(ffa_status s);

/* Message of the last failed call on ctx ("" if none); valid until the next
 * call on ctx. */
const char* ffa_last_error(const ffa_ctx* ctx);

/* Number of periodogram rows of a series of nsamp samples (Sec. 2.3, 5.3):
 * the kept trial periods of every transform of every pseudo-octave. A row of
 * transform (k, p) with m rows is kept when its period
 * P_s = tau_k p^2 / (p - s/(m-1)) is below both (p + 1) tau_k, past which
 * trials overlap the next transform (Sec. 2.3), and P_max. Host only. */
ffa_status ffa_plan_rows(const ffa_search_params* params, int64_t nsamp, int64_t* rows);

/* Exports the plan row by row, in periodogram order (octave k, bins p, row s;
 * ascending period). Every HOST array holds `capacity` entries; any may be
 * NULL. period: P_s in seconds (Eq. for P_s, Sec. 2.3); bins: p; m: rows of
 * the transform; s: row index; octave: k; ds_fx: downsampling factor of the
 * octave in 32.32 fixed point. FFA_ERR_BUFFER_TOO_SMALL if capacity < rows. */
ffa_status ffa_plan_export(const ffa_search_params* params, int64_t nsamp, double* period,
                           int32_t* bins, int32_t* m, int32_t* s, int32_t* octave,
                           uint64_t* ds_fx, int64_t capacity);

/* Periodogram of one series (Sec. 5.3 - 5.5).
 * The widest downsampling window of the plan (the last pseudo-octave's
 * factor, about period_max / (bins_min tsamp)) must satisfy floor(ds) <=
 * 16,382, as for ffa_downsample; FFA_ERR_INVALID_ARG otherwise.
 *   series       DEVICE, nsamp samples of params->dtype.
 *   period_host  HOST, capacity_rows doubles or NULL: trial period of each row.
 *   bins_host    HOST, capacity_rows int32 or NULL: bins p of each row.
 *   snr_dev      DEVICE, capacity_rows x num_widths FP32, row-major: for each
 *                kept trial period and boxcar width, the best S/N over phase.
 * A degenerate series (zero or non-finite variance with normalise = 1) gives
 * NaN S/N; ffa_sync_status then reports FFA_ERR_DEGENERATE. */
ffa_status ffa_search(ffa_ctx* ctx, const void* series, int64_t nsamp,
                      const ffa_search_params* params, double* period_host, int32_t* bins_host,
                      float* snr_dev, int64_t capacity_rows, void* stream);

/* Periodograms of nseries series of uneven lengths and parameters.
 *   series       HOST array of nseries DEVICE pointers.
 *   nsamp        HOST array of nseries lengths.
 *   params       HOST array of nseries parameter sets (their num_widths must
 *                all be equal).
 *   row_offset   HOST array of nseries: first row of series i in snr_dev; the
 *                rows of series i are [row_offset[i], row_offset[i] + rows_i).
 *   snr_dev      DEVICE, capacity_rows x num_widths FP32.
 *   use_graph    1: capture the device work of the call in a hipGraph the
 *                first time a batch of this shape is seen and replay it on
 *                later calls with the same shape and pointers; 0: launch
 *                directly. */
ffa_status ffa_search_batch(ffa_ctx* ctx, int32_t nseries, const void* const* series,
                            const int64_t* nsamp, const ffa_search_params* params,
                            const int64_t* row_offset, float* snr_dev, int64_t capacity_rows,
                            int32_t use_graph, void* stream);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid allocation): ffa_search with no
 * device allocation of its own. Arguments, outputs and errors as ffa_search.
 * Every intermediate buffer (the tables of the search, the de-reddened copy
 * of the series when params->median_window > 0, the statistics, the
 * downsampled series and the scratch rows between passes) is carved from a
 * static device workspace of FFA_NOALLOC_WORKSPACE_BYTES that each device the
 * library runs on holds until the process ends; the call allocates no device
 * memory, but it waits for `stream` once, after copying its tables into the
 * workspace and before queueing its kernels. Limits: the series' tables and
 * downsampled samples plus two scratch buffers, each holding the largest
 * transform's m * p floats, must fit the workspace (a 2^23-sample series over
 * 0.5 - 10 s at 64 us and 240 - 259 bins does, with room to spare); otherwise
 * FFA_ERR_INVALID_ARG with a message, and nothing is queued. The tiling is the
 * context's with per-pass launches (its persistent flag is ignored).
 * All calls on one device share the workspace, which keeps the last call's
 * contents: calls that overlap on one device (other streams, other threads,
 * other contexts) race and must not be made. The workspace's status word is
 * cleared by each call; ffa_sync_status reports a degenerate series of the
 * latest call. */
#define FFA_NOALLOC_WORKSPACE_BYTES (128u << 20)
ffa_status ffa_search_noalloc(ffa_ctx* ctx, const void* series, int64_t nsamp,
                              const ffa_search_params* params, double* period_host,
                              int32_t* bins_host, float* snr_dev, int64_t capacity_rows,
                              void* stream);

/* Dynamic duty-cycle resolution (Sec. 5.6): the period range of one series
 * split into nranges consecutive sub-ranges, each searched with its own
 * parameters (typically more phase bins at longer periods), the periodograms
 * concatenated in range order.
 *   series, nsamp  DEVICE series of nsamp samples, as ffa_search.
 *   ranges       HOST array of nranges parameter sets with equal tsamp,
 *                normalise, dtype and widths (so w_max < every bins_min), in
 *                ascending period order without overlap (period_max of range k
 *                <= period_min of range k + 1); FFA_ERR_INVALID_ARG otherwise.
 *   period_host, bins_host  HOST or NULL, as ffa_search, over all rows.
 *   range_row0   HOST, nranges + 1 int64 or NULL: first row of each range
 *                and, last, the total number of rows.
 *   snr_dev      DEVICE, capacity_rows x num_widths FP32.
 * The series is normalised (if asked) and downsampled once per range. */
ffa_status ffa_search_ranges(ffa_ctx* ctx, const void* series, int64_t nsamp,
                             const ffa_search_params* ranges, int32_t nranges,
                             double* period_host, int32_t* bins_host, int64_t* range_row0,
                             float* snr_dev, int64_t capacity_rows, void* stream);

/* Folding transform alone (Sec. 2.1, 2.2), for parity checks: in and out are
 * DEVICE m x p FP32 arrays, row-major; row s of out is the profile folded along
 * the path that drifts s bins over the m rows. 1 <= m, 2 <= p <= 1280,
 * m * p < 2^31. */
ffa_status ffa_transform(ffa_ctx* ctx, const float* in, int32_t m, int32_t p, float* out,
                         void* stream);

/* Normalisation statistics (Sec. 5.2): stats_dev (DEVICE, 2 doubles) receives
 * the mean and the population standard deviation of the series, computed in
 * FP64. */
ffa_status ffa_series_stats(ffa_ctx* ctx, const void* series, int64_t nsamp, int32_t dtype,
                            double* stats_dev, void* stream);

/* Real-factor downsampling (Sec. 5.3, App. A.4) of one series: output j is
 * the overlap-weighted sum of the normalised input over the window
 * [j ds, (j+1) ds), ds = ds_fx / 2^32 samples; with stats_dev = NULL no
 * normalisation is applied, else (x - mean) / std with stats_dev as written by
 * ffa_series_stats. out_dev (DEVICE, 16-byte aligned) receives nout samples
 * of `dtype`; nout <= floor(nsamp * 2^32 / ds_fx), ds_fx >= 2^32, and the
 * window must leave a downsampling block room: floor(ds_fx / 2^32) <= 16,382.
 * FFA_ERR_INVALID_ARG otherwise. */
ffa_status ffa_downsample(ffa_ctx* ctx, const void* series, int64_t nsamp, int32_t dtype,
                          const double* stats_dev, uint64_t ds_fx, int64_t nout, void* out_dev,
                          void* stream);

/* De-reddening by a running median (Sec. 5.2): the low-frequency noise
 * subtracted before the series is normalised and searched. out[i] =
 * series[i] - the median of the `window` samples centred on i (window odd,
 * >= 1), the window cut at the ends of the series; the median of n samples
 * is their ((n - 1) / 2)-th smallest value, 0-based (the lower middle value
 * for an even count, which only occurs at the ends). The filter leaves any
 * constant impulse narrower than half the window intact. series: DEVICE,
 * nsamp samples of `dtype`; out_dev: DEVICE, nsamp samples of `out_dtype`
 * (may not alias series). The median is one of the samples, so with FP32
 * output the result is the exact difference rounded once. Non-finite
 * samples give unspecified medians. Asynchronous on `stream`. */
ffa_status ffa_running_median(ffa_ctx* ctx, const void* series, int64_t nsamp, int32_t dtype,
                              int32_t window, void* out_dev, int32_t out_dtype, void* stream);

/* Waits for the stream and reports FFA_ERR_DEGENERATE if a series normalised
 * since the previous call to ffa_sync_status had zero or non-finite variance. */
ffa_status ffa_sync_status(ffa_ctx* ctx, void* stream);

/* Tile shapes and scheduling of the search kernels. lds_rows: rows of a
 * profile tile held in LDS (0 = the largest that fits); levels_per_pass:
 * merge levels per pass above the bottom subtrees (1..5); persistent: 1 runs
 * all passes of a group of series in one persistent launch (tiles taken in
 * ticket order, later passes waiting on per-transform completion counters),
 * 0 launches one kernel per pass; waves_per_group: 16 (one workgroup per CU
 * with all 160 KiB of LDS) or 8 (two workgroups per CU, 80 KiB each);
 * range_waves_per_group: the same for the passes after the first (range
 * tiles), 0 = as waves_per_group (a persistent launch uses waves_per_group for
 * every pass). */
typedef struct {
  int32_t lds_rows;
  int32_t levels_per_pass;
  int32_t persistent;
  int32_t waves_per_group;
  int32_t range_waves_per_group;
} ffa_tiling;

/* Reads or sets the context's tiling. */
ffa_status ffa_get_tiling(const ffa_ctx* ctx, ffa_tiling* out);
ffa_status ffa_set_tiling(ffa_ctx* ctx, const ffa_tiling* tiling);

/* Times candidate tilings (8 or 16 waves per workgroup, the same or the other
 * size for the range passes, 3, 4 or 5 levels per pass, per-pass or persistent
 * launches, the largest tile that fits or tiles of at most 40 rows) on a
 * representative batch (same
 * arguments as ffa_search_batch; outputs go to a context-owned buffer) with
 * HIP events on `stream`, keeps the fastest in the context and, if cache_path
 * is not NULL, appends it to that text file keyed by a hash of the batch's
 * shape; a later call with the same shape and file reads the choice back
 * without timing. *best receives the chosen tiling (may be NULL). The call
 * synchronises the stream. */
ffa_status ffa_autotune(ffa_ctx* ctx, int32_t nseries, const void* const* series,
                        const int64_t* nsamp, const ffa_search_params* params,
                        const char* cache_path, ffa_tiling* best, void* stream);

/* Periodogram peak detection (Sec. 5.5 and its peak-detection figure).
 * Each width trial is searched on its own. Its S/N against trial frequency
 * nu = 1 / P is cut into segments of width dz_seg / T (T = nsamp * tsamp,
 * the length of the series; segment i covers [nu_lo + i dnu, nu_lo +
 * (i + 1) dnu), nu_lo the lowest trial frequency). A segment of at least
 * min_points rows, all finite, gives a control point at its centre
 * frequency: median + k_sigma * IQR / 1.349, the quartiles taken by linear
 * interpolation between order statistics. A polynomial of the given degree
 * in log(nu), fitted to the control points by unweighted least squares, is
 * the threshold (none with fewer than degree + 1 control points). The rows
 * whose S/N exceeds it form clusters, in frequency order, while consecutive
 * members are at most cluster_gap / T apart; a peak is the brightest member
 * of a cluster (the first in row order on equal S/N). */
typedef struct {
  double dz_seg;       /* segment width in units of 1 / T, > 0 (the paper: a few) */
  double k_sigma;      /* threshold height in robust sigmas (the paper's default: 6) */
  int32_t degree;      /* polynomial degree, 0..4 (the paper's default: 2) */
  int32_t min_points;  /* fewest rows of a segment with a control point, >= 1 */
  double cluster_gap;  /* largest frequency step inside a cluster, units of 1 / T, >= 0 */
} ffa_peak_params;

typedef struct {
  int64_t row;         /* row of the peak's brightest member in its series' periodogram */
  double period;       /* trial period of that row, seconds */
  double threshold;    /* threshold at that row */
  float snr;           /* S/N of that row and width */
  int32_t series;      /* index of the series in the call */
  int32_t width_index; /* index of the boxcar width */
  int32_t members;     /* rows above the threshold in the cluster */
} ffa_peak;

/* Peaks of the periodograms of nseries series, as written by
 * ffa_search_batch with the same nsamp, params and row_offset (HOST arrays of
 * nseries; num_widths equal across series). snr_dev (DEVICE, capacity_rows x
 * num_widths FP32) is read only. Every segment may hold at most 8192 rows
 * (FFA_ERR_INVALID_ARG otherwise; lower dz_seg).
 *   peaks_host   HOST, capacity_peaks records: the peaks ordered by series,
 *                width and row. Not written when there are more peaks than
 *                capacity_peaks; the call then returns FFA_ERR_BUFFER_TOO_SMALL.
 *   npeaks_host  HOST, nseries counts of peaks per series (always written on
 *                success and on FFA_ERR_BUFFER_TOO_SMALL).
 *   poly_host    HOST, nseries x num_widths x (degree + 1) doubles, or NULL:
 *                the threshold's coefficients c_0 .. c_degree in powers of
 *                log(nu); NaN for a width without a threshold.
 * The call waits for `stream`. A periodogram with non-finite S/N (a
 * degenerate series) gives no control point in the segments it touches. */
ffa_status ffa_find_peaks_batch(ffa_ctx* ctx, int32_t nseries, const int64_t* nsamp,
                                const ffa_search_params* params, const int64_t* row_offset,
                                const float* snr_dev, int64_t capacity_rows,
                                const ffa_peak_params* peak_params, ffa_peak* peaks_host,
                                int64_t capacity_peaks, int64_t* npeaks_host, double* poly_host,
                                void* stream);

/* ------------------------------------------------------------------------
 * Multi-DM pipeline pieces (Sec. 5.7). The search runs once per dispersion
 * measure (DM) trial; around it the paper chooses the DM trials to search by
 * the classical smearing rule, groups the peaks of all trials into clusters
 * in frequency and flags clusters that are harmonics of others. The paper
 * gives no rules for these; the ones below are this library's. All three are
 * host computations on host arrays (lists of a few thousand entries) and need
 * no context or GPU. Each returns FFA_ERR_INVALID_ARG (nothing written) for a
 * null pointer, a negative count, or the conditions named.
 * ------------------------------------------------------------------------ */

/* The DM trials to search. A DM error dDM smears a pulse across the band by
 * k_DM * dDM * (f_lo^-2 - f_hi^-2), k_DM = 4.148808e3 s MHz^2 pc^-1 cm^3;
 * the DM step is the dDM whose half gives max_smear_s. Of the given trials,
 * the fewest are chosen such that every given trial lies within half a step
 * of a chosen one (greedy from the lowest DM, which is optimal on a line).
 *   dm         HOST, n DM trials in pc cm^-3, ascending (else an error).
 *   f_lo_mhz, f_hi_mhz  band edges, 0 < f_lo < f_hi; max_smear_s > 0.
 *   keep       HOST, n int32: the indices of the chosen trials, ascending.
 *   nkeep      HOST, one int32: how many were chosen. */
ffa_status ffa_select_dm_trials(const double* dm, int32_t n, double f_lo_mhz, double f_hi_mhz,
                                double max_smear_s, int32_t* keep, int32_t* nkeep);

/* Clusters of peaks in frequency: ordered by frequency, peaks belong to one
 * cluster while consecutive ones are at most tol_hz apart (DM and width play
 * no part). Clusters are numbered in ascending frequency; a cluster's
 * parameters are those of its brightest member (the lowest index among equal
 * S/N).
 *   freq, snr    HOST, n frequencies (Hz, finite) and S/N of the peaks.
 *   tol_hz       >= 0 (typically the periodogram's cluster gap / T).
 *   cluster_of   HOST, n int32: the cluster of each peak.
 *   brightest    HOST, n int32: the brightest peak of cluster c at [c].
 *   members      HOST, n int32: the member count of cluster c at [c].
 *   nclusters    HOST, one int32. */
ffa_status ffa_cluster_frequencies(const double* freq, const float* snr, int32_t n, double tol_hz,
                                   int32_t* cluster_of, int32_t* brightest, int32_t* members,
                                   int32_t* nclusters);

/* Harmonic flags: entry j is a harmonic of entry i when i is brighter (higher
 * S/N, or equal S/N and a lower index) and, for coprime n, m in
 * [1, max_order] other than n = m = 1, |f_j - (n / m) f_i| <= tol_hz (1 + n/m).
 * The parent is the brightest such i, its ratio the one of smallest n + m,
 * then smallest n. Entries need not be sorted.
 *   freq, snr    HOST, n frequencies (Hz, > 0, finite) and S/N (e.g. of the
 *                clusters' brightest peaks).
 *   tol_hz >= 0; 1 <= max_order <= 64.
 *   parent       HOST, n int32: i, or -1 when j is no harmonic.
 *   harm_num, harm_den  HOST, n int32: n and m (0 when no parent). */
ffa_status ffa_flag_harmonics(const double* freq, const float* snr, int32_t n, double tol_hz,
                              int32_t max_order, int32_t* parent, int32_t* harm_num,
                              int32_t* harm_den);

/* Per-kernel device time of the calls made while timing is on. Each launch
 * is bracketed by HIP events on the stream it runs on (not inside captured
 * graphs). */
typedef struct {
  double stats_ms;             /* FP64 statistics kernels (Sec. 5.2) */
  double downsample_ms;        /* downsampling kernel (Sec. 5.3) */
  double fold_ms;              /* folding-transform + S/N kernels (Sec. 2.2, 5.4) */
  int64_t stats_launches;
  int64_t downsample_launches;
  int64_t fold_launches;
  int64_t profiles;            /* periodogram rows produced */
  int64_t folded_cells;        /* sum of m * p over the transforms folded */
  int64_t input_samples;       /* raw samples read */
  int64_t downsampled_samples; /* samples written by the downsampler */
  double peaks_ms;             /* peak-detection kernels (Sec. 5.5) */
  int64_t peaks_launches;      /* timed peak-detection steps: control points, fit, selection */
  double median_ms;            /* running-median de-reddening kernels (Sec. 5.2) */
  int64_t median_launches;
} ffa_kernel_times;

/* Turns per-kernel timing on (1) or off (0) for the calls that follow. */
ffa_status ffa_set_timing(ffa_ctx* ctx, int32_t enable);

/* Waits for the timed work, returns the totals since the last reset and
 * resets them when `reset` is 1. */
ffa_status ffa_read_timing(ffa_ctx* ctx, ffa_kernel_times* out, int32_t reset);

#ifdef __cplusplus
}
#endif

#endif /* FFA_MI355X_H */
