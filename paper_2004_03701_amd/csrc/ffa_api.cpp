// C ABI of the FFA search: argument checks, plan and table caches, device
// workspace, launches and graph capture.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <map>
#include <memory>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/ffa.h"
#include "ffa_internal.hpp"
#include "ffa_kernels.hpp"
#include "ffa_peaks.hpp"
#include "ffa_plan.hpp"

namespace ffa {
hipError_t launch_norm_from_stats(const double* stats, float* norm, hipStream_t stream);
}

using namespace ffa;

namespace {

// Grow-only device buffer. Growing frees the old allocation, so a buffer the
// context owns is grown through grow(), which drops the captured graphs.
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  ~DevBuf() {
    if (ptr) (void)hipFree(ptr);
  }
  // Grows to at least n bytes (contents are not kept); `zero` clears a new
  // allocation (never called inside a graph capture: every buffer is
  // reserved before one starts).
  hipError_t reserve(size_t n, bool zero = false) {
    if (n <= bytes) return hipSuccess;
    if (ptr) {
      hipError_t e = hipDeviceSynchronize();
      if (e != hipSuccess) return e;
      (void)hipFree(ptr);
      ptr = nullptr;
      bytes = 0;
    }
    size_t want = std::max<size_t>(n, 256);
    hipError_t e = hipMalloc(&ptr, want);
    if (e != hipSuccess) {
      ptr = nullptr;
      return e;
    }
    bytes = want;
    return zero ? hipMemset(ptr, 0, want) : hipSuccess;
  }
  template <typename T>
  T* as() const {
    return static_cast<T*>(ptr);
  }
};


// Smallest scratch budget (floats per buffer) a call lowers the context's to
// when the device cannot allocate the scratch of larger groups.
constexpr size_t kMinScratchBudgetCells = size_t(1) << 26;

// Key of a plan: every parameter that changes it.
std::string plan_key(const ffa_search_params& a, int64_t nsamp) {
  std::ostringstream k;
  k.precision(17);
  k << a.tsamp << ',' << a.period_min << ',' << a.period_max << ',' << a.bins_min << ','
    << a.bins_max << ',' << nsamp << ',' << a.num_widths << ':';
  for (int q = 0; q < a.num_widths; ++q) k << a.widths[q] << ',';
  return k.str();
}

// Device tables of one batch job: series, octaves, transforms, scales and
// tiles, plus the launch list.
struct Launch {
  size_t tile_off;
  int32_t ntiles;
};
struct Group {
  std::vector<Launch> passes;  // one launch per pass, or
  Launch persist{0, 0};        // all passes in one persistent launch
  int32_t ncounters = 0;
  size_t need_off = 0;
};
struct Job {
  int32_t nseries = 0;
  int32_t dtype = 0;
  int32_t num_widths = 0;
  int32_t wmax = 0;
  int32_t max_p = 0;
  int32_t min_p = 0;
  int32_t widths[kMaxWidths] = {0};
  bool any_normalise = false;
  int32_t ds_lds_floats = 0;
  int64_t ds_blocks = 0;
  int64_t ds_total = 0;     // elements of the downsampled buffer
  int64_t ds_samples = 0;   // downsampled samples (the buffer less its padding)
  int64_t scr_cells = 0;    // floats per scratch buffer
  int64_t rows = 0;         // periodogram rows
  int64_t cells = 0;        // sum of m * p
  int64_t input_samples = 0;
  std::vector<Group> groups;
  bool persistent = false;
  Tiling tiling;            // tiling the tables were built for
  int32_t max_counters = 0;
  DevBuf series, oct, xf, scales, tiles, need, src_rows;
  DevBuf blk;  // series of each downsampling block (batches of more than one series)
  int32_t stats_blocks = 0;
  // Series de-reddened first (Sec. 5.2): the running median of series `index`
  // goes to element `off` of the de-reddened buffer, which the series table
  // then points at.
  struct Median {
    int32_t index;
    const void* src;
    int64_t nsamp;
    int32_t window;
    int64_t off;
  };
  std::vector<Median> medians;
  int64_t dered_elems = 0;
  DevBuf dered;
};

// Host copies of a job's device tables, before they are placed on the device.
struct HostTables {
  std::vector<SeriesDev> sd;
  std::vector<OctaveDev> od;
  std::vector<XformDesc> xf;
  std::vector<float> scales;
  std::vector<TileDesc> tiles;
  std::vector<int32_t> src_rows, need;
  std::vector<int32_t> blk;
};

// Device addresses of a job's tables (in the job's own buffers, or in a
// caller-provided workspace).
struct JobTables {
  const SeriesDev* series = nullptr;
  const OctaveDev* oct = nullptr;
  const XformDesc* xf = nullptr;
  const float* scales = nullptr;
  const TileDesc* tiles = nullptr;
  const int32_t* src_rows = nullptr;
  const int32_t* need = nullptr;
  const int32_t* blk = nullptr;  // null: one series
  void* dered = nullptr;  // de-reddened series (storage type)
};

// Device workspace a job's launches use besides its tables.
struct Workspace {
  void* ds = nullptr;          // downsampled series (FP32)
  float* scr0 = nullptr;       // scratch rows between passes, ping-pong
  float* scr1 = nullptr;
  double* stats = nullptr;     // 2 doubles per series
  float* norm = nullptr;       // 2 floats per series
  double* partials = nullptr;  // statistics partial sums
  int32_t* flag = nullptr;     // status word
  int32_t* counters = nullptr; // persistent launches: completion counters
  int32_t* ticket = nullptr;   // and the tile ticket
};

}  // namespace

struct NaJob {
  std::unique_ptr<Job> job;          // metadata; its device buffers stay empty
  std::vector<unsigned char> packed; // the status word's 256 bytes (not copied), then the
                                     // tables, each at a 256-byte boundary; offsets are
                                     // from the start of the workspace
  size_t off_series = 0, off_oct = 0, off_xf = 0, off_scales = 0, off_tiles = 0,
         off_src_rows = 0;
  // workspace layout past the tables
  size_t off_stats = 0, off_norm = 0, off_flag = 0, off_partials = 0, off_dered = 0, off_ds = 0,
         off_scr0 = 0, off_scr1 = 0;
};

namespace {

struct GraphEntry {
  hipGraphExec_t exec = nullptr;
  std::shared_ptr<Job> job;  // the tables the graph's launches read
  ~GraphEntry() {
    if (exec) (void)hipGraphExecDestroy(exec);
  }
};

}  // namespace

// Event pairs bracketing timed launches.
// Frequency tables of one plan for peak detection (Sec. 5.5): every row's
// trial frequency and its log, and the rows of every frequency segment in
// row order (rows ascend in period, so a segment is a run of rows).
struct PeakPlan {
  std::vector<double> nu, lognu;
  std::vector<int32_t> seg_begin, seg_end;
  std::vector<double> seg_x;  // log of the segment's centre frequency
  int32_t max_seg = 0;        // rows of the largest segment
};

// A job of ffa_search_noalloc: its tables packed into one host block that a
// call copies to the start of the static workspace, and where the rest of
// the workspace goes.
struct NaJob;

struct TimedLaunch {
  int kind;  // 0 stats, 1 downsample, 2 fold, 3 peak detection, 4 running median
  hipEvent_t start, stop;
};

struct ffa_ctx {
  int device = 0;
  bool timing = false;
  std::vector<TimedLaunch> pending;
  std::vector<hipEvent_t> event_pool;
  ffa_kernel_times times{};
  std::string last_error;
  Tiling tiling;
  std::map<std::string, std::shared_ptr<SeriesPlan>> plans;
  std::map<std::string, std::shared_ptr<Job>> jobs;
  std::map<std::string, std::shared_ptr<GraphEntry>> graphs;
  DevBuf ds_buf, scr0, scr1, stats, norm, partials, flag, tune_out;
  DevBuf full_ht, full_rot, full_off;  // merge schedules of full subtrees
  DevBuf full_pops, full_pops_off;      // their pair schedules
  DevBuf counters, ticket;              // persistent scheduler state
  std::map<std::string, std::shared_ptr<PeakPlan>> peak_plans;
  DevBuf pk_series, pk_nu, pk_lognu, pk_segb, pk_sege, pk_segx, pk_mid, pk_big;  // peak-detection tables
  DevBuf pk_ctrl, pk_fits, pk_flags, pk_peaks, pk_count;          // and workspace
  std::string pk_key;    // batch the peak-detection tables were uploaded for
  int32_t pk_max_nseg = 0, pk_max_seg = 0, pk_nmid = 0, pk_nbig = 0;
  int num_cus = 256;
  void* na_ws = nullptr;         // static workspace of ffa_search_noalloc on this device
  bool na_used = false;          // its status word has been written
  std::map<std::string, std::shared_ptr<NaJob>> na_jobs;
  size_t scratch_budget_cells = size_t(1) << 32;  // floats per scratch buffer (16 GiB); a
                                                  // call that cannot allocate it lowers it
};

namespace {

ffa_status fail(ffa_ctx* ctx, ffa_status st, const std::string& msg) {
  if (ctx) ctx->last_error = msg;
  return st;
}

ffa_status hip_fail(ffa_ctx* ctx, hipError_t e, const char* what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return fail(ctx, e == hipErrorOutOfMemory ? FFA_ERR_NOMEM : FFA_ERR_DEVICE, m);
}

#define HIP_TRY(ctx, call, what)                    \
  do {                                              \
    hipError_t _e = (call);                         \
    if (_e != hipSuccess) return hip_fail(ctx, _e, what); \
  } while (0)

// Grows a context-owned device buffer. Captured graphs hold the addresses of
// the context's buffers, so every graph is dropped when one of them moves.
hipError_t grow(ffa_ctx* ctx, DevBuf& b, size_t n, bool zero = false) {
  void* before = b.ptr;
  hipError_t e = b.reserve(n, zero);
  if (b.ptr != before) ctx->graphs.clear();
  return e;
}

ffa_status get_plan(ffa_ctx* ctx, const ffa_search_params& a, int64_t nsamp,
                    std::shared_ptr<SeriesPlan>* out) {
  std::string err;
  ffa_status st = validate_params(a, &err);
  if (st != FFA_OK) return fail(ctx, st, err);
  const std::string key = plan_key(a, nsamp);
  if (ctx) {
    auto it = ctx->plans.find(key);
    if (it != ctx->plans.end()) {
      *out = it->second;
      return FFA_OK;
    }
  }
  auto plan = std::make_shared<SeriesPlan>();
  st = build_series_plan(a, nsamp, plan.get(), &err);
  if (st != FFA_OK) return fail(ctx, st, err);
  if (ctx) ctx->plans[key] = plan;
  *out = plan;
  return FFA_OK;
}

template <typename T>
hipError_t upload(DevBuf& b, const std::vector<T>& v) {
  hipError_t e = b.reserve(std::max<size_t>(v.size() * sizeof(T), 16));
  if (e != hipSuccess) return e;
  if (v.empty()) return hipSuccess;
  return hipMemcpy(b.ptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
}

// Builds the tables of a batch of series on the host: transforms grouped so
// that a group's intermediate rows fit `budget_cells` floats per scratch
// buffer (a transform larger than that forms a group of its own). Series
// pointers are stored in the tables, so a job is keyed by them too.
ffa_status build_job(ffa_ctx* ctx, int32_t nseries, const void* const* series,
                     const int64_t* nsamp, const ffa_search_params* params,
                     const int64_t* row_offset, const std::vector<std::shared_ptr<SeriesPlan>>& plans,
                     size_t budget_cells, const Tiling& tiling, Job* job, HostTables* ht) {
  job->nseries = nseries;
  job->tiling = tiling;
  job->dtype = params[0].dtype;
  job->num_widths = params[0].num_widths;
  for (int q = 0; q < job->num_widths; ++q) job->widths[q] = params[0].widths[q];
  job->wmax = job->widths[job->num_widths - 1];
  std::vector<SeriesDev>& sd = ht->sd;
  std::vector<OctaveDev>& od = ht->od;
  std::vector<XformDesc>& xf = ht->xf;
  std::vector<float>& scales = ht->scales;
  sd.assign(nseries, SeriesDev{});
  int64_t ds_off = 0, chunk = 0;
  job->ds_lds_floats = 0;
  // transforms grouped so that each group's scratch fits the budget
  struct GroupSpan {
    size_t xf0, xf1;
    int64_t cells;
  };
  std::vector<GroupSpan> spans;
  int64_t gcells = 0;
  size_t gx0 = 0;
  for (int i = 0; i < nseries; ++i) {
    const SeriesPlan& pl = *plans[i];
    const ffa_search_params& a = params[i];
    if (pl.oct.size() > 128)
      return fail(ctx, FFA_ERR_INVALID_ARG, "more than 128 pseudo-octaves: period range too wide");
    sd[i].ptr = series[i];
    sd[i].nsamp = nsamp[i];
    if (a.median_window > 0) {
      job->medians.push_back(Job::Median{i, series[i], nsamp[i], a.median_window, job->dered_elems});
      job->dered_elems += nsamp[i];
    }
    sd[i].chunk0 = chunk;
    sd[i].oct0 = (int32_t)od.size();
    sd[i].noct = (int32_t)pl.oct.size();
    sd[i].normalise = a.normalise;
    // block length from the series' own plan, so that its downsampled samples
    // do not depend on the other series of the batch
    sd[i].halo = (int32_t)(pl.ds_fx_max >> 32) + 2;
    sd[i].block = downsample_block_samples(sd[i].halo);
    sd[i].pad = 0;
    if (sd[i].block <= 0)
      return fail(ctx, FFA_ERR_INVALID_ARG,
                  "downsampling factor too large for a downsampling block (period_max / bins_min)");
    job->ds_lds_floats = std::max<int32_t>(job->ds_lds_floats, downsample_lds_floats(sd[i].block, sd[i].halo));
    if (a.normalise) job->any_normalise = true;
    const int64_t nblk = (nsamp[i] + sd[i].block - 1) / sd[i].block;
    chunk += nblk;
    if (nseries > 1) ht->blk.insert(ht->blk.end(), (size_t)nblk, i);
    for (const Octave& o : pl.oct) od.push_back(OctaveDev{o.ds_fx, o.nsamp, ds_off + o.ds_off, 1.0 / (double)o.ds_fx});
    // a series that fits a group stays in one; a larger one is split
    if ((size_t)(gcells + pl.cells) > budget_cells && gcells > 0) {
      spans.push_back(GroupSpan{gx0, xf.size(), gcells});
      gx0 = xf.size();
      gcells = 0;
    }
    for (const Transform& t : pl.tr) {
      if ((size_t)(gcells + (int64_t)t.m * t.p) > budget_cells && gcells > 0) {
        spans.push_back(GroupSpan{gx0, xf.size(), gcells});
        gx0 = xf.size();
        gcells = 0;
      }
      XformDesc x;
      x.in_off = ds_off + pl.oct[t.octave].ds_off;
      x.scr_off = gcells;
      x.out_row0 = row_offset[i] + t.row0;
      x.m = t.m;
      x.p = t.p;
      x.keep = t.keep;
      x.scale_off = (int32_t)scales.size();
      const double var = pl.oct[t.octave].var;
      for (int q = 0; q < a.num_widths; ++q)
        scales.push_back((float)(1.0 / sqrt((double)t.m * (double)a.widths[q] * var)));
      gcells += (int64_t)t.m * t.p;
      job->max_p = std::max(job->max_p, t.p);
      job->min_p = job->min_p > 0 ? std::min(job->min_p, t.p) : t.p;
      xf.push_back(x);
    }
    ds_off += pl.ds_total;
    job->ds_samples += pl.ds_samples;
    job->rows += pl.rows;
    job->cells += pl.cells;
    job->input_samples += nsamp[i];
  }
  spans.push_back(GroupSpan{gx0, xf.size(), gcells});
  job->ds_total = ds_off;
  job->ds_blocks = chunk;
  std::vector<TileDesc>& tiles = ht->tiles;
  std::vector<int32_t>& need = ht->need;
  job->scr_cells = 0;
  job->persistent = tiling.persistent != 0;
  if (job->persistent) job->tiling.range_waves = 0;  // one launch: one workgroup size
  for (const GroupSpan& g : spans) {
    Group grp;
    if (!job->persistent) {
      std::vector<std::vector<TileDesc>> passes;
      for (size_t k = g.xf0; k < g.xf1; ++k) {
        const XformDesc& x = xf[k];
        if (!plan_transform_tiles((int32_t)k, x.m, x.p, x.keep, rows_capacity(x.p, job->tiling),
                                  range_rows_capacity(x.p, job->tiling),
                                  job->tiling.levels_per_pass, false, &passes))
          return fail(ctx, FFA_ERR_INVALID_ARG, "a transform's tiles do not fit the tile rows");
      }
      for (auto& ps : passes) {
        grp.passes.push_back(Launch{tiles.size(), (int32_t)ps.size()});
        tiles.insert(tiles.end(), ps.begin(), ps.end());
      }
    } else {
      // Ticket order: pass k of the transforms of chunk c runs in slot c + k,
      // so a transform's later passes follow its first pass closely (its
      // intermediate rows are still in the caches) and never wait long.
      constexpr int kChunkXf = 32;
      struct Keyed {
        int64_t slot, pass, xf, idx;
        TileDesc t;
      };
      std::vector<Keyed> all;
      grp.need_off = need.size();
      for (size_t k = g.xf0; k < g.xf1; ++k) {
        const XformDesc& x = xf[k];
        std::vector<std::vector<TileDesc>> passes;
        if (!plan_transform_tiles((int32_t)k, x.m, x.p, x.keep, rows_capacity(x.p, job->tiling),
                                  range_rows_capacity(x.p, job->tiling),
                                  job->tiling.levels_per_pass, false, &passes))
          return fail(ctx, FFA_ERR_INVALID_ARG, "a transform's tiles do not fit the tile rows");
        const int64_t local = (int64_t)(k - g.xf0);
        const int32_t cbase = (int32_t)(local * kMaxPasses);
        for (int pk = 0; pk < kMaxPasses; ++pk)
          need.push_back(pk < (int)passes.size() ? (int32_t)passes[pk].size() : 0);
        if ((int)passes.size() > kMaxPasses)
          return fail(ctx, FFA_ERR_INVALID_ARG, "transform needs too many passes");
        for (int pk = 0; pk < (int)passes.size(); ++pk) {
          for (size_t ti = 0; ti < passes[pk].size(); ++ti) {
            TileDesc t = passes[pk][ti];
            t.dep = pk > 0 ? cbase + pk - 1 : -1;
            t.done = pk + 1 < (int)passes.size() ? cbase + pk : -1;
            all.push_back(Keyed{local / kChunkXf + pk, pk, local, (int64_t)ti, t});
          }
        }
      }
      std::stable_sort(all.begin(), all.end(), [](const Keyed& a, const Keyed& b) {
        if (a.slot != b.slot) return a.slot < b.slot;
        if (a.pass != b.pass) return a.pass < b.pass;
        if (a.xf != b.xf) return a.xf < b.xf;
        return a.idx < b.idx;
      });
      grp.persist = Launch{tiles.size(), (int32_t)all.size()};
      for (const Keyed& kt : all) tiles.push_back(kt.t);
      grp.ncounters = (int32_t)((g.xf1 - g.xf0) * kMaxPasses);
      job->max_counters = std::max(job->max_counters, grp.ncounters);
    }
    job->groups.push_back(grp);
    job->scr_cells = std::max(job->scr_cells, g.cells);
  }
  // stats: enough blocks per series to fill the chip
  int64_t maxn = 0;
  for (int i = 0; i < nseries; ++i) maxn = std::max(maxn, nsamp[i]);
  job->stats_blocks = (int32_t)std::min<int64_t>(
      std::max<int64_t>(1, (2048 + nseries - 1) / nseries), std::max<int64_t>(1, maxn / 4096));
  attach_source_rows(&tiles, xf.data(), &ht->src_rows);
  return FFA_OK;
}

size_t elem_bytes(int32_t dtype) { return dtype == FFA_F32 ? 4 : 2; }

// Points the series table of de-reddened series at their copies (base: the
// de-reddened buffer).
void point_at_dered(const Job& job, void* base, HostTables* ht) {
  for (const Job::Median& m : job.medians)
    ht->sd[m.index].ptr = static_cast<unsigned char*>(base) + m.off * elem_bytes(job.dtype);
}

// Places a job's tables in its own device buffers.
ffa_status upload_job(ffa_ctx* ctx, Job* job, HostTables& ht) {
  if (job->dered_elems > 0) {
    HIP_TRY(ctx, job->dered.reserve((size_t)job->dered_elems * elem_bytes(job->dtype) + 16),
            "allocate de-reddened series");
    point_at_dered(*job, job->dered.ptr, &ht);
  }
  HIP_TRY(ctx, upload(job->series, ht.sd), "upload series table");
  HIP_TRY(ctx, upload(job->oct, ht.od), "upload octave table");
  HIP_TRY(ctx, upload(job->xf, ht.xf), "upload transform table");
  HIP_TRY(ctx, upload(job->scales, ht.scales), "upload scale table");
  HIP_TRY(ctx, upload(job->tiles, ht.tiles), "upload tile table");
  HIP_TRY(ctx, upload(job->src_rows, ht.src_rows), "upload source-row table");
  HIP_TRY(ctx, upload(job->need, ht.need), "upload dependency table");
  if (!ht.blk.empty()) HIP_TRY(ctx, upload(job->blk, ht.blk), "upload block table");
  return FFA_OK;
}

JobTables job_tables(const Job& job) {
  JobTables t;
  t.series = job.series.as<SeriesDev>();
  t.oct = job.oct.as<OctaveDev>();
  t.xf = job.xf.as<XformDesc>();
  t.scales = job.scales.as<float>();
  t.tiles = job.tiles.as<TileDesc>();
  t.src_rows = job.src_rows.as<int32_t>();
  t.need = job.need.as<int32_t>();
  t.blk = job.nseries > 1 ? job.blk.as<int32_t>() : nullptr;
  t.dered = job.dered.ptr;
  return t;
}

Workspace ctx_workspace(ffa_ctx* ctx) {
  Workspace w;
  w.ds = ctx->ds_buf.ptr;
  w.scr0 = ctx->scr0.as<float>();
  w.scr1 = ctx->scr1.as<float>();
  w.stats = ctx->stats.as<double>();
  w.norm = ctx->norm.as<float>();
  w.partials = ctx->partials.as<double>();
  w.flag = ctx->flag.as<int32_t>();
  w.counters = ctx->counters.as<int32_t>();
  w.ticket = ctx->ticket.as<int32_t>();
  return w;
}

// Grows the context workspace for a job. Captured graphs hold the old
// addresses, so they are dropped whenever a buffer moves.
ffa_status reserve_job(ffa_ctx* ctx, const Job& job) {
  const size_t db = job.dtype == FFA_F32 ? 4 : 2;  // downsampled series: the input's type
  DevBuf* bufs[] = {&ctx->ds_buf, &ctx->scr0, &ctx->scr1, &ctx->stats, &ctx->norm,
                    &ctx->partials, &ctx->flag, &ctx->counters, &ctx->ticket};
  const size_t want[] = {(size_t)job.ds_total * db + 16,
                         (size_t)job.scr_cells * 4 + 16,
                         (size_t)job.scr_cells * 4 + 16,
                         (size_t)job.nseries * 2 * sizeof(double),
                         (size_t)job.nseries * kNormFloats * sizeof(float),
                         (size_t)job.nseries * job.stats_blocks * 2 * sizeof(double),
                         16,
                         (size_t)std::max(job.max_counters, 1) * sizeof(int32_t),
                         16};
  for (int b = 0; b < 9; ++b) {
    // the status flag is read before anything has written it
    HIP_TRY(ctx, grow(ctx, *bufs[b], want[b], bufs[b] == &ctx->flag), "allocate workspace");
  }
  return FFA_OK;
}

void set_schedules(ffa_ctx* ctx, PassArgs* pa) {
  pa->full_ht = ctx->full_ht.as<uint32_t>();
  pa->full_rot = ctx->full_rot.as<uint16_t>();
  pa->full_off = ctx->full_off.as<int32_t>();
  pa->full_pops = ctx->full_pops.as<uint32_t>();
  pa->full_pops_off = ctx->full_pops_off.as<int32_t>();
}

hipError_t take_event(ffa_ctx* ctx, hipEvent_t* ev) {
  if (!ctx->event_pool.empty()) {
    *ev = ctx->event_pool.back();
    ctx->event_pool.pop_back();
    return hipSuccess;
  }
  return hipEventCreate(ev);
}

// Brackets a launch with events when timing is on.
struct TimedScope {
  ffa_ctx* ctx;
  int kind;
  hipStream_t stream;
  bool on;
  hipEvent_t a = nullptr, b = nullptr;
  TimedScope(ffa_ctx* c, int k, hipStream_t s, bool enabled) : ctx(c), kind(k), stream(s), on(enabled) {
    if (on && take_event(ctx, &a) == hipSuccess && take_event(ctx, &b) == hipSuccess)
      on = hipEventRecord(a, stream) == hipSuccess;
    else
      on = false;
  }
  ~TimedScope() {
    if (on && hipEventRecord(b, stream) == hipSuccess) ctx->pending.push_back(TimedLaunch{kind, a, b});
  }
};

// Queues the device work of a job whose tables and workspace are in place.
ffa_status enqueue_work(ffa_ctx* ctx, const Job& job, const JobTables& tb, const Workspace& ws,
                        float* snr, hipStream_t stream, bool timed) {
  if (timed) {
    ctx->times.profiles += job.rows;
    ctx->times.folded_cells += job.cells;
    ctx->times.input_samples += job.input_samples;
    ctx->times.downsampled_samples += job.ds_samples;
  }
  const SeriesDev* sd = tb.series;
  for (const Job::Median& m : job.medians) {
    TimedScope ts(ctx, 4, stream, timed);
    HIP_TRY(ctx, launch_running_median(m.src, m.nsamp, job.dtype, m.window,
                                       static_cast<unsigned char*>(tb.dered) +
                                           m.off * elem_bytes(job.dtype),
                                       job.dtype, ws.flag, stream),
            "running median kernel");
  }
  if (job.any_normalise) {
    TimedScope ts(ctx, 0, stream, timed);
    HIP_TRY(ctx, launch_stats(sd, job.nseries, job.dtype, job.stats_blocks, ws.partials, ws.stats,
                              ws.norm, ws.flag, stream),
            "stats kernels");
  }
  {
  TimedScope ts(ctx, 1, stream, timed);
  // the downsampled series are stored in the input's type (BF16 and FP16
  // storage halve the fold's input reads); the fold converts them on load
  HIP_TRY(ctx, launch_downsample(sd, tb.blk, tb.oct, ws.norm, job.dtype, ws.ds, job.dtype,
                                 job.ds_blocks, job.ds_lds_floats, stream),
          "downsample kernel");
  }
  PassArgs pa{};
  pa.lds_rows_cap = job.tiling.lds_rows;
  pa.waves = job.tiling.waves;
  pa.xf = tb.xf;
  pa.in = ws.ds;
  pa.in_dtype = job.dtype;
  pa.num_widths = job.num_widths;
  pa.scr0 = ws.scr0;
  pa.scr1 = ws.scr1;
  pa.out_rows = nullptr;
  pa.snr = snr;
  pa.scales = tb.scales;
  for (int q = 0; q < kMaxWidths; ++q) pa.widths[q] = job.widths[q];
  pa.wmax = job.wmax;
  pa.max_p = job.max_p;
  pa.width_set = width_set_of(job.widths, job.num_widths);
  const bool pairs = pairs_only_launch(job.min_p, job.max_p, pa.width_set);
  set_schedules(ctx, &pa);
  pa.ticket = ws.ticket;
  pa.counters = ws.counters;
  pa.error_flag = ws.flag;
  pa.spin_limit = 1 << 22;
  pa.src_rows = tb.src_rows;
  const TileDesc* tiles = tb.tiles;
  for (const Group& g : job.groups) {
    if (job.persistent) {
      pa.tiles = tiles + g.persist.tile_off;
      pa.ntiles = g.persist.ntiles;
      pa.need = tb.need + g.need_off;
      TimedScope ts(ctx, 2, stream, timed);
      HIP_TRY(ctx, launch_persist(pa, g.ncounters, ctx->num_cus * (kWavesLarge / job.tiling.waves),
                                  stream),
              "persistent fold kernel");
      continue;
    }
    for (size_t k = 0; k < g.passes.size(); ++k) {
      const Launch& l = g.passes[k];
      pa.tiles = tiles + l.tile_off;
      pa.ntiles = l.ntiles;
      // a first pass holds full tiles only, a later pass range tiles only
      pa.pairs_only = pairs ? (k == 0 ? 2 : 3) : 0;
      pa.waves = k == 0 ? job.tiling.waves : job.tiling.waves_of_range();
      TimedScope ts(ctx, 2, stream, timed);
      HIP_TRY(ctx, launch_pass(pa, stream), "fold pass kernel");
    }
  }
  return FFA_OK;
}

// Queues the device work of a job in the context's workspace.
ffa_status enqueue_job(ffa_ctx* ctx, Job& job, float* snr, hipStream_t stream, bool timed) {
  ffa_status rst = reserve_job(ctx, job);
  if (rst != FFA_OK) return rst;
  return enqueue_work(ctx, job, job_tables(job), ctx_workspace(ctx), snr, stream, timed);
}

std::string job_key(int32_t nseries, const void* const* series, const int64_t* nsamp,
                    const ffa_search_params* params, const int64_t* row_offset,
                    const Tiling& tiling) {
  std::ostringstream k;
  k << nseries << '|' << tiling.lds_rows << ',' << tiling.levels_per_pass << ','
    << tiling.persistent << ',' << tiling.waves << ',' << tiling.range_waves << '|';
  for (int i = 0; i < nseries; ++i)
    k << series[i] << ',' << row_offset[i] << ',' << params[i].normalise << ','
      << params[i].dtype << ',' << params[i].median_window << ','
      << plan_key(params[i], nsamp[i]) << ';';
  return k.str();
}

ffa_status check_batch_args(ffa_ctx* ctx, int32_t nseries, const void* const* series,
                            const int64_t* nsamp, const ffa_search_params* params) {
  if (!series || !nsamp || !params || nseries < 1)
    return fail(ctx, FFA_ERR_INVALID_ARG, "null batch array or nseries < 1");
  for (int i = 0; i < nseries; ++i) {
    if (!series[i]) return fail(ctx, FFA_ERR_INVALID_ARG, "null series pointer");
    if (params[i].num_widths != params[0].num_widths || params[i].dtype != params[0].dtype)
      return fail(ctx, FFA_ERR_INVALID_ARG, "all series of a batch need the same dtype and number of widths");
    if (params[i].widths && params[0].widths)
      for (int q = 0; q < params[0].num_widths && q < params[i].num_widths; ++q)
        if (params[i].widths[q] != params[0].widths[q])
          return fail(ctx, FFA_ERR_INVALID_ARG, "all series of a batch need the same widths");
  }
  return FFA_OK;
}

// Shared body of ffa_search and ffa_search_batch.
ffa_status run_batch(ffa_ctx* ctx, int32_t nseries, const void* const* series,
                     const int64_t* nsamp, const ffa_search_params* params,
                     const int64_t* row_offset, float* snr, int64_t capacity_rows,
                     int32_t use_graph, hipStream_t stream) {
  ffa_status st = check_batch_args(ctx, nseries, series, nsamp, params);
  if (st != FFA_OK) return st;
  if (!row_offset || !snr) return fail(ctx, FFA_ERR_INVALID_ARG, "null row_offset or snr");
  std::vector<std::shared_ptr<SeriesPlan>> plans(nseries);
  for (int i = 0; i < nseries; ++i) {
    st = get_plan(ctx, params[i], nsamp[i], &plans[i]);
    if (st != FFA_OK) return st;
    if (row_offset[i] < 0 || row_offset[i] + plans[i]->rows > capacity_rows)
      return fail(ctx, FFA_ERR_BUFFER_TOO_SMALL, "snr buffer too small for the periodogram rows");
  }
  std::string key;
  std::shared_ptr<Job> job;
  for (;;) {
    key = job_key(nseries, series, nsamp, params, row_offset, ctx->tiling);
    auto it = ctx->jobs.find(key);
    if (it != ctx->jobs.end()) {
      job = it->second;
    } else {
      if (ctx->jobs.size() > 64) ctx->jobs.clear();
      job = std::make_shared<Job>();
      HostTables ht;
      st = build_job(ctx, nseries, series, nsamp, params, row_offset, plans,
                     ctx->scratch_budget_cells, ctx->tiling, job.get(), &ht);
      if (st != FFA_OK) return st;
      st = upload_job(ctx, job.get(), ht);
      if (st != FFA_OK) return st;
      ctx->jobs[key] = job;
    }
    st = reserve_job(ctx, *job);
    if (st != FFA_ERR_NOMEM || ctx->scratch_budget_cells <= kMinScratchBudgetCells) break;
    // the device cannot hold the scratch of groups this large: smaller
    // groups (more launches) with buffers a quarter the size
    ctx->scratch_budget_cells /= 4;
    ctx->jobs.clear();
    ctx->graphs.clear();
    (void)hipGetLastError();  // the failed allocation must not be reported by a later launch
    ctx->last_error.clear();
  }
  if (st != FFA_OK) return st;
  if (!use_graph) return enqueue_job(ctx, *job, snr, stream, ctx->timing);
  std::ostringstream gk;
  gk << key << "|snr=" << (const void*)snr << "|stream=" << (const void*)stream;
  st = reserve_job(ctx, *job);
  if (st != FFA_OK) return st;
  auto git = ctx->graphs.find(gk.str());
  if (git == ctx->graphs.end()) {
    // allocate everything before capture so no allocation happens inside it
    st = reserve_job(ctx, *job);
    if (st != FFA_OK) return st;
    hipStream_t cap = stream;
    bool own = false;
    if (cap == nullptr) {
      HIP_TRY(ctx, hipStreamCreateWithFlags(&cap, hipStreamNonBlocking), "create capture stream");
      own = true;
    }
    hipGraph_t graph = nullptr;
    HIP_TRY(ctx, hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal), "begin capture");
    ffa_status est = enqueue_job(ctx, *job, snr, cap, false);
    hipError_t ce = hipStreamEndCapture(cap, &graph);
    if (own) (void)hipStreamDestroy(cap);
    if (est != FFA_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return est;
    }
    if (ce != hipSuccess) return hip_fail(ctx, ce, "end capture");
    auto ge = std::make_shared<GraphEntry>();
    ge->job = job;
    hipError_t ie = hipGraphInstantiate(&ge->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) return hip_fail(ctx, ie, "instantiate graph");
    if (ctx->graphs.size() > 16) ctx->graphs.clear();
    git = ctx->graphs.emplace(gk.str(), ge).first;
  }
  HIP_TRY(ctx, hipGraphLaunch(git->second->exec, stream), "graph launch");
  return FFA_OK;
}

// Frequency segments of a plan's rows (Sec. 5.5): nu = 1 / P, segment
// floor((nu - nu_lo) / dnu) with dnu = dz_seg / T, all in FP64.
ffa_status build_peak_plan(ffa_ctx* ctx, const SeriesPlan& plan, double T, double dz_seg,
                           PeakPlan* out) {
  const int64_t R = plan.rows;
  if (R >= (int64_t(1) << 31)) return fail(ctx, FFA_ERR_INVALID_ARG, "too many periodogram rows");
  out->nu.resize(R);
  out->lognu.resize(R);
  for (const Transform& t : plan.tr) {
    const Octave& o = plan.oct[t.octave];
    for (int32_t r = 0; r < t.keep; ++r) {
      const double nu = 1.0 / trial_period(r, t.m, t.p, o.tau);
      out->nu[t.row0 + r] = nu;
      out->lognu[t.row0 + r] = std::log(nu);
    }
  }
  if (R == 0) return FFA_OK;
  const double nu_lo = *std::min_element(out->nu.begin(), out->nu.end());
  const double dnu = dz_seg / T;
  int64_t cur = -1;
  for (int64_t r = 0; r < R; ++r) {
    const int64_t id = (int64_t)std::floor((out->nu[r] - nu_lo) / dnu);
    if (r > 0 && id > cur)
      return fail(ctx, FFA_ERR_DEVICE, "trial frequencies are not descending along the rows");
    if (r == 0 || id != cur) {
      if (r > 0) out->seg_end.push_back((int32_t)r);
      out->seg_begin.push_back((int32_t)r);
      out->seg_x.push_back(std::log(nu_lo + ((double)id + 0.5) * dnu));
      cur = id;
    }
  }
  out->seg_end.push_back((int32_t)R);
  for (size_t i = 0; i < out->seg_begin.size(); ++i)
    out->max_seg = std::max(out->max_seg, out->seg_end[i] - out->seg_begin[i]);
  return FFA_OK;
}

// Power-basis coefficients in x of sum_j c_j ((x - xbar) s)^j.
void expand_poly(const PeakFitDev& f, int degree, double* out) {
  for (int j = 0; j <= degree; ++j) out[j] = 0.0;
  // binomial expansion of (s x - s xbar)^j
  for (int j = 0; j <= degree; ++j) {
    double binom = 1.0;  // C(j, l)
    for (int l = 0; l <= j; ++l) {
      out[l] += f.c[j] * binom * std::pow(f.inv_scale, j) * std::pow(-f.xbar, j - l);
      binom = binom * (j - l) / (l + 1);
    }
  }
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

template <typename T>
void pack_table(std::vector<unsigned char>* out, size_t* off, const std::vector<T>& v) {
  *off = align256(out->size());
  out->resize(*off + std::max<size_t>(v.size() * sizeof(T), 16), 0);
  if (!v.empty()) memcpy(out->data() + *off, v.data(), v.size() * sizeof(T));
}

// Plans a search of one series inside the static workspace: the tables first
// (after the status word), then statistics, the downsampled series, and two
// scratch buffers sharing what is left, the transforms grouped to fit them.
ffa_status build_na_job(ffa_ctx* ctx, const void* series, int64_t nsamp,
                        const ffa_search_params& a, const std::shared_ptr<SeriesPlan>& plan,
                        NaJob* nj) {
  std::vector<std::shared_ptr<SeriesPlan>> plans{plan};
  const int64_t zero = 0;
  Tiling tiling = ctx->tiling;
  tiling.persistent = 0;  // per-pass launches: no counters in the workspace
  int64_t largest = 0;
  for (const Transform& t : plan->tr) largest = std::max<int64_t>(largest, (int64_t)t.m * t.p);
  // tables and fixed parts do not depend on the grouping: size them with
  // every transform in one group, then group for the space that remains
  size_t budget = size_t(1) << 40;
  for (int round = 0; round < 2; ++round) {
    if (round == 1) {
      const size_t fixed = nj->off_scr0;
      std::ostringstream msg;
      msg << "ffa_search_noalloc: ";
      if (fixed + 2 * 512 >= kNoAllocBytes) {
        msg << "the series' tables and downsampled samples (" << fixed
            << " bytes) exceed the static workspace of " << kNoAllocBytes << " bytes; use ffa_search";
        return fail(ctx, FFA_ERR_INVALID_ARG, msg.str());
      }
      budget = ((kNoAllocBytes - fixed) / 2 - 512) / 4;
      if ((int64_t)budget < largest) {
        msg << "a transform's " << largest << " intermediate cells exceed the " << budget
            << " left per scratch buffer in the static workspace of " << kNoAllocBytes
            << " bytes; use ffa_search";
        return fail(ctx, FFA_ERR_INVALID_ARG, msg.str());
      }
    }
    nj->job.reset(new Job());
    HostTables ht;
    ffa_status st = build_job(ctx, 1, &series, &nsamp, &a, &zero, plans, budget, tiling,
                              nj->job.get(), &ht);
    if (st != FFA_OK) return st;
    const Job& job = *nj->job;
    nj->packed.assign(kNoAllocHeader, 0);
    // the de-reddened copies sit past the tables, whose size does not depend
    // on the pointers: lay out once with the pointers unset, then set them
    pack_table(&nj->packed, &nj->off_series, ht.sd);
    pack_table(&nj->packed, &nj->off_oct, ht.od);
    pack_table(&nj->packed, &nj->off_xf, ht.xf);
    pack_table(&nj->packed, &nj->off_scales, ht.scales);
    pack_table(&nj->packed, &nj->off_tiles, ht.tiles);
    pack_table(&nj->packed, &nj->off_src_rows, ht.src_rows);
    size_t o = align256(nj->packed.size());
    nj->off_stats = o;
    o = align256(o + 2 * sizeof(double));
    nj->off_norm = o;
    o = align256(o + kNormFloats * sizeof(float));
    nj->off_partials = o;
    o = align256(o + (size_t)job.stats_blocks * 2 * sizeof(double));
    nj->off_dered = o;
    o = align256(o + (size_t)job.dered_elems * elem_bytes(job.dtype) + 16);
    nj->off_ds = o;
    o = align256(o + (size_t)job.ds_total * elem_bytes(job.dtype) + 16);
    nj->off_scr0 = o;
    o = align256(o + (size_t)job.scr_cells * 4 + 16);
    nj->off_scr1 = o;
    o = align256(o + (size_t)job.scr_cells * 4 + 16);
    if (round == 1 && o > kNoAllocBytes)
      return fail(ctx, FFA_ERR_DEVICE, "ffa_search_noalloc: workspace layout overflow");
    if (round == 1 && !job.medians.empty()) {
      point_at_dered(job, static_cast<unsigned char*>(ctx->na_ws) + nj->off_dered, &ht);
      memcpy(nj->packed.data() + nj->off_series, ht.sd.data(), ht.sd.size() * sizeof(SeriesDev));
    }
  }
  return FFA_OK;
}

}  // namespace

extern "C" {

ffa_status ffa_create(int device, ffa_ctx** out) {
  if (!out) return FFA_ERR_INVALID_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return FFA_ERR_DEVICE;
  if (hipSetDevice(device) != hipSuccess) return FFA_ERR_DEVICE;
  ffa_ctx* c = new (std::nothrow) ffa_ctx();
  if (!c) return FFA_ERR_NOMEM;
  c->device = device;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
    c->num_cus = prop.multiProcessorCount;
  if (noalloc_setup(device, &c->na_ws) != hipSuccess) {
    delete c;
    return FFA_ERR_DEVICE;
  }
  std::vector<uint32_t> ht;
  std::vector<uint16_t> rot;
  std::vector<int32_t> off;
  build_full_schedules(&ht, &rot, &off);
  std::vector<uint32_t> pops;
  std::vector<int32_t> pops_off;
  build_full_pair_ops(&pops, &pops_off);
  if (upload(c->full_ht, ht) != hipSuccess || upload(c->full_rot, rot) != hipSuccess ||
      upload(c->full_off, off) != hipSuccess || upload(c->full_pops, pops) != hipSuccess ||
      upload(c->full_pops_off, pops_off) != hipSuccess) {
    delete c;
    return FFA_ERR_DEVICE;
  }
  *out = c;
  return FFA_OK;
}

ffa_status ffa_destroy(ffa_ctx* ctx) {
  if (!ctx) return FFA_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  for (const TimedLaunch& t : ctx->pending) {
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.stop);
  }
  for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
  delete ctx;
  return FFA_OK;
}

const char* ffa_status_string(ffa_status s) {
  switch (s) {
    case FFA_OK: return "ok";
    case FFA_ERR_INVALID_ARG: return "invalid argument";
    case FFA_ERR_RANGE: return "period range not searchable with these parameters";
    case FFA_ERR_BUFFER_TOO_SMALL: return "output buffer too small";
    case FFA_ERR_NOMEM: return "out of memory";
    case FFA_ERR_DEVICE: return "HIP device error";
    case FFA_ERR_DEGENERATE: return "degenerate series (zero or non-finite variance)";
    case FFA_ERR_NOT_IMPLEMENTED: return "not implemented";
  }
  return "unknown status";
}

const char* ffa_last_error(const ffa_ctx* ctx) { return ctx ? ctx->last_error.c_str() : ""; }

ffa_status ffa_plan_rows(const ffa_search_params* params, int64_t nsamp, int64_t* rows) {
  if (!params || !rows) return FFA_ERR_INVALID_ARG;
  std::shared_ptr<SeriesPlan> plan;
  ffa_status st = get_plan(nullptr, *params, nsamp, &plan);
  if (st != FFA_OK) return st;
  *rows = plan->rows;
  return FFA_OK;
}

ffa_status ffa_plan_export(const ffa_search_params* params, int64_t nsamp, double* period,
                           int32_t* bins, int32_t* m, int32_t* s, int32_t* octave,
                           uint64_t* ds_fx, int64_t capacity) {
  if (!params) return FFA_ERR_INVALID_ARG;
  std::shared_ptr<SeriesPlan> plan;
  ffa_status st = get_plan(nullptr, *params, nsamp, &plan);
  if (st != FFA_OK) return st;
  if (capacity < plan->rows) return FFA_ERR_BUFFER_TOO_SMALL;
  for (const Transform& t : plan->tr) {
    const Octave& o = plan->oct[t.octave];
    for (int32_t r = 0; r < t.keep; ++r) {
      const int64_t row = t.row0 + r;
      if (period) period[row] = trial_period(r, t.m, t.p, o.tau);
      if (bins) bins[row] = t.p;
      if (m) m[row] = t.m;
      if (s) s[row] = r;
      if (octave) octave[row] = t.octave;
      if (ds_fx) ds_fx[row] = o.ds_fx;
    }
  }
  return FFA_OK;
}

ffa_status ffa_search(ffa_ctx* ctx, const void* series, int64_t nsamp,
                      const ffa_search_params* params, double* period_host, int32_t* bins_host,
                      float* snr_dev, int64_t capacity_rows, void* stream) {
  if (!ctx) return FFA_ERR_INVALID_ARG;
  if (!series || !params || !snr_dev)
    return fail(ctx, FFA_ERR_INVALID_ARG, "null series, params or snr pointer");
  std::shared_ptr<SeriesPlan> plan;
  ffa_status st = get_plan(ctx, *params, nsamp, &plan);
  if (st != FFA_OK) return st;
  if (capacity_rows < plan->rows)
    return fail(ctx, FFA_ERR_BUFFER_TOO_SMALL, "snr buffer too small for the periodogram rows");
  if (period_host || bins_host) {
    for (const Transform& t : plan->tr) {
      const Octave& o = plan->oct[t.octave];
      for (int32_t r = 0; r < t.keep; ++r) {
        if (period_host) period_host[t.row0 + r] = trial_period(r, t.m, t.p, o.tau);
        if (bins_host) bins_host[t.row0 + r] = t.p;
      }
    }
  }
  const int64_t zero = 0;
  return run_batch(ctx, 1, &series, &nsamp, params, &zero, snr_dev, capacity_rows, 0,
                   static_cast<hipStream_t>(stream));
}

ffa_status ffa_search_noalloc(ffa_ctx* ctx, const void* series, int64_t nsamp,
                              const ffa_search_params* params, double* period_host,
                              int32_t* bins_host, float* snr_dev, int64_t capacity_rows,
                              void* stream) {
  if (!ctx) return FFA_ERR_INVALID_ARG;
  if (!series || !params || !snr_dev)
    return fail(ctx, FFA_ERR_INVALID_ARG, "null series, params or snr pointer");
  if (!ctx->na_ws) return fail(ctx, FFA_ERR_DEVICE, "no static workspace on this device");
  std::shared_ptr<SeriesPlan> plan;
  ffa_status st = get_plan(ctx, *params, nsamp, &plan);
  if (st != FFA_OK) return st;
  if (capacity_rows < plan->rows)
    return fail(ctx, FFA_ERR_BUFFER_TOO_SMALL, "snr buffer too small for the periodogram rows");
  const int64_t zero = 0;
  const Tiling na_tiling{ctx->tiling.lds_rows, ctx->tiling.levels_per_pass, 0, ctx->tiling.waves,
                         ctx->tiling.range_waves};
  const std::string key = job_key(1, &series, &nsamp, params, &zero, na_tiling);
  std::shared_ptr<NaJob> nj;
  auto it = ctx->na_jobs.find(key);
  if (it != ctx->na_jobs.end()) {
    nj = it->second;
  } else {
    nj = std::make_shared<NaJob>();
    st = build_na_job(ctx, series, nsamp, *params, plan, nj.get());
    if (st != FFA_OK) return st;
    if (ctx->na_jobs.size() >= 16) ctx->na_jobs.clear();
    ctx->na_jobs[key] = nj;
  }
  if (period_host || bins_host) {
    for (const Transform& t : plan->tr) {
      const Octave& o = plan->oct[t.octave];
      for (int32_t r = 0; r < t.keep; ++r) {
        if (period_host) period_host[t.row0 + r] = trial_period(r, t.m, t.p, o.tau);
        if (bins_host) bins_host[t.row0 + r] = t.p;
      }
    }
  }
  hipStream_t hs = static_cast<hipStream_t>(stream);
  unsigned char* ws = static_cast<unsigned char*>(ctx->na_ws);
  // the tables go after the status word; the copy is complete (and the host
  // block free) before any kernel of this call is queued
  HIP_TRY(ctx, hipMemcpyAsync(ws + kNoAllocHeader, nj->packed.data() + kNoAllocHeader,
                              nj->packed.size() - kNoAllocHeader, hipMemcpyHostToDevice, hs),
          "copy tables to the workspace");
  HIP_TRY(ctx, hipStreamSynchronize(hs), "synchronise");
  int32_t* flag = reinterpret_cast<int32_t*>(ws + kNoAllocFlagOffset);
  HIP_TRY(ctx, launch_clear_flag(flag, hs), "clear status word");
  ctx->na_used = true;
  JobTables tb;
  tb.series = reinterpret_cast<const SeriesDev*>(ws + nj->off_series);
  tb.oct = reinterpret_cast<const OctaveDev*>(ws + nj->off_oct);
  tb.xf = reinterpret_cast<const XformDesc*>(ws + nj->off_xf);
  tb.scales = reinterpret_cast<const float*>(ws + nj->off_scales);
  tb.tiles = reinterpret_cast<const TileDesc*>(ws + nj->off_tiles);
  tb.src_rows = reinterpret_cast<const int32_t*>(ws + nj->off_src_rows);
  tb.dered = ws + nj->off_dered;
  Workspace w;
  w.stats = reinterpret_cast<double*>(ws + nj->off_stats);
  w.norm = reinterpret_cast<float*>(ws + nj->off_norm);
  w.partials = reinterpret_cast<double*>(ws + nj->off_partials);
  w.ds = ws + nj->off_ds;
  w.scr0 = reinterpret_cast<float*>(ws + nj->off_scr0);
  w.scr1 = reinterpret_cast<float*>(ws + nj->off_scr1);
  w.flag = flag;
  return enqueue_work(ctx, *nj->job, tb, w, snr_dev, hs, ctx->timing);
}

ffa_status ffa_search_ranges(ffa_ctx* ctx, const void* series, int64_t nsamp,
                             const ffa_search_params* ranges, int32_t nranges,
                             double* period_host, int32_t* bins_host, int64_t* range_row0,
                             float* snr_dev, int64_t capacity_rows, void* stream) {
  if (!ctx) return FFA_ERR_INVALID_ARG;
  if (!series || !ranges || nranges < 1 || !snr_dev)
    return fail(ctx, FFA_ERR_INVALID_ARG, "null series, ranges or snr pointer, or nranges < 1");
  for (int32_t k = 0; k < nranges; ++k) {
    const ffa_search_params& r = ranges[k];
    if (r.tsamp != ranges[0].tsamp || r.normalise != ranges[0].normalise)
      return fail(ctx, FFA_ERR_INVALID_ARG, "sub-ranges need the same tsamp and normalise");
    if (k > 0 && !(ranges[k - 1].period_max <= r.period_min))
      return fail(ctx, FFA_ERR_INVALID_ARG,
                  "sub-ranges must be in ascending period order without overlap");
  }
  std::vector<int64_t> row0(nranges + 1, 0);
  std::vector<std::shared_ptr<SeriesPlan>> plans(nranges);
  for (int32_t k = 0; k < nranges; ++k) {
    ffa_status st = get_plan(ctx, ranges[k], nsamp, &plans[k]);
    if (st != FFA_OK) return st;
    row0[k + 1] = row0[k] + plans[k]->rows;
  }
  if (capacity_rows < row0[nranges])
    return fail(ctx, FFA_ERR_BUFFER_TOO_SMALL, "snr buffer too small for the periodogram rows");
  if (range_row0)
    for (int32_t k = 0; k <= nranges; ++k) range_row0[k] = row0[k];
  if (period_host || bins_host)
    for (int32_t k = 0; k < nranges; ++k)
      for (const Transform& t : plans[k]->tr) {
        const Octave& o = plans[k]->oct[t.octave];
        for (int32_t r = 0; r < t.keep; ++r) {
          const int64_t row = row0[k] + t.row0 + r;
          if (period_host) period_host[row] = trial_period(r, t.m, t.p, o.tau);
          if (bins_host) bins_host[row] = t.p;
        }
      }
  // one batch whose entries are the same series with each range's parameters
  std::vector<const void*> ptrs(nranges, series);
  std::vector<int64_t> ns(nranges, nsamp);
  return run_batch(ctx, nranges, ptrs.data(), ns.data(), ranges, row0.data(), snr_dev,
                   capacity_rows, 0, static_cast<hipStream_t>(stream));
}

ffa_status ffa_search_batch(ffa_ctx* ctx, int32_t nseries, const void* const* series,
                            const int64_t* nsamp, const ffa_search_params* params,
                            const int64_t* row_offset, float* snr_dev, int64_t capacity_rows,
                            int32_t use_graph, void* stream) {
  if (!ctx) return FFA_ERR_INVALID_ARG;
  return run_batch(ctx, nseries, series, nsamp, params, row_offset, snr_dev, capacity_rows,
                   use_graph, static_cast<hipStream_t>(stream));
}

ffa_status ffa_transform(ffa_ctx* ctx, const float* in, int32_t m, int32_t p, float* out,
                         void* stream) {
  if (!ctx) return FFA_ERR_INVALID_ARG;
  if (!in || !out) return fail(ctx, FFA_ERR_INVALID_ARG, "null in or out");
  if (m < 1 || p < 2 || p > kMaxBins || (int64_t)m * p > (int64_t(1) << 31))
    return fail(ctx, FFA_ERR_INVALID_ARG, "need 1 <= m, 2 <= p <= 1280, m * p < 2^31");
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::vector<XformDesc> xf(1);
  xf[0].in_off = 0;
  xf[0].scr_off = 0;
  xf[0].out_row0 = 0;
  xf[0].m = m;
  xf[0].p = p;
  xf[0].keep = m;
  xf[0].scale_off = 0;
  std::vector<std::vector<TileDesc>> passes;
  if (m == 1) {
    HIP_TRY(ctx, hipMemcpyAsync(out, in, (size_t)p * 4, hipMemcpyDeviceToDevice, st), "copy");
    return FFA_OK;
  }
  if (!plan_transform_tiles(0, m, p, m, rows_capacity(p, ctx->tiling),
                            range_rows_capacity(p, ctx->tiling), ctx->tiling.levels_per_pass, true,
                            &passes))
    return fail(ctx, FFA_ERR_INVALID_ARG, "the transform's tiles do not fit the tile rows");
  std::vector<TileDesc> tiles;
  std::vector<Launch> launches;
  for (auto& ps : passes) {
    launches.push_back(Launch{tiles.size(), (int32_t)ps.size()});
    tiles.insert(tiles.end(), ps.begin(), ps.end());
  }
  // per-call tables live as long as the context (kept in a small job)
  auto job = std::make_shared<Job>();
  std::vector<int32_t> src_rows;
  attach_source_rows(&tiles, xf.data(), &src_rows);
  HIP_TRY(ctx, upload(job->xf, xf), "upload transform table");
  HIP_TRY(ctx, upload(job->tiles, tiles), "upload tile table");
  HIP_TRY(ctx, upload(job->src_rows, src_rows), "upload source-row table");
  HIP_TRY(ctx, grow(ctx, ctx->scr0, (size_t)m * p * 4 + 16), "allocate scratch");
  HIP_TRY(ctx, grow(ctx, ctx->scr1, (size_t)m * p * 4 + 16), "allocate scratch");
  PassArgs pa{};
  pa.lds_rows_cap = ctx->tiling.lds_rows;
  pa.waves = ctx->tiling.waves;
  pa.xf = job->xf.as<XformDesc>();
  pa.in = in;
  pa.in_dtype = FFA_F32;
  pa.num_widths = 1;
  pa.widths[0] = 1;
  pa.wmax = 1;
  pa.max_p = p;
  pa.width_set = kWidthsGeneral;
  set_schedules(ctx, &pa);
  pa.scr0 = ctx->scr0.as<float>();
  pa.scr1 = ctx->scr1.as<float>();
  pa.out_rows = out;
  pa.src_rows = job->src_rows.as<int32_t>();
  // rows short enough for the pair forms run the kernels compiled for them
  // (a first pass holds full tiles only, a later pass range tiles only)
  const bool pairs = pair_forms_fit(p);
  for (size_t k = 0; k < launches.size(); ++k) {
    const Launch& l = launches[k];
    pa.tiles = job->tiles.as<TileDesc>() + l.tile_off;
    pa.ntiles = l.ntiles;
    pa.pairs_only = pairs ? (k == 0 ? 2 : 3) : 0;
    pa.waves = k == 0 ? ctx->tiling.waves : ctx->tiling.waves_of_range();
    HIP_TRY(ctx, launch_pass(pa, st), "fold pass kernel");
  }
  // keep the tables alive until the work is done
  HIP_TRY(ctx, hipStreamSynchronize(st), "synchronise");
  return FFA_OK;
}

ffa_status ffa_series_stats(ffa_ctx* ctx, const void* series, int64_t nsamp, int32_t dtype,
                            double* stats_dev, void* stream) {
  if (!ctx) return FFA_ERR_INVALID_ARG;
  if (!series || !stats_dev) return fail(ctx, FFA_ERR_INVALID_ARG, "null series or stats");
  if (nsamp < 1 || nsamp > INT32_MAX) return fail(ctx, FFA_ERR_INVALID_ARG, "nsamp out of range");
  if (dtype != FFA_F32 && dtype != FFA_BF16 && dtype != FFA_F16)
    return fail(ctx, FFA_ERR_INVALID_ARG, "unknown dtype");
  hipStream_t st = static_cast<hipStream_t>(stream);
  SeriesDev sd{series, nsamp, 0, 0, 0, 1, 0, 0, 0};
  DevBuf tmp;
  HIP_TRY(ctx, tmp.reserve(sizeof(SeriesDev)), "allocate");
  HIP_TRY(ctx, hipMemcpy(tmp.ptr, &sd, sizeof sd, hipMemcpyHostToDevice), "upload");
  const int32_t bps = (int32_t)std::max<int64_t>(1, std::min<int64_t>(2048, nsamp / 4096));
  HIP_TRY(ctx, grow(ctx, ctx->partials, (size_t)bps * 2 * sizeof(double)), "allocate");
  HIP_TRY(ctx, grow(ctx, ctx->norm, kNormFloats * sizeof(float)), "allocate");
  HIP_TRY(ctx, grow(ctx, ctx->flag, 16, true), "allocate");
  HIP_TRY(ctx, launch_stats(tmp.as<SeriesDev>(), 1, dtype, bps, ctx->partials.as<double>(),
                            stats_dev, ctx->norm.as<float>(), ctx->flag.as<int32_t>(), st),
          "stats kernels");
  HIP_TRY(ctx, hipStreamSynchronize(st), "synchronise");
  return FFA_OK;
}

ffa_status ffa_downsample(ffa_ctx* ctx, const void* series, int64_t nsamp, int32_t dtype,
                          const double* stats_dev, uint64_t ds_fx, int64_t nout, void* out_dev,
                          void* stream) {
  if (!ctx) return FFA_ERR_INVALID_ARG;
  if (!series || !out_dev) return fail(ctx, FFA_ERR_INVALID_ARG, "null series or out");
  if (reinterpret_cast<uintptr_t>(out_dev) & 15)  // outputs are stored 16 bytes at a time
    return fail(ctx, FFA_ERR_INVALID_ARG, "out must be 16-byte aligned");
  if (nsamp < 1 || nsamp > INT32_MAX) return fail(ctx, FFA_ERR_INVALID_ARG, "nsamp out of range");
  if (dtype != FFA_F32 && dtype != FFA_BF16 && dtype != FFA_F16)
    return fail(ctx, FFA_ERR_INVALID_ARG, "unknown dtype");
  if (ds_fx < (uint64_t(1) << 32) || (ds_fx >> 32) > (uint64_t)nsamp)
    return fail(ctx, FFA_ERR_INVALID_ARG, "need 2^32 <= ds_fx <= nsamp * 2^32");
  const int64_t nmax = (int64_t)(((uint64_t)nsamp << 32) / ds_fx);
  if (nout < 0 || nout > nmax) return fail(ctx, FFA_ERR_INVALID_ARG, "nout too large");
  if (nout == 0) return FFA_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int32_t halo = (int32_t)(ds_fx >> 32) + 2;
  const int32_t bs = downsample_block_samples(halo);
  if (bs <= 0) return fail(ctx, FFA_ERR_INVALID_ARG, "downsampling factor too large");
  SeriesDev sd{series, nsamp, 0, 0, 1, stats_dev ? 1 : 0, halo, bs, 0};
  OctaveDev od{ds_fx, nout, 0, 1.0 / (double)ds_fx};
  DevBuf t1, t2;
  HIP_TRY(ctx, t1.reserve(sizeof sd), "allocate");
  HIP_TRY(ctx, t2.reserve(sizeof od), "allocate");
  HIP_TRY(ctx, hipMemcpy(t1.ptr, &sd, sizeof sd, hipMemcpyHostToDevice), "upload");
  HIP_TRY(ctx, hipMemcpy(t2.ptr, &od, sizeof od, hipMemcpyHostToDevice), "upload");
  HIP_TRY(ctx, grow(ctx, ctx->norm, kNormFloats * sizeof(float)), "allocate");
  if (stats_dev)
    HIP_TRY(ctx, launch_norm_from_stats(stats_dev, ctx->norm.as<float>(), st), "norm kernel");
  const int64_t nblocks = (nsamp + bs - 1) / bs;
  HIP_TRY(ctx, launch_downsample(t1.as<SeriesDev>(), nullptr, t2.as<OctaveDev>(), ctx->norm.as<float>(),
                                 dtype, out_dev, dtype, nblocks, downsample_lds_floats(bs, halo), st),
          "downsample kernel");
  HIP_TRY(ctx, hipStreamSynchronize(st), "synchronise");
  return FFA_OK;
}

ffa_status ffa_running_median(ffa_ctx* ctx, const void* series, int64_t nsamp, int32_t dtype,
                              int32_t window, void* out_dev, int32_t out_dtype, void* stream) {
  if (!ctx) return FFA_ERR_INVALID_ARG;
  if (!series || !out_dev) return fail(ctx, FFA_ERR_INVALID_ARG, "null series or out");
  if (nsamp < 1 || nsamp > INT32_MAX) return fail(ctx, FFA_ERR_INVALID_ARG, "nsamp out of range");
  if (dtype != FFA_F32 && dtype != FFA_BF16 && dtype != FFA_F16)
    return fail(ctx, FFA_ERR_INVALID_ARG, "unknown dtype");
  if (out_dtype != FFA_F32 && out_dtype != FFA_BF16 && out_dtype != FFA_F16)
    return fail(ctx, FFA_ERR_INVALID_ARG, "unknown out_dtype");
  if (window < 1 || window % 2 == 0)
    return fail(ctx, FFA_ERR_INVALID_ARG, "the median window must be odd and positive");
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(ctx, grow(ctx, ctx->flag, 16, true), "allocate status word");
  HIP_TRY(ctx, launch_running_median(series, nsamp, dtype, window, out_dev, out_dtype,
                                     ctx->flag.as<int32_t>(), st),
          "running median kernel");
  return FFA_OK;
}

ffa_status ffa_sync_status(ffa_ctx* ctx, void* stream) {
  if (!ctx) return FFA_ERR_INVALID_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(ctx, hipStreamSynchronize(st), "synchronise");
  int32_t f = 0;
  if (ctx->flag.ptr) {
    HIP_TRY(ctx, hipMemcpy(&f, ctx->flag.ptr, sizeof f, hipMemcpyDeviceToHost), "read flag");
    HIP_TRY(ctx, launch_clear_flag(ctx->flag.as<int32_t>(), st), "clear flag");
  }
  if (ctx->na_used) {  // the status word of the no-allocation search
    int32_t g = 0;
    int32_t* na_flag = reinterpret_cast<int32_t*>(static_cast<unsigned char*>(ctx->na_ws) +
                                                  kNoAllocFlagOffset);
    HIP_TRY(ctx, hipMemcpy(&g, na_flag, sizeof g, hipMemcpyDeviceToHost), "read flag");
    HIP_TRY(ctx, launch_clear_flag(na_flag, st), "clear flag");
    f |= g;
  }
  HIP_TRY(ctx, hipStreamSynchronize(st), "synchronise");
  if (f & 2) return fail(ctx, FFA_ERR_DEVICE, "a fold dependency wait timed out");
  if (f & kMedErrBit) return fail(ctx, FFA_ERR_DEVICE, "running median: a block bound failed");
  if (f) return fail(ctx, FFA_ERR_DEGENERATE, "a normalised series had zero or non-finite variance");
  return FFA_OK;
}

ffa_status ffa_get_tiling(const ffa_ctx* ctx, ffa_tiling* out) {
  if (!ctx || !out) return FFA_ERR_INVALID_ARG;
  out->lds_rows = ctx->tiling.lds_rows;
  out->levels_per_pass = ctx->tiling.levels_per_pass;
  out->persistent = ctx->tiling.persistent;
  out->waves_per_group = ctx->tiling.waves;
  out->range_waves_per_group = ctx->tiling.range_waves;
  return FFA_OK;
}

ffa_status ffa_set_tiling(ffa_ctx* ctx, const ffa_tiling* t) {
  if (!ctx || !t) return FFA_ERR_INVALID_ARG;
  if (t->lds_rows < 0 || (t->lds_rows > 0 && t->lds_rows < 16) || t->levels_per_pass < 1 ||
      t->levels_per_pass > kMaxRangeLevels || (t->persistent != 0 && t->persistent != 1) ||
      (t->waves_per_group != kWavesLarge && t->waves_per_group != kWavesSmall) ||
      (t->range_waves_per_group != 0 && t->range_waves_per_group != kWavesLarge &&
       t->range_waves_per_group != kWavesSmall))
    return fail(ctx, FFA_ERR_INVALID_ARG,
                "need lds_rows = 0 or >= 16, 1 <= levels_per_pass <= 5, persistent 0 or 1, "
                "waves_per_group 8 or 16, range_waves_per_group 0, 8 or 16");
  ctx->tiling.lds_rows = t->lds_rows;
  ctx->tiling.levels_per_pass = t->levels_per_pass;
  ctx->tiling.persistent = t->persistent;
  ctx->tiling.waves = t->waves_per_group;
  ctx->tiling.range_waves = t->range_waves_per_group;
  return FFA_OK;
}

ffa_status ffa_set_timing(ffa_ctx* ctx, int32_t enable) {
  if (!ctx || (enable != 0 && enable != 1)) return FFA_ERR_INVALID_ARG;
  ctx->timing = enable != 0;
  return FFA_OK;
}

ffa_status ffa_read_timing(ffa_ctx* ctx, ffa_kernel_times* out, int32_t reset) {
  if (!ctx || !out) return FFA_ERR_INVALID_ARG;
  for (const TimedLaunch& t : ctx->pending) {
    HIP_TRY(ctx, hipEventSynchronize(t.stop), "synchronise timing event");
    float ms = 0.0f;
    HIP_TRY(ctx, hipEventElapsedTime(&ms, t.start, t.stop), "read timing event");
    if (t.kind == 0) {
      ctx->times.stats_ms += ms;
      ctx->times.stats_launches += 1;
    } else if (t.kind == 1) {
      ctx->times.downsample_ms += ms;
      ctx->times.downsample_launches += 1;
    } else if (t.kind == 2) {
      ctx->times.fold_ms += ms;
      ctx->times.fold_launches += 1;
    } else if (t.kind == 4) {
      ctx->times.median_ms += ms;
      ctx->times.median_launches += 1;
    } else {
      ctx->times.peaks_ms += ms;
      ctx->times.peaks_launches += 1;
    }
    ctx->event_pool.push_back(t.start);
    ctx->event_pool.push_back(t.stop);
  }
  ctx->pending.clear();
  *out = ctx->times;
  if (reset) ctx->times = ffa_kernel_times{};
  return FFA_OK;
}

// Rows of the smaller tile shape the autotuner tries next to the largest
// that fits (0): enough for the depth-5 subtrees of a 1073-row transform.
constexpr int32_t kTuneSmallTileRows = 40;

ffa_status ffa_autotune(ffa_ctx* ctx, int32_t nseries, const void* const* series,
                        const int64_t* nsamp, const ffa_search_params* params,
                        const char* cache_path, ffa_tiling* best, void* stream) {
  if (!ctx) return FFA_ERR_INVALID_ARG;
  ffa_status st = check_batch_args(ctx, nseries, series, nsamp, params);
  if (st != FFA_OK) return st;
  hipStream_t hs = static_cast<hipStream_t>(stream);
  // key of the batch's shape: everything that changes the tile tables
  std::string shape;
  {
    std::ostringstream k;
    k << nseries << '|';
    for (int i = 0; i < nseries; ++i)
      k << params[i].dtype << ',' << plan_key(params[i], nsamp[i]) << ';';
    uint64_t h = 1469598103934665603ull;  // FNV-1a
    for (unsigned char c : k.str()) h = (h ^ c) * 1099511628211ull;
    char buf[32];
    snprintf(buf, sizeof buf, "%016llx", (unsigned long long)h);
    shape = buf;
  }
  auto report = [&](const Tiling& t) {
    ctx->tiling = t;
    if (best) {
      best->lds_rows = t.lds_rows;
      best->levels_per_pass = t.levels_per_pass;
      best->persistent = t.persistent;
      best->waves_per_group = t.waves;
      best->range_waves_per_group = t.range_waves;
    }
  };
  if (cache_path) {
    if (FILE* f = fopen(cache_path, "r")) {
      char key[64];
      int lr, lv, pe, wv, rw;
      bool hit = false;
      Tiling t;
      while (fscanf(f, "%63s %d %d %d %d %d", key, &lr, &lv, &pe, &wv, &rw) == 6) {
        if (shape == key) {
          t.lds_rows = lr;
          t.levels_per_pass = lv;
          t.persistent = pe;
          t.waves = wv;
          t.range_waves = rw;
          hit = true;
        }
      }
      fclose(f);
      if (hit) {
        report(t);
        return FFA_OK;
      }
    }
  }
  // output rows of the batch, packed
  std::vector<int64_t> offs(nseries);
  int64_t rows = 0;
  for (int i = 0; i < nseries; ++i) {
    std::shared_ptr<SeriesPlan> plan;
    st = get_plan(ctx, params[i], nsamp[i], &plan);
    if (st != FFA_OK) return st;
    offs[i] = rows;
    rows += plan->rows;
  }
  HIP_TRY(ctx, ctx->tune_out.reserve((size_t)rows * params[0].num_widths * 4 + 16),
          "allocate autotune output");
  float* out = ctx->tune_out.as<float>();
  hipEvent_t e0, e1;
  HIP_TRY(ctx, hipEventCreate(&e0), "create event");
  HIP_TRY(ctx, hipEventCreate(&e1), "create event");
  const Tiling saved = ctx->tiling;
  Tiling winner = saved;
  float best_ms = 1e30f;
  const bool timing = ctx->timing;
  ctx->timing = false;
  for (int waves : {kWavesSmall, kWavesLarge})
    for (int range_waves : {0, kWavesSmall + kWavesLarge - waves})
    for (int levels : {3, 4, 5})
      for (int persistent : {0, 1})
      for (int lds_rows : {0, kTuneSmallTileRows}) {
        if (persistent && range_waves) continue;  // one launch: one workgroup size
        Tiling t;
        t.waves = waves;
        t.range_waves = range_waves;
        t.levels_per_pass = levels;
        t.persistent = persistent;
        t.lds_rows = lds_rows;
        ctx->tiling = t;
        // first call builds the tables and warms the caches
        st = run_batch(ctx, nseries, series, nsamp, params, offs.data(), out, rows, 0, hs);
        if (st != FFA_OK) break;
        float ms_total = 0.0f;
        for (int rep = 0; rep < 2; ++rep) {
          HIP_TRY(ctx, hipEventRecord(e0, hs), "record event");
          st = run_batch(ctx, nseries, series, nsamp, params, offs.data(), out, rows, 0, hs);
          if (st != FFA_OK) break;
          HIP_TRY(ctx, hipEventRecord(e1, hs), "record event");
          HIP_TRY(ctx, hipEventSynchronize(e1), "synchronise event");
          float ms = 0.0f;
          HIP_TRY(ctx, hipEventElapsedTime(&ms, e0, e1), "read event");
          ms_total += ms;
        }
        if (st != FFA_OK) break;
        if (ms_total < best_ms) {
          best_ms = ms_total;
          winner = t;
        }
        // drop the candidate's tables: only the winner's are kept below
        ctx->jobs.clear();
      }
  ctx->timing = timing;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != FFA_OK) {
    ctx->tiling = saved;
    return st;
  }
  report(winner);
  if (cache_path) {
    if (FILE* f = fopen(cache_path, "a")) {
      fprintf(f, "%s %d %d %d %d %d\n", shape.c_str(), winner.lds_rows, winner.levels_per_pass,
              winner.persistent, winner.waves, winner.range_waves);
      fclose(f);
    }
  }
  return FFA_OK;
}

ffa_status ffa_find_peaks_batch(ffa_ctx* ctx, int32_t nseries, const int64_t* nsamp,
                                const ffa_search_params* params, const int64_t* row_offset,
                                const float* snr_dev, int64_t capacity_rows,
                                const ffa_peak_params* pp, ffa_peak* peaks_host,
                                int64_t capacity_peaks, int64_t* npeaks_host, double* poly_host,
                                void* stream) {
  if (!ctx) return FFA_ERR_INVALID_ARG;
  if (nseries < 1 || !nsamp || !params || !row_offset || !snr_dev || !pp || !npeaks_host ||
      capacity_peaks < 0 || (capacity_peaks > 0 && !peaks_host) || capacity_rows < 0)
    return fail(ctx, FFA_ERR_INVALID_ARG, "null argument, nseries < 1 or negative capacity");
  if (!(pp->dz_seg > 0.0) || !std::isfinite(pp->dz_seg) || !std::isfinite(pp->k_sigma) ||
      pp->degree < 0 || pp->degree > kPeakMaxDegree || pp->min_points < 1 ||
      !(pp->cluster_gap >= 0.0) || !std::isfinite(pp->cluster_gap))
    return fail(ctx, FFA_ERR_INVALID_ARG,
                "peak parameters: dz_seg > 0, finite k_sigma, degree 0..4, min_points >= 1, "
                "finite cluster_gap >= 0");
  const int32_t nw = params[0].num_widths;
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(ctx, hipSetDevice(ctx->device), "set device");
  // plans and their frequency tables; the device tables (one copy per
  // distinct plan, and the series table) are uploaded again only when the
  // batch differs from the previous call's
  std::vector<std::shared_ptr<SeriesPlan>> plans(nseries);
  std::vector<std::shared_ptr<PeakPlan>> pks(nseries);
  std::vector<std::string> keys(nseries);
  std::ostringstream call_key;
  call_key.precision(17);
  call_key << nseries << '|' << pp->cluster_gap << '|';
  for (int32_t i = 0; i < nseries; ++i) {
    if (params[i].num_widths != nw)
      return fail(ctx, FFA_ERR_INVALID_ARG, "all series need the same number of widths");
    ffa_status rs = get_plan(ctx, params[i], nsamp[i], &plans[i]);
    if (rs != FFA_OK) return rs;
    const SeriesPlan& plan = *plans[i];
    if (row_offset[i] < 0 || row_offset[i] + plan.rows > capacity_rows)
      return fail(ctx, FFA_ERR_INVALID_ARG, "series rows past capacity_rows");
    std::ostringstream key;
    key.precision(17);
    key << plan_key(params[i], nsamp[i]) << '|' << pp->dz_seg;
    keys[i] = key.str();
    auto it = ctx->peak_plans.find(keys[i]);
    if (it != ctx->peak_plans.end()) {
      pks[i] = it->second;
    } else {
      pks[i] = std::make_shared<PeakPlan>();
      ffa_status bs = build_peak_plan(ctx, plan, (double)nsamp[i] * params[i].tsamp,
                                      pp->dz_seg, pks[i].get());
      if (bs != FFA_OK) return bs;
      ctx->peak_plans[keys[i]] = pks[i];
    }
    call_key << keys[i] << '@' << row_offset[i] << ';';
  }
  if (call_key.str() != ctx->pk_key) {
    ctx->pk_key.clear();
    std::vector<PeakSeriesDev> sdev(nseries);
    std::vector<double> nu, lognu, segx;
    std::vector<int32_t> segb, sege, mid, big;
    std::map<std::string, std::pair<int64_t, int32_t>> placed;  // key -> (freq0, seg0)
    int32_t max_nseg = 0, max_seg = 0;
    for (int32_t i = 0; i < nseries; ++i) {
      const PeakPlan& pk = *pks[i];
      auto pl = placed.find(keys[i]);
      if (pl == placed.end()) {
        pl = placed.emplace(keys[i], std::make_pair((int64_t)nu.size(), (int32_t)segb.size())).first;
        nu.insert(nu.end(), pk.nu.begin(), pk.nu.end());
        lognu.insert(lognu.end(), pk.lognu.begin(), pk.lognu.end());
        segb.insert(segb.end(), pk.seg_begin.begin(), pk.seg_begin.end());
        sege.insert(sege.end(), pk.seg_end.begin(), pk.seg_end.end());
        segx.insert(segx.end(), pk.seg_x.begin(), pk.seg_x.end());
      }
      PeakSeriesDev& d = sdev[i];
      d.snr_row0 = row_offset[i];
      d.rows = plans[i]->rows;
      d.freq0 = pl->second.first;
      d.seg0 = pl->second.second;
      d.nseg = (int32_t)pk.seg_begin.size();
      d.gap = pp->cluster_gap / ((double)nsamp[i] * params[i].tsamp);
      max_nseg = std::max(max_nseg, d.nseg);
      max_seg = std::max(max_seg, pk.max_seg);
      for (int32_t q = 0; q < d.nseg; ++q) {
        const int32_t len = pk.seg_end[q] - pk.seg_begin[q];
        if (len > kPeakWaveSortMax) {
          std::vector<int32_t>& to = len > 2 * kPeakWaveSortMax ? big : mid;
          to.push_back(i);
          to.push_back(q);
        }
      }
    }
    if (max_seg > kPeakSegMax)
      return fail(ctx, FFA_ERR_INVALID_ARG,
                  "a frequency segment holds more than 8192 rows: lower dz_seg");
    HIP_TRY(ctx, upload(ctx->pk_series, sdev), "upload peak series table");
    HIP_TRY(ctx, upload(ctx->pk_nu, nu), "upload frequencies");
    HIP_TRY(ctx, upload(ctx->pk_lognu, lognu), "upload log frequencies");
    HIP_TRY(ctx, upload(ctx->pk_segb, segb), "upload segments");
    HIP_TRY(ctx, upload(ctx->pk_sege, sege), "upload segments");
    HIP_TRY(ctx, upload(ctx->pk_segx, segx), "upload segment centres");
    HIP_TRY(ctx, upload(ctx->pk_mid, mid), "upload large segments");
    HIP_TRY(ctx, upload(ctx->pk_big, big), "upload large segments");
    ctx->pk_nmid = (int32_t)(mid.size() / 2);
    ctx->pk_nbig = (int32_t)(big.size() / 2);
    ctx->pk_key = call_key.str();
    ctx->pk_max_nseg = max_nseg;
    ctx->pk_max_seg = max_seg;
  }
  const int32_t max_nseg = ctx->pk_max_nseg;
  const size_t nfit = (size_t)nseries * nw;
  int64_t max_rows = 0;
  for (int32_t i = 0; i < nseries; ++i) max_rows = std::max(max_rows, plans[i]->rows);
  const int64_t nwords = (max_rows + 63) / 64;
  HIP_TRY(ctx, ctx->pk_flags.reserve(std::max<size_t>(nfit * nwords * 8, 16)), "peak flags");
  HIP_TRY(ctx, ctx->pk_ctrl.reserve(std::max<size_t>(nfit * std::max(max_nseg, 1) * 8, 16)),
          "peak control points");
  HIP_TRY(ctx, ctx->pk_fits.reserve(nfit * sizeof(PeakFitDev)), "peak fits");
  HIP_TRY(ctx, ctx->pk_peaks.reserve(std::max<int64_t>(capacity_peaks, 1) * sizeof(PeakDev)),
          "peak records");
  HIP_TRY(ctx, ctx->pk_count.reserve((size_t)(nseries + 1) * 4), "peak counters");
  HIP_TRY(ctx, hipMemsetAsync(ctx->pk_count.ptr, 0, (size_t)(nseries + 1) * 4, st),
          "clear peak counters");
  PeakArgs a{};
  a.series = ctx->pk_series.as<PeakSeriesDev>();
  a.nseries = nseries;
  a.num_widths = nw;
  a.max_nseg = max_nseg;
  a.degree = pp->degree;
  a.min_points = pp->min_points;
  a.k_sigma = pp->k_sigma;
  a.snr = snr_dev;
  a.nu = ctx->pk_nu.as<double>();
  a.lognu = ctx->pk_lognu.as<double>();
  a.seg_begin = ctx->pk_segb.as<int32_t>();
  a.seg_end = ctx->pk_sege.as<int32_t>();
  a.seg_x = ctx->pk_segx.as<double>();
  a.mid = ctx->pk_mid.as<int32_t>();
  a.big = ctx->pk_big.as<int32_t>();
  a.nmid = ctx->pk_nmid;
  a.nbig = ctx->pk_nbig;
  a.ctrl = ctx->pk_ctrl.as<double>();
  a.fits = ctx->pk_fits.as<PeakFitDev>();
  a.flags = ctx->pk_flags.as<uint64_t>();
  a.nwords = nwords;
  a.peaks = ctx->pk_peaks.as<PeakDev>();
  a.capacity = capacity_peaks;
  a.count = ctx->pk_count.as<int32_t>();
  {
    TimedScope ts(ctx, 3, st, ctx->timing);
    HIP_TRY(ctx, launch_peak_ctrl(a, st), "peak control-point kernels");
  }
  {
    TimedScope ts(ctx, 3, st, ctx->timing);
    HIP_TRY(ctx, launch_peak_fit(a, st), "peak fit kernel");
  }
  {
    TimedScope ts(ctx, 3, st, ctx->timing);
    HIP_TRY(ctx, launch_peak_scan(a, st), "peak scan kernel");
  }
  std::vector<int32_t> cnt(nseries + 1);
  std::vector<PeakFitDev> fits(nfit);
  HIP_TRY(ctx, hipMemcpyAsync(cnt.data(), ctx->pk_count.ptr, cnt.size() * 4, hipMemcpyDeviceToHost, st),
          "read peak counters");
  HIP_TRY(ctx, hipMemcpyAsync(fits.data(), ctx->pk_fits.ptr, nfit * sizeof(PeakFitDev),
                              hipMemcpyDeviceToHost, st),
          "read peak fits");
  HIP_TRY(ctx, hipStreamSynchronize(st), "synchronise peak detection");
  for (int32_t i = 0; i < nseries; ++i) npeaks_host[i] = cnt[1 + i];
  if (poly_host) {
    const int nc = pp->degree + 1;
    for (size_t q = 0; q < nfit; ++q) {
      if (fits[q].ok)
        expand_poly(fits[q], pp->degree, poly_host + q * nc);
      else
        for (int j = 0; j < nc; ++j) poly_host[q * nc + j] = NAN;
    }
  }
  const int64_t total = cnt[0];
  if (total > capacity_peaks)
    return fail(ctx, FFA_ERR_BUFFER_TOO_SMALL, "more peaks than capacity_peaks");
  std::vector<PeakDev> pk(total);
  if (total > 0) {
    HIP_TRY(ctx, hipMemcpy(pk.data(), ctx->pk_peaks.ptr, total * sizeof(PeakDev), hipMemcpyDeviceToHost),
            "read peaks");
  }
  std::sort(pk.begin(), pk.end(), [](const PeakDev& x, const PeakDev& y) {
    if (x.series != y.series) return x.series < y.series;
    if (x.width != y.width) return x.width < y.width;
    return x.row < y.row;
  });
  for (int64_t q = 0; q < total; ++q) {
    const PeakDev& d = pk[q];
    const SeriesPlan& plan = *plans[d.series];
    // period of the row from the plan (the same formula as ffa_plan_export);
    // transforms are in row order, so the row's transform is the last one
    // starting at or before it that keeps rows
    double period = NAN;
    auto it = std::upper_bound(plan.tr.begin(), plan.tr.end(), d.row,
                               [](int64_t row, const Transform& t) { return row < t.row0; });
    while (it != plan.tr.begin()) {
      const Transform& t = *--it;
      if (t.keep == 0) continue;
      if (d.row < t.row0 + t.keep)
        period = trial_period(d.row - t.row0, t.m, t.p, plan.oct[t.octave].tau);
      break;
    }
    ffa_peak& o = peaks_host[q];
    o.row = d.row;
    o.period = period;
    o.threshold = d.threshold;
    o.snr = d.snr;
    o.series = d.series;
    o.width_index = d.width;
    o.members = d.members;
  }
  return FFA_OK;
}

}  // extern "C"
