// C ABI of the batched TaylorF2 likelihood library (see include/gwlnl.h).
// Validates arguments on the host, sizes the library-owned workspace, plans
// the launch and enqueues the kernels of gw_kernels.hip on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "gw_build_id.h"
#include "gw_internal.h"
#include "gw_plan.h"
#include "gwlnl.h"

// Tile-kernel blocks per CU by (form, precision, detectors, tile bins).
using OccupancyCache = std::map<std::tuple<int, int, int, int>, int>;

struct gw_workspace {
    int device = 0;
    int n_cu = 0;
    OccupancyCache occupancy;
    // single-event plans chosen by timing, by (detectors, precision and form,
    // log2 bins, log2 samples): (tile bins, work-queue rounds)
    bool tune_single = true;
    std::map<std::tuple<int, int, int, int>, std::pair<int, int>> single_tuning;
    void *base = nullptr;
    size_t capacity = 0;
    bool timing = false;
    std::vector<hipEvent_t> events;   // start/stop pairs of the hot kernel
    int64_t timed = 0;                 // pairs recorded since timing was enabled
    // ragged batches: a captured graph of the last plan, replayed while the
    // call (events, pointers, precision) and the workspace stay the same
    hipStream_t capture_stream = nullptr;
    std::vector<unsigned char> ragged_key;
    hipGraph_t ragged_graph = nullptr;
    hipGraphExec_t ragged_exec = nullptr;
    // autotuned (tile bins, chunk bins) by (max detectors, precision, size bucket)
    std::map<std::tuple<int, int, int>, std::pair<int, int64_t>> ragged_tuning;
    int last_tile_bins = 0;
    int64_t last_chunk_bins = 0;
    // the bin tables (tab1, tab2) in the arena are those of this grid at
    // these offsets, written by an earlier call on the workspace's stream order
    bool tables_valid = false;
    gw_grid tables_grid{};
    size_t tables_tab1 = 0, tables_tab2 = 0;
    // a call on this workspace has been captured into a graph: the arena
    // never grows again (growing frees it)
    bool pinned = false;
};

// One event prepared for relative binning: a single device allocation
// carved into the sections below (layout in gw_internal.h, namespace rb).
struct gw_relbin {
    int device = 0;
    gw_grid grid{};
    int n_det = 0, n_param = 0;
    unsigned flags = 0;
    int64_t n_rb = 0;                 // bins B; edges B + 1
    gw::DetGeom geom{};
    void *mem = nullptr;
    int64_t *edge_idx = nullptr;
    gw::rb::RbEdge *edges = nullptr;
    gw::rb::RbCoef *coef = nullptr;
    gw::rb::RbEnds *ends = nullptr;
    double *raw = nullptr, *bin_dd = nullptr, *totals = nullptr, *fid = nullptr;
};

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char *where)
{
    return fail(GW_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

// Sets the workspace's device current for the lifetime of the guard.
struct DeviceGuard {
    int previous = -1;
    bool ok = true;
    explicit DeviceGuard(int device)
    {
        if (hipGetDevice(&previous) != hipSuccess) { ok = false; return; }
        if (previous != device && hipSetDevice(device) != hipSuccess) ok = false;
    }
    ~DeviceGuard()
    {
        int now = -1;
        if (previous >= 0 && hipGetDevice(&now) == hipSuccess && now != previous) (void)hipSetDevice(previous);
    }
};

constexpr size_t kAlign = 256;
#define GW_PI_HOST 3.141592653589793
constexpr unsigned kLnlFlags = GW_FLAG_DIRECT | GW_FLAG_TERM_ISCO | GW_FLAG_ADD_NORM;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Bump allocator over the workspace arena: sections are carved in order.
struct Carver {
    size_t offset = 0;
    size_t take(size_t bytes)
    {
        const size_t at = offset;
        offset = align_up(offset + bytes);
        return at;
    }
};

void drop_ragged_graph(gw_workspace *ws)
{
    if (ws->ragged_exec) (void)hipGraphExecDestroy(ws->ragged_exec);
    if (ws->ragged_graph) (void)hipGraphDestroy(ws->ragged_graph);
    ws->ragged_exec = nullptr;
    ws->ragged_graph = nullptr;
    ws->ragged_key.clear();
}

// True while `stream` is recording into a graph.  A captured call must carry
// every kernel that fills what it reads, since its replays run later, after
// other calls may have changed the arena.
bool capturing(hipStream_t stream)
{
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(stream, &st) == hipSuccess && st != hipStreamCaptureStatusNone;
}

// Bin tables of `grid` at (tab1, tab2): launch their kernel unless the arena
// already holds them there.  A call under capture always records the kernel,
// and pins the workspace; on a pinned workspace the tables are never taken as
// held (a graph replay may rewrite the arena at any time), so every call
// launches the kernel.
hipError_t bin_tables(gw_workspace *ws, const gw_grid &grid, size_t off1, size_t off2, gw::Tab1 *tab1,
                      gw::Tab2 *tab2, hipStream_t stream)
{
    if (capturing(stream)) ws->pinned = true;
    if (!ws->pinned && ws->tables_valid && ws->tables_tab1 == off1 && ws->tables_tab2 == off2 &&
        ws->tables_grid.f_low == grid.f_low && ws->tables_grid.delta_f == grid.delta_f &&
        ws->tables_grid.n_bins == grid.n_bins)
        return hipSuccess;
    ws->tables_valid = false;
    hipError_t e = gw::launch_event_tables(grid, tab1, tab2, stream);
    if (e != hipSuccess || ws->pinned) return e;
    ws->tables_valid = true;
    ws->tables_grid = grid;
    ws->tables_tab1 = off1;
    ws->tables_tab2 = off2;
    return hipSuccess;
}

// Grows the arena to `bytes` (freeing the old one), unless it is large enough.
// A call being captured into a graph may not grow it: the graph would hold
// pointers into an arena allocated during capture.
// Once a call on the workspace has been captured, the arena is pinned: a graph
// may still refer to it, so it never grows (which would free it) again.
int ensure_capacity(gw_workspace *ws, size_t bytes, hipStream_t stream)
{
    const bool captured = capturing(stream);
    if (captured) ws->pinned = true;
    if (bytes <= ws->capacity) return GW_OK;
    if (captured)
        return fail(GW_EINVAL, "the workspace is too small for a call under graph capture: "
                               "size it first (gw_workspace_reserve, or one eager call of the same shape)");
    if (ws->pinned)
        return fail(GW_EINVAL, "a graph captured from a call on this workspace may still use its memory, so it "
                               "cannot grow; use another workspace for larger calls");
    ws->tables_valid = false;
    drop_ragged_graph(ws);               // its kernels point into the old arena
    if (ws->base) {
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize before growing the workspace");
        e = hipFree(ws->base);
        ws->base = nullptr;
        ws->capacity = 0;
        if (e != hipSuccess) return hip_fail(e, "hipFree");
    }
    const size_t want = align_up(bytes + bytes / 8);
    hipError_t e = hipMalloc(&ws->base, want);
    if (e != hipSuccess) {
        ws->base = nullptr;
        return fail(GW_ENOMEM, "workspace hipMalloc of " + std::to_string(want) + " bytes failed");
    }
    ws->capacity = want;
    return GW_OK;
}

int check_grid(const gw_grid *grid)
{
    if (!grid) return fail(GW_EINVAL, "grid is NULL");
    if (!(grid->delta_f > 0.0) || !std::isfinite(grid->delta_f)) return fail(GW_EINVAL, "delta_f must be finite and > 0");
    if (!(grid->f_low > 0.0) || !std::isfinite(grid->f_low)) return fail(GW_EINVAL, "f_low must be finite and > 0");
    if (grid->n_bins < 1) return fail(GW_EINVAL, "n_bins must be >= 1");
    return GW_OK;
}

int check_dets(int n_det, const gw_detector *dets, int n_param, gw::DetGeom *geom)
{
    std::memset(geom, 0, sizeof(*geom));
    if (!gw::param_has_sky(n_param)) return GW_OK;   // optimally oriented: geometry unused
    if (!dets) return fail(GW_EINVAL, "dets is NULL");
    for (int d = 0; d < n_det; ++d) {
        for (int i = 0; i < 9; ++i) {
            if (!std::isfinite(dets[d].tensor[i])) return fail(GW_EINVAL, "detector tensor is not finite");
            geom->tensor[d][i] = dets[d].tensor[i];
        }
        for (int i = 0; i < 3; ++i) {
            if (!std::isfinite(dets[d].vertex[i])) return fail(GW_EINVAL, "detector vertex is not finite");
            geom->vertex[d][i] = dets[d].vertex[i];
        }
    }
    return GW_OK;
}

// Launch plan of one event for a device with n_cu compute units, with the
// given tile size and work-queue rounds (tile_bins 0: the largest tile the
// LDS budget allows; rounds < 0: GW_TILE_ROUNDS).  occ caches occupancies.
gw::TilePlan plan_tiles_on(int n_cu, OccupancyCache &occ, int64_t n_bins, int n_det, int64_t n_samples, bool mixed,
                           int form, int tile_bins = 0, int rounds = -1)
{
    if (tile_bins <= 0) tile_bins = gw::tile_bins_for(n_det, form, mixed);
    int &o = occ[std::make_tuple(form, mixed ? 1 : 0, n_det, tile_bins)];
    if (o == 0) o = gw::lnl_tile_blocks_per_cu(n_det, tile_bins, mixed, form);
    return gw::plan_single_event(n_bins, n_samples, form, tile_bins, (int64_t)n_cu * o,
                                 rounds < 0 ? GW_TILE_ROUNDS : rounds);
}

int log2_bucket(int64_t n) { return n > 0 ? (int)std::floor(std::log2((double)n)) : 0; }

std::tuple<int, int, int, int> tuning_key(int64_t n_bins, int n_det, int64_t n_samples, bool mixed, int form)
{
    return std::make_tuple(n_det, (mixed ? 1 : 0) + 2 * form, log2_bucket(n_bins), log2_bucket(n_samples));
}

// The plan gw_lnl_batch uses on this workspace: the tuned one of the size
// bucket when the autotuner has timed it, else the default.
gw::TilePlan plan_tiles(gw_workspace *ws, int64_t n_bins, int n_det, int64_t n_samples, bool mixed, int form)
{
    auto it = ws->single_tuning.find(tuning_key(n_bins, n_det, n_samples, mixed, form));
    if (it != ws->single_tuning.end())
        return plan_tiles_on(ws->n_cu, ws->occupancy, n_bins, n_det, n_samples, mixed, form, it->second.first,
                             it->second.second);
    return plan_tiles_on(ws->n_cu, ws->occupancy, n_bins, n_det, n_samples, mixed, form);
}

// Workspace sections of one event.  The direct-form tables and the prefix
// sums are carved only when the call's flags use them.
struct LnlLayout {
    size_t tab1, tab2, dcoef, edir, vdir, qprefix, qoffsets, prep_partials, event_sums, k_limit, records, partials,
        queue, total;
    int prep_blocks;
};

LnlLayout lnl_layout(int64_t n_bins, int n_det, int64_t n_samples, const gw::TilePlan &plan, unsigned flags)
{
    LnlLayout l;
    Carver c;
    const bool direct = (flags & GW_FLAG_DIRECT) != 0, isco = (flags & GW_FLAG_TERM_ISCO) != 0;
    l.prep_blocks = (int)((n_bins + gw::kBlock - 1) / gw::kBlock);
    l.tab1 = c.take(sizeof(gw::Tab1) * n_bins);
    l.tab2 = c.take(sizeof(gw::Tab2) * n_bins);
    l.dcoef = c.take(sizeof(double2) * n_bins * n_det);
    l.edir = direct ? c.take(sizeof(double2) * n_bins * n_det) : 0;
    l.vdir = direct ? c.take(sizeof(double) * n_bins * n_det) : 0;
    l.qprefix = isco ? c.take(sizeof(double) * n_bins * n_det) : 0;
    l.qoffsets = isco ? c.take(sizeof(double) * (size_t)l.prep_blocks * n_det) : 0;
    l.prep_partials = c.take(sizeof(double) * gw::kPrepPerDet * n_det * l.prep_blocks);
    l.event_sums = c.take(sizeof(double) * gw::kEventSums);
    l.k_limit = c.take(sizeof(int64_t));
    l.records = c.take(sizeof(double) * gw::record_fields(n_det) * std::max<int64_t>(n_samples, 1));
    l.partials = c.take(sizeof(double) * (size_t)plan.n_chunks * n_samples);   // one total per chunk and sample
    l.queue = c.take(sizeof(unsigned) * gw::kQueues);
    l.total = c.offset;
    return l;
}

template <typename T>
T *at(gw_workspace *ws, size_t offset)
{
    return reinterpret_cast<T *>(static_cast<char *>(ws->base) + offset);
}

int check_common(gw_workspace *ws, const gw_grid *grid, int n_det_min, int n_det, int n_param, int64_t n_samples)
{
    if (!ws) return fail(GW_EINVAL, "workspace is NULL");
    if (int rc = check_grid(grid)) return rc;
    if (n_det < n_det_min || n_det > gw::kMaxDet) return fail(GW_EINVAL, "n_det out of range");
    if (!gw::valid_n_param(n_param)) return fail(GW_EINVAL, "n_param must be 5, 7, 9 or 11");
    if (n_samples < 0) return fail(GW_EINVAL, "n_samples must be >= 0");
    return GW_OK;
}

// The start/stop events of the next timed hot-kernel launch, or two nullptrs
// while timing is off.  The pair counts once timer_stop has recorded its stop.
int timer_pair(gw_workspace *ws, hipStream_t stream, hipEvent_t *start, hipEvent_t *stop)
{
    *start = *stop = nullptr;
    if (!ws->timing || capturing(stream)) return GW_OK;
    while ((size_t)(2 * ws->timed + 2) > ws->events.size()) {
        hipEvent_t ev;
        hipError_t e = hipEventCreate(&ev);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
        ws->events.push_back(ev);
    }
    *start = ws->events[2 * ws->timed];
    *stop = ws->events[2 * ws->timed + 1];
    return GW_OK;
}

int timer_stop(gw_workspace *ws, hipEvent_t stop, hipStream_t stream)
{
    if (!stop) return GW_OK;
    hipError_t e = hipEventRecord(stop, stream);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    ++ws->timed;
    return GW_OK;
}

// The kernels of one gw_lnl_batch call over device memory at `base`, laid
// out by `l` for `plan`.  With a workspace, the bin tables it already holds
// are reused and the hot kernel is timed when timing is on; without one
// (ws == nullptr) every kernel is launched and nothing is timed.
int lnl_enqueue(gw_workspace *ws, char *base, const LnlLayout &l, const gw::TilePlan &plan, const gw_grid &grid,
                int n_det, const gw::DetGeom &geom, const gw_c128 *data, const double *psd, const double *theta,
                int n_param, int64_t n_samples, double *lnl_out, bool mixed, unsigned flags, hipStream_t stream)
{
    const int form = gw::tile_form(flags);
    const bool isco = (flags & GW_FLAG_TERM_ISCO) != 0;
    auto sec = [base](size_t offset) { return static_cast<void *>(base + offset); };
    gw::EventBuffers eb;
    eb.tab1 = static_cast<gw::Tab1 *>(sec(l.tab1));
    eb.tab2 = static_cast<gw::Tab2 *>(sec(l.tab2));
    eb.dcoef = static_cast<double2 *>(sec(l.dcoef));
    eb.edir = l.edir ? static_cast<double2 *>(sec(l.edir)) : nullptr;
    eb.vdir = l.vdir ? static_cast<double *>(sec(l.vdir)) : nullptr;
    eb.qprefix = l.qprefix ? static_cast<double *>(sec(l.qprefix)) : nullptr;
    eb.qoffsets = l.qoffsets ? static_cast<double *>(sec(l.qoffsets)) : nullptr;
    eb.prep = static_cast<double *>(sec(l.prep_partials));
    eb.prep_blocks = l.prep_blocks;
    eb.sums = static_cast<double *>(sec(l.event_sums));
    eb.k_limit = static_cast<int64_t *>(sec(l.k_limit));
    eb.queue = plan.rounds > 0 ? static_cast<unsigned *>(sec(l.queue)) : nullptr;
    auto *rec = static_cast<double *>(sec(l.records));
    auto *part = static_cast<double2 *>(sec(l.partials));
    hipError_t e;
    if (ws)
        e = bin_tables(ws, grid, l.tab1, l.tab2, eb.tab1, eb.tab2, stream);
    else
        e = gw::launch_event_tables(grid, eb.tab1, eb.tab2, stream);
    if (e != hipSuccess) return hip_fail(e, "event tables");
    gw::SamplePrep sp;
    sp.n_samples = n_samples;
    sp.n_param = n_param;
    sp.isco = isco ? 1 : 0;
    sp.geom = geom;
    sp.theta = theta;
    sp.records = rec;
    if ((e = gw::launch_event_data(grid, n_det, data, psd, eb, flags, &sp, stream)) != hipSuccess)
        return hip_fail(e, "event data and sample prep");
    if (form == gw::kFormSplitIsco && (e = gw::launch_isco_limit(n_samples, rec, eb.k_limit, stream)) != hipSuccess)
        return hip_fail(e, "template-end limit");
    hipEvent_t t_start = nullptr, t_stop = nullptr;
    if (ws) {
        if (int rc = timer_pair(ws, stream, &t_start, &t_stop)) return rc;
    }
    if (t_start && (e = hipEventRecord(t_start, stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    if ((e = gw::launch_lnl_tiles(grid, n_det, n_samples, plan, mixed, form, eb, rec, part, stream)) != hipSuccess)
        return hip_fail(e, "lnl tiles");
    if (ws) {
        if (int rc = timer_stop(ws, t_stop, stream)) return rc;
    }
    if ((e = gw::launch_lnl_finalize(grid, n_samples, n_det, plan, part, rec, eb, flags, lnl_out, stream)) !=
        hipSuccess)
        return hip_fail(e, "lnl finalize");
    return GW_OK;
}

bool same_plan(const gw::TilePlan &a, const gw::TilePlan &b)
{
    return a.tile_bins == b.tile_bins && a.rounds == b.rounds && a.chunk_bins == b.chunk_bins &&
           a.n_chunks == b.n_chunks && a.n_groups == b.n_groups && a.blocks == b.blocks;
}

// The distinct plans the autotuner times for a size class: tile bins, the
// largest the LDS budget allows and half of it; work-queue rounds 0, 4, 6 and
// 8 (only 0 with the template end).  A rounds request the size cannot take
// falls back to one item per block, so some requests give the same plan.
std::vector<gw::TilePlan> tuning_candidates(gw_workspace *ws, int64_t n_bins, int n_det, int64_t n_samples,
                                            bool mixed, int form)
{
    const int big = gw::tile_bins_for(n_det, form, mixed);
    std::vector<gw::TilePlan> plans;
    for (int tb : {big, big / 2}) {
        if (tb < 64) continue;
        for (int r : {0, 4, 6, 8}) {
            if (form == gw::kFormSplitIsco && r > 0) continue;
            const gw::TilePlan p = plan_tiles_on(ws->n_cu, ws->occupancy, n_bins, n_det, n_samples, mixed, form, tb, r);
            bool seen = false;
            for (const gw::TilePlan &q : plans) seen = seen || same_plan(p, q);
            if (!seen) plans.push_back(p);
        }
    }
    return plans;
}

// Calls of at least this many (sample, bin) pairs are worth timing plans for.
constexpr double kTuneMinPairs = 1 << 24;
// A candidate replaces the default plan only when it is faster by this
// fraction, so that timing noise between plans of equal speed does not make
// the choice differ from one run to the next.
constexpr float kTuneMargin = 0.03f;

// The autotuner of gw_lnl_batch: times the whole call under every candidate
// plan of the size class, twice each in interleaved passes after one warm-up
// call, and records for the class the fastest by its shorter time, or the
// default plan unless the fastest beats it by kTuneMargin.  The caller then
// computes the call's result with that plan.  It waits for the caller's
// stream.
int tune_single_event(gw_workspace *ws, const gw_grid &grid, int n_det, const gw::DetGeom &geom,
                      const gw_c128 *data, const double *psd, const double *theta, int n_param, int64_t n_samples,
                      double *lnl_out, bool mixed, unsigned flags, hipStream_t stream)
{
    const int form = gw::tile_form(flags);
    const std::vector<gw::TilePlan> plans = tuning_candidates(ws, grid.n_bins, n_det, n_samples, mixed, form);
    size_t need = 0;
    for (const gw::TilePlan &p : plans) need = std::max(need, lnl_layout(grid.n_bins, n_det, n_samples, p, flags).total);
    if (int rc = ensure_capacity(ws, need, stream)) return rc;
    const bool timing = ws->timing;
    ws->timing = false;                  // the trial calls are not measurements of the caller's
    hipEvent_t ev[2];
    hipError_t e = hipEventCreate(&ev[0]);
    if (e == hipSuccess && (e = hipEventCreate(&ev[1])) != hipSuccess) (void)hipEventDestroy(ev[0]);
    if (e != hipSuccess) {
        ws->timing = timing;
        return hip_fail(e, "hipEventCreate");
    }
    std::vector<float> best(plans.size(), 0.0f);
    int rc = GW_OK;
    for (int pass = -1; pass < 2 && rc == GW_OK; ++pass) {
        for (size_t i = 0; i < plans.size() && rc == GW_OK; ++i) {
            if (pass < 0 && i > 0) break;    // one warm-up call lets the clock settle
            const LnlLayout l = lnl_layout(grid.n_bins, n_det, n_samples, plans[i], flags);
            if ((e = hipEventRecord(ev[0], stream)) != hipSuccess) { rc = hip_fail(e, "hipEventRecord"); break; }
            if ((rc = lnl_enqueue(ws, static_cast<char *>(ws->base), l, plans[i], grid, n_det, geom, data, psd, theta,
                                  n_param, n_samples, lnl_out, mixed, flags, stream)) != GW_OK)
                break;
            float ms = 0.0f;
            if ((e = hipEventRecord(ev[1], stream)) != hipSuccess || (e = hipEventSynchronize(ev[1])) != hipSuccess ||
                (e = hipEventElapsedTime(&ms, ev[0], ev[1])) != hipSuccess) {
                rc = hip_fail(e, "timing a plan");
                break;
            }
            if (pass >= 0 && (pass == 0 || ms < best[i])) best[i] = ms;
        }
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    ws->timing = timing;
    if (rc != GW_OK) return rc;
    const gw::TilePlan def = plan_tiles_on(ws->n_cu, ws->occupancy, grid.n_bins, n_det, n_samples, mixed, form);
    size_t pick = 0, dflt = plans.size();
    for (size_t i = 0; i < plans.size(); ++i) {
        if (best[i] < best[pick]) pick = i;
        if (same_plan(plans[i], def)) dflt = i;
    }
    if (dflt < plans.size() && best[pick] > (1.0f - kTuneMargin) * best[dflt]) pick = dflt;
    ws->single_tuning[tuning_key(grid.n_bins, n_det, n_samples, mixed, form)] = {plans[pick].tile_bins,
                                                                                  plans[pick].rounds};
    return GW_OK;
}

int lnl_one_event(gw_workspace *ws, const gw_grid &grid, int n_det, const gw::DetGeom &geom, const gw_c128 *data,
                  const double *psd, const double *theta, int n_param, int64_t n_samples, double *lnl_out,
                  bool mixed, unsigned flags, hipStream_t stream)
{
    drop_ragged_graph(ws);               // the arena is about to be laid out for one event
    const int form = gw::tile_form(flags);
    if (ws->tune_single && !ws->pinned && !capturing(stream) &&
        (double)grid.n_bins * (double)n_samples >= kTuneMinPairs &&
        ws->single_tuning.find(tuning_key(grid.n_bins, n_det, n_samples, mixed, form)) == ws->single_tuning.end()) {
        if (int rc = tune_single_event(ws, grid, n_det, geom, data, psd, theta, n_param, n_samples, lnl_out, mixed,
                                       flags, stream))
            return rc;
    }
    const gw::TilePlan plan = plan_tiles(ws, grid.n_bins, n_det, n_samples, mixed, form);
    const LnlLayout l = lnl_layout(grid.n_bins, n_det, n_samples, plan, flags);
    if (int rc = ensure_capacity(ws, l.total, stream)) return rc;
    return lnl_enqueue(ws, static_cast<char *>(ws->base), l, plan, grid, n_det, geom, data, psd, theta, n_param,
                       n_samples, lnl_out, mixed, flags, stream);
}

// ------------------------------------------------------------------ allocation-free likelihood
// Device memory of gw_lnl_batch_static: one array per GPU, held from the
// library's load until the process ends.  Host code never passes `scratch`
// itself to a kernel or a copy (in host code the name is a host-side stand-in,
// not a device address); it uses the address hipGetSymbolAddress returns for
// the device that is current.
constexpr size_t kStaticScratchBytes = (size_t)GW_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kStaticMaxDevices = 64;

struct StaticDevice {
    bool ready = false;
    char *ptr = nullptr;                 // device address of `scratch` on this device
    int n_cu = 0;
    OccupancyCache occupancy;
};

std::mutex g_static_mutex;
StaticDevice g_static[kStaticMaxDevices];

// The scratch address and CU count of the current device, looked up once
// per device (with that device current).  Allocates nothing.
int static_device(int device, StaticDevice **out)
{
    if (device < 0 || device >= kStaticMaxDevices) return fail(GW_EINVAL, "device index out of range");
    StaticDevice &d = g_static[device];
    if (!d.ready) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        int n_cu = 0;
        e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device);
        if (e != hipSuccess || n_cu < 1) return hip_fail(e, "hipDeviceGetAttribute(multiprocessor count)");
        d.ptr = static_cast<char *>(ptr);
        d.n_cu = n_cu;
        d.ready = true;
    }
    *out = &d;
    return GW_OK;
}

// ------------------------------------------------------------------ ragged batches
// Host description of one ragged pass: device arrays, their offsets in the
// workspace arena, and the launch record.
struct RaggedPlan {
    std::vector<gw::RaggedEvent> events;
    std::vector<int2> block_map, groups;
    std::vector<gw::WorkItem> items;     // all classes, class by class
    std::vector<int> class_begin;        // first item of each class
    gw::RaggedLaunch launch{};
    size_t off_events = 0, off_block_map = 0, off_groups = 0, off_geoms = 0, off_items = 0, off_counters = 0;
    size_t total = 0;
};

int64_t ragged_pairs(int n_events, const gw_event *events)
{
    int64_t p = 0;
    for (int i = 0; i < n_events; ++i) p += events[i].n_samples * events[i].grid.n_bins;
    return p;
}

// Lays out the workspace for a ragged pass with the given tile shape and
// fills the host arrays; device pointers are relative to `base`.
RaggedPlan ragged_plan(gw_workspace *ws, int n_events, const gw_event *events, const gw_c128 *data,
                       const double *psd, const double *theta, int n_param, double *lnl, bool mixed, unsigned flags,
                       int tile_bins, int64_t chunk_bins, char *base)
{
    const bool direct = (flags & GW_FLAG_DIRECT) != 0, isco = (flags & GW_FLAG_TERM_ISCO) != 0;
    const int form = gw::tile_form(flags);
    RaggedPlan p;
    Carver c;
    p.events.resize(n_events);
    std::vector<std::vector<gw::WorkItem>> by_det(gw::kMaxDet + 1);
    std::vector<int64_t> cost_of;
    for (int e = 0; e < n_events; ++e) {
        const gw_event &ev = events[e];
        gw::RaggedEvent &re = p.events[e];
        std::memset(&re, 0, sizeof(re));
        const int64_t m = ev.grid.n_bins, s = ev.n_samples;
        re.n_bins = m;
        re.n_samples = s;
        re.f_low = ev.grid.f_low;
        re.df = ev.grid.delta_f;
        re.n_det = ev.n_det;
        re.chunk_bins = std::min<int64_t>(chunk_bins, m);
        re.n_chunks = (int)((m + re.chunk_bins - 1) / re.chunk_bins);
        re.prep_blocks = (int)((m + gw::kBlock - 1) / gw::kBlock);
        re.data = reinterpret_cast<const double2 *>(data + ev.data_offset);
        re.psd = psd + ev.data_offset;
        re.theta = theta ? theta + ev.theta_offset * n_param : nullptr;
        re.lnl = lnl ? lnl + ev.theta_offset : nullptr;
        re.tab1 = reinterpret_cast<gw::Tab1 *>(base + c.take(sizeof(gw::Tab1) * m));
        re.tab2 = reinterpret_cast<gw::Tab2 *>(base + c.take(sizeof(gw::Tab2) * m));
        re.dcoef = reinterpret_cast<double2 *>(base + c.take(sizeof(double2) * m * ev.n_det));
        re.edir = direct ? reinterpret_cast<double2 *>(base + c.take(sizeof(double2) * m * ev.n_det)) : nullptr;
        re.vdir = direct ? reinterpret_cast<double *>(base + c.take(sizeof(double) * m * ev.n_det)) : nullptr;
        re.qprefix = isco ? reinterpret_cast<double *>(base + c.take(sizeof(double) * m * ev.n_det)) : nullptr;
        re.qoffsets = isco ? reinterpret_cast<double *>(base + c.take(sizeof(double) * re.prep_blocks * ev.n_det))
                           : nullptr;
        re.rec = reinterpret_cast<double *>(base + c.take(sizeof(double) * gw::record_fields(ev.n_det) *
                                                           std::max<int64_t>(s, 1)));
        re.partials = reinterpret_cast<double2 *>(base + c.take(sizeof(double) * re.n_chunks * s));
        re.prep = reinterpret_cast<double *>(base + c.take(sizeof(double) * gw::kPrepPerDet * ev.n_det *
                                                            re.prep_blocks));
        re.sums = reinterpret_cast<double *>(base + c.take(sizeof(double) * gw::kEventSums));
        for (int b = 0; b < re.prep_blocks; ++b) p.block_map.push_back(make_int2(e, b));
        const int n_groups = (int)((s + gw::kBlock - 1) / gw::kBlock);
        for (int gi = 0; gi < n_groups; ++gi) {
            p.groups.push_back(make_int2(e, gi));
            const int64_t rows = std::min<int64_t>(gw::kBlock, s - (int64_t)gi * gw::kBlock);
            for (int ch = 0; ch < re.n_chunks; ++ch) {
                const int64_t bins = std::min(re.chunk_bins, m - (int64_t)ch * re.chunk_bins);
                // a block's time follows its bins; rows only change how full it is
                (void)rows;
                by_det[ev.n_det].push_back(gw::WorkItem{e, gi, ch, (int)std::min<int64_t>(bins, 0x7fffffff)});
            }
        }
    }
    gw::RaggedLaunch &L = p.launch;
    L.n_events = n_events;
    L.n_prep_blocks = (int)p.block_map.size();
    L.n_groups = (int)p.groups.size();
    L.n_param = n_param;
    L.tile_bins = tile_bins;
    L.mixed = mixed;
    L.flags = flags;
    L.n_classes = 0;
    for (int d = 1; d <= gw::kMaxDet; ++d) {
        auto &v = by_det[d];
        if (v.empty()) continue;
        // largest items first, ties by (event, group, chunk) so the order is reproducible
        std::stable_sort(v.begin(), v.end(), [](const gw::WorkItem &x, const gw::WorkItem &y) {
            return x.bins > y.bins;
        });
        gw::RaggedClass &rc = L.classes[L.n_classes++];
        rc.n_det = d;
        rc.n_items = (int)v.size();
        const int occ = gw::lnl_ragged_blocks_per_cu(d, tile_bins, mixed, form);
        rc.grid = (int)std::min<int64_t>((int64_t)ws->n_cu * occ, (int64_t)v.size());
        p.class_begin.push_back((int)p.items.size());
        p.items.insert(p.items.end(), v.begin(), v.end());
    }
    p.off_events = c.take(sizeof(gw::RaggedEvent) * std::max(n_events, 1));
    p.off_block_map = c.take(sizeof(int2) * std::max<size_t>(p.block_map.size(), 1));
    p.off_groups = c.take(sizeof(int2) * std::max<size_t>(p.groups.size(), 1));
    p.off_geoms = c.take(sizeof(gw::DetGeom) * std::max(n_events, 1));
    p.off_items = c.take(sizeof(gw::WorkItem) * std::max<size_t>(p.items.size(), 1));
    p.off_counters = c.take(sizeof(unsigned) * gw::kMaxDet);
    p.total = c.offset;
    L.events = reinterpret_cast<const gw::RaggedEvent *>(base + p.off_events);
    L.block_map = reinterpret_cast<const int2 *>(base + p.off_block_map);
    L.groups = reinterpret_cast<const int2 *>(base + p.off_groups);
    L.geoms = reinterpret_cast<const gw::DetGeom *>(base + p.off_geoms);
    L.counters = reinterpret_cast<unsigned *>(base + p.off_counters);
    for (int i = 0; i < L.n_classes; ++i) {
        L.classes[i].items = reinterpret_cast<const gw::WorkItem *>(base + p.off_items) + p.class_begin[i];
        L.classes[i].counter = L.counters + i;
    }
    return p;
}

// Plans with the arena's real base, growing it first if needed, and copies
// the host arrays to the device.  Waits for `stream` (the arena may still be
// in use by earlier work there).
int ragged_materialise(gw_workspace *ws, int n_events, const gw_event *events, const std::vector<gw::DetGeom> &geoms,
                       const gw_c128 *data, const double *psd, const double *theta, int n_param, double *lnl,
                       bool mixed, unsigned flags, int tile_bins, int64_t chunk_bins, hipStream_t stream,
                       RaggedPlan *out)
{
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    RaggedPlan sizing = ragged_plan(ws, n_events, events, data, psd, theta, n_param, lnl, mixed, flags, tile_bins,
                                    chunk_bins, nullptr);
    if (int rc = ensure_capacity(ws, sizing.total, stream)) return rc;
    ws->tables_valid = false;            // the ragged layout overwrites the arena
    *out = ragged_plan(ws, n_events, events, data, psd, theta, n_param, lnl, mixed, flags, tile_bins, chunk_bins,
                       static_cast<char *>(ws->base));
    char *base = static_cast<char *>(ws->base);
    struct Copy { size_t off; const void *src; size_t bytes; };
    const Copy copies[] = {
        {out->off_events, out->events.data(), sizeof(gw::RaggedEvent) * out->events.size()},
        {out->off_block_map, out->block_map.data(), sizeof(int2) * out->block_map.size()},
        {out->off_groups, out->groups.data(), sizeof(int2) * out->groups.size()},
        {out->off_geoms, geoms.data(), sizeof(gw::DetGeom) * geoms.size()},
        {out->off_items, out->items.data(), sizeof(gw::WorkItem) * out->items.size()},
    };
    for (const Copy &cp : copies) {
        if (cp.bytes == 0) continue;
        e = hipMemcpy(base + cp.off, cp.src, cp.bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy of the ragged plan");
    }
    return GW_OK;
}

int capture_stream(gw_workspace *ws)
{
    if (ws->capture_stream) return GW_OK;
    hipError_t e = hipStreamCreateWithFlags(&ws->capture_stream, hipStreamNonBlocking);
    return e == hipSuccess ? GW_OK : hip_fail(e, "hipStreamCreateWithFlags");
}

// Times one ragged pass (after one untimed pass) on the workspace's own stream.
int time_ragged(gw_workspace *ws, const RaggedPlan &p, float *ms)
{
    hipEvent_t t0, t1;
    hipError_t e = hipEventCreate(&t0);
    if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    e = hipEventCreate(&t1);
    if (e != hipSuccess) { (void)hipEventDestroy(t0); return hip_fail(e, "hipEventCreate"); }
    int rc = GW_OK;
    if ((e = gw::launch_ragged(p.launch, ws->capture_stream)) != hipSuccess ||
        (e = hipEventRecord(t0, ws->capture_stream)) != hipSuccess ||
        (e = gw::launch_ragged(p.launch, ws->capture_stream)) != hipSuccess ||
        (e = hipEventRecord(t1, ws->capture_stream)) != hipSuccess || (e = hipEventSynchronize(t1)) != hipSuccess ||
        (e = hipEventElapsedTime(ms, t0, t1)) != hipSuccess)
        rc = hip_fail(e, "timing a ragged pass");
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    return rc;
}

// Key of a ragged call: its events, pointers, precision and flags.
std::vector<unsigned char> ragged_key(int n_events, const gw_event *events, const void *data, const void *psd,
                                      const void *theta, int n_param, const void *lnl, bool mixed, unsigned flags)
{
    std::vector<unsigned char> k(sizeof(gw_event) * n_events + 4 * sizeof(void *) + 3 * sizeof(int));
    unsigned char *w = k.data();
    if (n_events) std::memcpy(w, events, sizeof(gw_event) * n_events);
    w += sizeof(gw_event) * n_events;
    const void *ptrs[4] = {data, psd, theta, lnl};
    std::memcpy(w, ptrs, sizeof(ptrs));
    w += sizeof(ptrs);
    const int tail[3] = {n_param, mixed ? 1 : 0, (int)flags};
    std::memcpy(w, tail, sizeof(tail));
    return k;
}

// Tile shapes the autotuner tries: LDS tile of the tile loop, bins per work item.
const int kTuneTiles[] = {256, 512};
const int64_t kTuneChunks[] = {4096, 8192, 16384, 32768};

int ragged_run(gw_workspace *ws, int n_events, const gw_event *events, const std::vector<gw::DetGeom> &geoms,
               const gw_c128 *data, const double *psd, const double *theta, int n_param, double *lnl, bool mixed,
               unsigned flags, hipStream_t stream)
{
    const int form = gw::tile_form(flags);
    int n_active = 0, max_det = 1;
    for (int i = 0; i < n_events; ++i) {
        if (events[i].n_samples > 0) ++n_active;
        max_det = std::max(max_det, events[i].n_det);
    }
    if (n_active == 0) return GW_OK;
    std::vector<gw_event> active;
    active.reserve(n_active);
    for (int i = 0; i < n_events; ++i)
        if (events[i].n_samples > 0) active.push_back(events[i]);
    std::vector<gw::DetGeom> active_geoms;
    for (int i = 0; i < n_events; ++i)
        if (events[i].n_samples > 0) active_geoms.push_back(geoms[i]);
    const int na = (int)active.size();
    const gw_event *ev = active.data();

    std::vector<unsigned char> key = ragged_key(na, ev, data, psd, theta, n_param, lnl, mixed, flags);
    if (ws->ragged_exec && key == ws->ragged_key) {
        hipError_t e = hipGraphLaunch(ws->ragged_exec, stream);
        return e == hipSuccess ? GW_OK : hip_fail(e, "hipGraphLaunch");
    }
    drop_ragged_graph(ws);
    if (int rc = capture_stream(ws)) return rc;
    // the autotuner and the plan upload run outside the caller's stream order
    hipError_t se = hipStreamSynchronize(stream);
    if (se != hipSuccess) return hip_fail(se, "hipStreamSynchronize");

    // tile shape: autotuned once per (detectors, precision and form, size bucket)
    const int64_t pairs = ragged_pairs(na, ev);
    const int bucket = pairs > 0 ? (int)std::floor(std::log2((double)pairs)) : 0;
    const auto tkey = std::make_tuple(max_det, (mixed ? 1 : 0) + 2 * form, bucket);
    auto it = ws->ragged_tuning.find(tkey);
    int tile_bins = 0;
    int64_t chunk_bins = 0;
    RaggedPlan plan;
    if (it == ws->ragged_tuning.end()) {
        float best = 0.0f;
        for (int tb : kTuneTiles) {
            if (gw::lnl_tile_lds_bytes(max_det, tb, form, mixed) > 80 * 1024) continue;
            for (int64_t cb : kTuneChunks) {
                if (int rc = ragged_materialise(ws, na, ev, active_geoms, data, psd, theta, n_param, lnl, mixed, flags,
                                                tb, cb, ws->capture_stream, &plan))
                    return rc;
                float ms = 0.0f;
                if (int rc = time_ragged(ws, plan, &ms)) return rc;
                if (tile_bins == 0 || ms < best) {
                    best = ms;
                    tile_bins = tb;
                    chunk_bins = cb;
                }
            }
        }
        ws->ragged_tuning[tkey] = {tile_bins, chunk_bins};
    } else {
        tile_bins = it->second.first;
        chunk_bins = it->second.second;
    }
    ws->last_tile_bins = tile_bins;
    ws->last_chunk_bins = chunk_bins;
    if (int rc = ragged_materialise(ws, na, ev, active_geoms, data, psd, theta, n_param, lnl, mixed, flags,
                                    tile_bins, chunk_bins, stream, &plan))
        return rc;
    hipError_t e = hipStreamSynchronize(ws->capture_stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");

    // capture the pass on the workspace's stream, replay it on the caller's
    e = hipStreamBeginCapture(ws->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    hipError_t le = gw::launch_ragged(plan.launch, ws->capture_stream);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(ws->capture_stream, &graph);
    if (le != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return hip_fail(le, "launching the ragged pass under capture");
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return hip_fail(e, "hipGraphInstantiate");
    }
    ws->ragged_graph = graph;
    ws->ragged_exec = exec;
    ws->ragged_key = std::move(key);
    e = hipGraphLaunch(exec, stream);
    return e == hipSuccess ? GW_OK : hip_fail(e, "hipGraphLaunch");
}

// dPsi(f) of the relative-binning edge rule, evaluated term by term in a
// fixed order without contraction into fused multiply-adds, so that the same
// arithmetic gives the same edges wherever it runs.
double rb_phase_bound(double f, double f_min, double f_max, double chi)
{
#pragma clang fp contract(off)
    static const double kGamma[5] = {-5.0 / 3.0, -2.0 / 3.0, 1.0, 5.0 / 3.0, 7.0 / 3.0};
    double total = 0.0;
    for (double g : kGamma) {
        const double fstar = g < 0.0 ? f_min : f_max;
        total = total + std::copysign(1.0, g) * std::pow(f / fstar, g);
    }
    return 2.0 * GW_PI_HOST * chi * total;
}

// Level of grid bin k under the edge rule: floor((dPsi(f_k) - dPsi(f_0)) / eps).
double rb_level(const gw_grid &g, int64_t k, double psi0, double f_max, double chi, double eps)
{
#pragma clang fp contract(off)
    const double f = g.f_low + (double)k * g.delta_f;
    return std::floor((rb_phase_bound(f, g.f_low, f_max, chi) - psi0) / eps);
}

int pop_run(gw_workspace *ws, int64_t n_events, int64_t n_per_event, const double *samples, bool prepared,
            int64_t n_hyper, const double *hyper, double *lnl_out, hipStream_t stream)
{
    if (!ws) return fail(GW_EINVAL, "workspace is NULL");
    if (n_events < 1 || n_per_event < 1 || n_hyper < 0) return fail(GW_EINVAL, "bad population sizes");
    if (!samples || (n_hyper > 0 && (!hyper || !lnl_out))) return fail(GW_EINVAL, "NULL population argument");
    if (gw::pop::weight_blocks(n_events, n_per_event) > 0x7fffffffLL || n_hyper > 0x7fffffffLL ||
        n_hyper * n_events / 4 > 0x7fffffffLL)
        return fail(GW_EINVAL, "population batch too large for one launch");
    if (n_hyper == 0) return GW_OK;
    DeviceGuard g(ws->device);
    if (!g.ok) return fail(GW_EDEVICE, "cannot select the workspace device");
    drop_ragged_graph(ws);               // the arena is about to be laid out for the population pass
    if (int rc = ensure_capacity(ws, gw::pop::workspace_bytes(n_events, n_per_event, n_hyper), stream)) return rc;
    ws->tables_valid = false;
    hipEvent_t t_start, t_stop;
    if (int rc = timer_pair(ws, stream, &t_start, &t_stop)) return rc;
    hipError_t e = gw::pop::launch(n_events, n_per_event, samples, prepared, n_hyper, hyper, ws->base, lnl_out,
                                   t_start, t_stop, stream);
    if (e != hipSuccess) return hip_fail(e, "gw_pop_lnl");
    if (t_stop) ++ws->timed;
    return GW_OK;
}

}  // namespace

namespace gw {
int set_error(int code, const std::string &msg) { return fail(code, msg); }

int check_build()
{
    const char *mine = source_hash_api();
    const char *units[] = {source_hash_kernels(), source_hash_flow(), source_hash_mcmc(), source_hash_pop(),
                           source_hash_relbin(), source_hash_waveform()};
    for (const char *u : units)
        if (std::strcmp(u, mine) != 0)
            return fail(GW_EABI, std::string("the library was linked from objects compiled from different sources (") +
                                     mine + " and " + u + "); rebuild it from one source tree");
    return GW_OK;
}
}  // namespace gw

GW_DEFINE_SOURCE_HASH(api)

extern "C" {

int gw_version(void) { return 301; }

const char *gw_source_hash(void) { return gw::source_hash_api(); }

int gw_abi_layout(int64_t *sizes_out, int capacity)
{
    const int64_t v[] = {(int64_t)sizeof(gw_c128), (int64_t)sizeof(gw_grid), (int64_t)sizeof(gw_detector),
                         (int64_t)sizeof(gw_event), (int64_t)offsetof(gw_event, dets), (int64_t)GW_MAX_DET};
    const int n = (int)(sizeof(v) / sizeof(v[0]));
    if (capacity < 0 || (capacity > 0 && !sizes_out)) return fail(GW_EINVAL, "bad output array");
    if (int rc = gw::check_build()) return rc;
    for (int i = 0; i < n && i < capacity; ++i) sizes_out[i] = v[i];
    return n;
}

const char *gw_last_error(void) { return g_last_error.c_str(); }

int gw_workspace_create(gw_workspace **ws, int device)
{
    if (!ws) return fail(GW_EINVAL, "ws is NULL");
    *ws = nullptr;
    if (int rc = gw::check_build()) return rc;
    int dev = device;
    if (dev < 0) {
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    }
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (dev >= count) return fail(GW_EINVAL, "device index out of range");
    auto *w = new gw_workspace();
    w->device = dev;
    e = hipDeviceGetAttribute(&w->n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess || w->n_cu < 1) {
        delete w;
        return hip_fail(e, "hipDeviceGetAttribute(multiprocessor count)");
    }
    *ws = w;
    return GW_OK;
}

int gw_workspace_destroy(gw_workspace *ws)
{
    if (!ws) return GW_OK;
    int rc = GW_OK;
    if (ws->base) {
        DeviceGuard g(ws->device);
        hipError_t e = hipDeviceSynchronize();
        if (e == hipSuccess) e = hipFree(ws->base);
        if (e != hipSuccess) rc = hip_fail(e, "freeing the workspace");
    }
    for (hipEvent_t ev : ws->events) (void)hipEventDestroy(ev);
    drop_ragged_graph(ws);
    if (ws->capture_stream) (void)hipStreamDestroy(ws->capture_stream);
    delete ws;
    return rc;
}

int gw_workspace_set_timing(gw_workspace *ws, int enable)
{
    if (!ws) return fail(GW_EINVAL, "workspace is NULL");
    ws->timing = enable != 0;
    ws->timed = 0;
    return GW_OK;
}

int gw_workspace_kernel_time(gw_workspace *ws, double *total_ms, int64_t *launches)
{
    if (!ws || !total_ms || !launches) return fail(GW_EINVAL, "NULL argument");
    *total_ms = 0.0;
    *launches = ws->timed;
    if (ws->timed == 0) return GW_OK;
    DeviceGuard g(ws->device);
    hipError_t e = hipEventSynchronize(ws->events[2 * ws->timed - 1]);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    double sum = 0.0;
    for (int64_t i = 0; i < ws->timed; ++i) {
        float ms = 0.0f;
        e = hipEventElapsedTime(&ms, ws->events[2 * i], ws->events[2 * i + 1]);
        if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
        sum += ms;
    }
    *total_ms = sum;
    return GW_OK;
}

int gw_workspace_reserve(gw_workspace *ws, int64_t n_bins, int n_det, int64_t n_samples)
{
    if (!ws) return fail(GW_EINVAL, "workspace is NULL");
    if (n_bins < 1 || n_det < 1 || n_det > gw::kMaxDet || n_samples < 0) return fail(GW_EINVAL, "bad reserve sizes");
    DeviceGuard g(ws->device);
    if (!g.ok) return fail(GW_EDEVICE, "cannot select the workspace device");
    // every plan a call within these sizes may run: the current one of each
    // form and precision and every candidate of the autotuner
    const unsigned all_flags = GW_FLAG_DIRECT | GW_FLAG_TERM_ISCO | GW_FLAG_ADD_NORM;
    size_t need = 0;
    for (int form = 0; form < gw::kForms; ++form)
        for (int mixed = 0; mixed < 2; ++mixed) {
            std::vector<gw::TilePlan> plans = tuning_candidates(ws, n_bins, n_det, n_samples, mixed != 0, form);
            plans.push_back(plan_tiles(ws, n_bins, n_det, n_samples, mixed != 0, form));
            for (const gw::TilePlan &p : plans) need = std::max(need, lnl_layout(n_bins, n_det, n_samples, p, all_flags).total);
        }
    size_t wave = align_up(sizeof(gw::Tab1) * n_bins) + align_up(sizeof(gw::Tab2) * n_bins) +
                  align_up(sizeof(double) * gw::record_fields(std::max(n_det, 2)) * std::max<int64_t>(n_samples, 1));
    return ensure_capacity(ws, std::max(need, wave), nullptr);
}

int64_t gw_workspace_bytes(const gw_workspace *ws) { return ws ? (int64_t)ws->capacity : 0; }

int gw_workspace_set_tuning(gw_workspace *ws, int enable)
{
    if (!ws) return fail(GW_EINVAL, "workspace is NULL");
    ws->tune_single = enable > 0;
    if (enable < 0) ws->single_tuning.clear();
    return GW_OK;
}

int gw_lnl_batch(gw_workspace *ws, const gw_grid *grid, int n_det, const gw_detector *dets, const gw_c128 *data,
                 const double *psd, const double *theta, int n_param, int64_t n_samples, double *lnl_out,
                 int precision, unsigned flags, hipStream_t stream)
{
    if (int rc = check_common(ws, grid, 1, n_det, n_param, n_samples)) return rc;
    if (!data || !psd) return fail(GW_EINVAL, "data or psd is NULL");
    if (n_samples > 0 && (!theta || !lnl_out)) return fail(GW_EINVAL, "theta or lnl_out is NULL");
    if (precision != GW_PREC_FP64 && precision != GW_PREC_MIXED) return fail(GW_EINVAL, "unknown precision");
    if (flags & ~kLnlFlags) return fail(GW_EINVAL, "unknown flag bits");
    gw::DetGeom geom;
    if (int rc = check_dets(n_det, dets, n_param, &geom)) return rc;
    if (n_samples == 0) return GW_OK;
    DeviceGuard g(ws->device);
    if (!g.ok) return fail(GW_EDEVICE, "cannot select the workspace device");
    return lnl_one_event(ws, *grid, n_det, geom, data, psd, theta, n_param, n_samples, lnl_out,
                         precision == GW_PREC_MIXED, flags, stream);
}

int64_t gw_lnl_batch_static_capacity(void) { return (int64_t)kStaticScratchBytes; }

int64_t gw_lnl_batch_static_bytes(const gw_grid *grid, int n_det, int64_t n_samples, int precision, unsigned flags)
{
    if (check_grid(grid) != GW_OK) return -1;
    if (n_det < 1 || n_det > gw::kMaxDet || n_samples < 0) return fail(GW_EINVAL, "n_det or n_samples out of range");
    if (precision != GW_PREC_FP64 && precision != GW_PREC_MIXED) return fail(GW_EINVAL, "unknown precision");
    if (flags & ~kLnlFlags) return fail(GW_EINVAL, "unknown flag bits");
    int device = 0;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lock(g_static_mutex);
    StaticDevice *d = nullptr;
    if (int rc = static_device(device, &d)) return rc;
    const gw::TilePlan plan = plan_tiles_on(d->n_cu, d->occupancy, grid->n_bins, n_det, n_samples,
                                            precision == GW_PREC_MIXED, gw::tile_form(flags));
    return (int64_t)lnl_layout(grid->n_bins, n_det, n_samples, plan, flags).total;
}

int gw_lnl_batch_static(const gw_grid *grid, int n_det, const gw_detector *dets, const gw_c128 *data,
                        const double *psd, const double *theta, int n_param, int64_t n_samples, double *lnl_out,
                        int precision, unsigned flags, hipStream_t stream)
{
    if (int rc = check_grid(grid)) return rc;
    if (n_det < 1 || n_det > gw::kMaxDet) return fail(GW_EINVAL, "n_det out of range");
    if (!gw::valid_n_param(n_param)) return fail(GW_EINVAL, "n_param must be 5, 7, 9 or 11");
    if (n_samples < 0) return fail(GW_EINVAL, "n_samples must be >= 0");
    if (!data || !psd) return fail(GW_EINVAL, "data or psd is NULL");
    if (n_samples > 0 && (!theta || !lnl_out)) return fail(GW_EINVAL, "theta or lnl_out is NULL");
    if (precision != GW_PREC_FP64 && precision != GW_PREC_MIXED) return fail(GW_EINVAL, "unknown precision");
    if (flags & ~kLnlFlags) return fail(GW_EINVAL, "unknown flag bits");
    if (int rc = gw::check_build()) return rc;
    gw::DetGeom geom;
    if (int rc = check_dets(n_det, dets, n_param, &geom)) return rc;
    if (n_samples == 0) return GW_OK;
    int device = 0;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    const bool mixed = precision == GW_PREC_MIXED;
    std::lock_guard<std::mutex> lock(g_static_mutex);
    StaticDevice *d = nullptr;
    if (int rc = static_device(device, &d)) return rc;
    const gw::TilePlan plan = plan_tiles_on(d->n_cu, d->occupancy, grid->n_bins, n_det, n_samples, mixed,
                                            gw::tile_form(flags));
    const LnlLayout l = lnl_layout(grid->n_bins, n_det, n_samples, plan, flags);
    if (l.total > kStaticScratchBytes)
        return fail(GW_EINVAL, "gw_lnl_batch_static: this call needs " + std::to_string(l.total) +
                                   " bytes of scratch, more than the library's static " +
                                   std::to_string(kStaticScratchBytes) + "; use gw_lnl_batch with a workspace");
    return lnl_enqueue(nullptr, d->ptr, l, plan, *grid, n_det, geom, data, psd, theta, n_param, n_samples, lnl_out,
                       mixed, flags, stream);
}

int gw_waveform_batch(gw_workspace *ws, const gw_grid *grid, int n_det, const gw_detector *dets,
                      const double *theta, int n_param, int64_t n_samples, gw_c128 *h_out, unsigned flags,
                      hipStream_t stream)
{
    if (int rc = check_common(ws, grid, 0, n_det, n_param, n_samples)) return rc;
    if (n_samples > 0 && (!theta || !h_out)) return fail(GW_EINVAL, "theta or h_out is NULL");
    if (flags & ~(unsigned)GW_FLAG_TERM_ISCO) return fail(GW_EINVAL, "waveform flags: only GW_FLAG_TERM_ISCO");
    gw::DetGeom geom;
    if (n_det > 0) {
        if (int rc = check_dets(n_det, dets, n_param, &geom)) return rc;
    } else {
        std::memset(&geom, 0, sizeof(geom));
    }
    if (n_samples == 0) return GW_OK;
    DeviceGuard g(ws->device);
    if (!g.ok) return fail(GW_EDEVICE, "cannot select the workspace device");
    const bool polar = n_det == 0;
    const int n_out = polar ? 2 : n_det;
    drop_ragged_graph(ws);               // the arena is about to be laid out for the waveform
    Carver c;
    const size_t o1 = c.take(sizeof(gw::Tab1) * grid->n_bins);
    const size_t o2 = c.take(sizeof(gw::Tab2) * grid->n_bins);
    const size_t orec = c.take(sizeof(double) * gw::record_fields(n_out) * n_samples);
    if (int rc = ensure_capacity(ws, c.offset, stream)) return rc;
    auto *tab1 = at<gw::Tab1>(ws, o1);
    auto *tab2 = at<gw::Tab2>(ws, o2);
    auto *rec = at<double>(ws, orec);
    hipError_t e;
    if ((e = bin_tables(ws, *grid, o1, o2, tab1, tab2, stream)) != hipSuccess) return hip_fail(e, "event tables");
    if ((e = gw::launch_sample_prep(*grid, n_samples, n_param, n_out, polar, (flags & GW_FLAG_TERM_ISCO) != 0, geom,
                                    theta, rec, stream)) != hipSuccess)
        return hip_fail(e, "sample prep");
    hipEvent_t t_start, t_stop;
    if (int rc = timer_pair(ws, stream, &t_start, &t_stop)) return rc;
    if (t_start && (e = hipEventRecord(t_start, stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    if ((e = gw::launch_waveform(*grid, n_out, n_samples, tab1, tab2, rec, h_out, stream)) != hipSuccess)
        return hip_fail(e, "waveform");
    return timer_stop(ws, t_stop, stream);
}

int gw_fill_c128(gw_c128 *out, int64_t n, double re, double im, hipStream_t stream)
{
    if (n < 0 || (n > 0 && !out)) return fail(GW_EINVAL, "bad arguments");
    int device = 0, n_cu = 0;
    hipError_t e = hipGetDevice(&device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess || n_cu < 1) return hip_fail(e, "gw_fill_c128: device attributes");
    e = gw::launch_fill_c128(n, re, im, out, n_cu, stream);
    return e == hipSuccess ? GW_OK : hip_fail(e, "gw_fill_c128");
}

int gw_lnl_ragged(gw_workspace *ws, int n_events, const gw_event *events, const gw_c128 *data_packed,
                  const double *psd_packed, const double *theta_packed, int n_param, double *lnl_out_packed,
                  int precision, unsigned flags, hipStream_t stream)
{
    if (!ws) return fail(GW_EINVAL, "workspace is NULL");
    if (n_events < 0) return fail(GW_EINVAL, "n_events must be >= 0");
    if (n_events > 0 && !events) return fail(GW_EINVAL, "events is NULL");
    if (n_events > 0 && (!data_packed || !psd_packed)) return fail(GW_EINVAL, "data or psd is NULL");
    if (precision != GW_PREC_FP64 && precision != GW_PREC_MIXED) return fail(GW_EINVAL, "unknown precision");
    if (flags & ~kLnlFlags) return fail(GW_EINVAL, "unknown flag bits");
    if (!gw::valid_n_param(n_param)) return fail(GW_EINVAL, "n_param must be 5, 7, 9 or 11");
    std::vector<gw::DetGeom> geoms(n_events);
    for (int i = 0; i < n_events; ++i) {
        const gw_event &ev = events[i];
        if (int rc = check_common(ws, &ev.grid, 1, ev.n_det, n_param, ev.n_samples)) return rc;
        if (ev.data_offset < 0 || ev.theta_offset < 0) return fail(GW_EINVAL, "negative event offset");
        if (ev.n_samples > 0 && (!theta_packed || !lnl_out_packed)) return fail(GW_EINVAL, "theta or lnl_out is NULL");
        if (ev.n_samples > (int64_t)0x7fffffff * gw::kBlock) return fail(GW_EINVAL, "too many samples in one event");
        if (int rc = check_dets(ev.n_det, ev.dets, n_param, &geoms[i])) return rc;
    }
    DeviceGuard g(ws->device);
    if (!g.ok) return fail(GW_EDEVICE, "cannot select the workspace device");
    return ragged_run(ws, n_events, events, geoms, data_packed, psd_packed, theta_packed, n_param, lnl_out_packed,
                      precision == GW_PREC_MIXED, flags, stream);
}

int gw_pop_lnl(gw_workspace *ws, int64_t n_events, int64_t n_per_event, const double *samples, int64_t n_hyper,
               const double *hyper, double *lnl_out, hipStream_t stream)
{
    return pop_run(ws, n_events, n_per_event, samples, false, n_hyper, hyper, lnl_out, stream);
}

int gw_pop_prepare(int64_t n_events, int64_t n_per_event, const double *samples, double *prepared_out,
                   hipStream_t stream)
{
    if (n_events < 1 || n_per_event < 1) return fail(GW_EINVAL, "bad population sizes");
    if (!samples || !prepared_out) return fail(GW_EINVAL, "NULL population argument");
    if ((n_events * n_per_event + 255) / 256 > 0x7fffffffLL) return fail(GW_EINVAL, "too many samples");
    hipError_t e = gw::pop::prepare(n_events, n_per_event, samples, prepared_out, stream);
    return e == hipSuccess ? GW_OK : hip_fail(e, "gw_pop_prepare");
}

int gw_pop_lnl_prepared(gw_workspace *ws, int64_t n_events, int64_t n_per_event, const double *prepared,
                        int64_t n_hyper, const double *hyper, double *lnl_out, hipStream_t stream)
{
    return pop_run(ws, n_events, n_per_event, prepared, true, n_hyper, hyper, lnl_out, stream);
}

int gw_rb_edges(const gw_grid *grid, double chi, double eps, int64_t *edges_out, int64_t capacity, int64_t *n_edges)
{
    if (!n_edges) return fail(GW_EINVAL, "n_edges is NULL");
    *n_edges = 0;
    if (int rc = check_grid(grid)) return rc;
    if (grid->n_bins < 2) return fail(GW_EINVAL, "relative binning needs n_bins >= 2");
    if (!(chi > 0.0) || !std::isfinite(chi) || !(eps > 0.0) || !std::isfinite(eps))
        return fail(GW_EINVAL, "chi and eps must be finite and > 0");
    const gw_grid g = *grid;
    const int64_t last = g.n_bins - 1;
    double f_max;
    {
#pragma clang fp contract(off)
        f_max = g.f_low + (double)last * g.delta_f;
    }
    const double psi0 = rb_phase_bound(g.f_low, g.f_low, f_max, chi);
    // dPsi rises with f, so the level never falls: each next edge is the first
    // bin whose level exceeds the current edge's, found by bisection.
    const double top = rb_level(g, last, psi0, f_max, chi, eps);
    std::vector<int64_t> out{0};
    int64_t k = 0;
    double level = rb_level(g, 0, psi0, f_max, chi, eps);
    while (level < top) {
        int64_t lo = k + 1, hi = last;
        while (lo < hi) {
            const int64_t mid = lo + (hi - lo) / 2;
            if (rb_level(g, mid, psi0, f_max, chi, eps) > level) hi = mid;
            else lo = mid + 1;
        }
        k = lo;
        level = rb_level(g, k, psi0, f_max, chi, eps);
        out.push_back(k);
    }
    if (out.back() != last) out.push_back(last);
    *n_edges = (int64_t)out.size();
    if (!edges_out) return GW_OK;
    if (capacity < *n_edges) return fail(GW_EINVAL, "edges_out too small");
    std::memcpy(edges_out, out.data(), sizeof(int64_t) * out.size());
    return GW_OK;
}

int gw_rb_create(gw_workspace *ws, const gw_grid *grid, int n_det, const gw_detector *dets, const gw_c128 *data,
                 const double *psd, const double *theta0, int n_param, const int64_t *edges, int64_t n_edges,
                 unsigned flags, gw_relbin **rb, hipStream_t stream)
{
    if (!rb) return fail(GW_EINVAL, "rb is NULL");
    *rb = nullptr;
    if (int rc = check_common(ws, grid, 1, n_det, n_param, 1)) return rc;
    if (!data || !psd || !theta0 || !edges) return fail(GW_EINVAL, "NULL argument");
    if (grid->n_bins < 2) return fail(GW_EINVAL, "relative binning needs n_bins >= 2");
    if (flags & ~(unsigned)GW_FLAG_ADD_NORM) return fail(GW_EINVAL, "relative binning flags: only GW_FLAG_ADD_NORM");
    if (n_edges < 2 || edges[0] != 0 || edges[n_edges - 1] != grid->n_bins - 1)
        return fail(GW_EINVAL, "edges must run from 0 to n_bins - 1");
    for (int64_t i = 1; i < n_edges; ++i)
        if (edges[i] <= edges[i - 1]) return fail(GW_EINVAL, "edges must rise strictly");
    if (n_edges - 1 > 0x7fffffffLL) return fail(GW_EINVAL, "too many bins");
    for (int i = 0; i < n_param; ++i)
        if (!std::isfinite(theta0[i])) return fail(GW_EINVAL, "theta0 is not finite");
    if (!(theta0[0] > 0.0) || !(theta0[1] > 0.0 && theta0[1] <= 1.0) || !(theta0[2] > 0.0) ||
        (gw::param_has_spins(n_param) &&
         (std::fabs(theta0[n_param - 2]) > 1.0 || std::fabs(theta0[n_param - 1]) > 1.0)))
        return fail(GW_EINVAL, "theta0 is outside the domain");
    gw::DetGeom geom;
    if (int rc = check_dets(n_det, dets, n_param, &geom)) return rc;
    DeviceGuard g(ws->device);
    if (!g.ok) return fail(GW_EDEVICE, "cannot select the workspace device");
    drop_ragged_graph(ws);               // the arena is about to be laid out for the preparation
    const int64_t n_rb = n_edges - 1;
    const int n_fields = gw::record_fields(n_det);
    Carver w;
    const size_t o1 = w.take(sizeof(gw::Tab1) * grid->n_bins);
    const size_t o2 = w.take(sizeof(gw::Tab2) * grid->n_bins);
    const size_t oth = w.take(sizeof(double) * n_param);
    if (int rc = ensure_capacity(ws, w.offset, stream)) return rc;
    Carver c;
    const size_t h_idx = c.take(sizeof(int64_t) * n_edges);
    const size_t h_edges = c.take(sizeof(gw::rb::RbEdge) * n_edges);
    const size_t h_coef = c.take(sizeof(gw::rb::RbCoef) * n_edges * n_det);
    const size_t h_ends = c.take(sizeof(gw::rb::RbEnds) * n_edges * n_det);
    const size_t h_raw = c.take(sizeof(double) * gw::rb::kRawPerDet * n_rb * n_det);
    const size_t h_dd = c.take(sizeof(double) * 2 * n_rb);
    const size_t h_tot = c.take(sizeof(double) * 2);
    const size_t h_fid = c.take(sizeof(double) * n_fields);
    auto *h = new gw_relbin();
    h->device = ws->device;
    h->grid = *grid;
    h->n_det = n_det;
    h->n_param = n_param;
    h->flags = flags;
    h->n_rb = n_rb;
    h->geom = geom;
    hipError_t e = hipMalloc(&h->mem, c.offset);
    if (e != hipSuccess) {
        delete h;
        return fail(GW_ENOMEM, "relative-binning hipMalloc failed");
    }
    char *base = static_cast<char *>(h->mem);
    h->edge_idx = reinterpret_cast<int64_t *>(base + h_idx);
    h->edges = reinterpret_cast<gw::rb::RbEdge *>(base + h_edges);
    h->coef = reinterpret_cast<gw::rb::RbCoef *>(base + h_coef);
    h->ends = reinterpret_cast<gw::rb::RbEnds *>(base + h_ends);
    h->raw = reinterpret_cast<double *>(base + h_raw);
    h->bin_dd = reinterpret_cast<double *>(base + h_dd);
    h->totals = reinterpret_cast<double *>(base + h_tot);
    h->fid = reinterpret_cast<double *>(base + h_fid);
    auto *tab1 = at<gw::Tab1>(ws, o1);
    auto *tab2 = at<gw::Tab2>(ws, o2);
    auto *th = at<double>(ws, oth);
    const char *where = nullptr;
    if ((e = hipMemcpyAsync(h->edge_idx, edges, sizeof(int64_t) * n_edges, hipMemcpyHostToDevice, stream)) !=
        hipSuccess)
        where = "copying the edges";
    else if ((e = hipMemcpyAsync(th, theta0, sizeof(double) * n_param, hipMemcpyHostToDevice, stream)) != hipSuccess)
        where = "copying theta0";
    else if ((e = bin_tables(ws, *grid, o1, o2, tab1, tab2, stream)) != hipSuccess)
        where = "event tables";
    else if ((e = gw::launch_sample_prep(*grid, 1, n_param, n_det, false, false, geom, th, h->fid, stream)) !=
             hipSuccess)
        where = "fiducial record";
    else if ((e = gw::rb::launch_edges(*grid, n_edges, h->edge_idx, h->edges, stream)) != hipSuccess)
        where = "edge tables";
    else if ((e = gw::rb::launch_summary(*grid, n_det, n_rb, h->edge_idx, tab1, tab2, h->fid, data, psd, h->edges,
                                         h->raw, h->coef, h->ends, h->bin_dd, h->totals, stream)) != hipSuccess)
        where = "summary data";
    else if ((e = hipStreamSynchronize(stream)) != hipSuccess)
        where = "waiting for the preparation";
    if (where) {
        (void)hipFree(h->mem);
        delete h;
        return hip_fail(e, where);
    }
    std::vector<double> rec(n_fields);
    if ((e = hipMemcpy(rec.data(), h->fid, sizeof(double) * n_fields, hipMemcpyDeviceToHost)) != hipSuccess) {
        (void)hipFree(h->mem);
        delete h;
        return hip_fail(e, "reading the fiducial record");
    }
    for (int d = 0; d < n_det; ++d) {
        const double pr = rec[gw::kRecDet + gw::kRecFieldsPerDet * d];
        const double pi = rec[gw::kRecDet + gw::kRecFieldsPerDet * d + 1];
        if (!(pr * pr + pi * pi > 0.0) || !std::isfinite(pr * pr + pi * pi)) {
            (void)hipFree(h->mem);
            delete h;
            return fail(GW_EINVAL, "the fiducial template vanishes on a detector");
        }
    }
    *rb = h;
    return GW_OK;
}

int gw_rb_destroy(gw_relbin *rb)
{
    if (!rb) return GW_OK;
    DeviceGuard g(rb->device);
    hipError_t e = hipFree(rb->mem);
    delete rb;
    return e == hipSuccess ? GW_OK : hip_fail(e, "hipFree");
}

int gw_rb_shape(const gw_relbin *rb, int64_t *n_rb, int *n_det)
{
    if (!rb || !n_rb || !n_det) return fail(GW_EINVAL, "NULL argument");
    *n_rb = rb->n_rb;
    *n_det = rb->n_det;
    return GW_OK;
}

int gw_rb_summary(const gw_relbin *rb, double *raw_out, double *totals_out)
{
    if (!rb) return fail(GW_EINVAL, "rb is NULL");
    DeviceGuard g(rb->device);
    if (!g.ok) return fail(GW_EDEVICE, "cannot select the handle's device");
    hipError_t e;
    if (raw_out &&
        (e = hipMemcpy(raw_out, rb->raw, sizeof(double) * gw::rb::kRawPerDet * rb->n_rb * rb->n_det,
                       hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "copying the summary data");
    if (totals_out && (e = hipMemcpy(totals_out, rb->totals, sizeof(double) * 2, hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "copying the totals");
    return GW_OK;
}

int gw_rb_lnl(gw_workspace *ws, const gw_relbin *rb, const double *theta, int64_t n_samples, double *lnl_out,
              int precision, hipStream_t stream)
{
    if (!ws || !rb) return fail(GW_EINVAL, "workspace or handle is NULL");
    if (n_samples < 0) return fail(GW_EINVAL, "n_samples must be >= 0");
    if (precision != GW_PREC_FP64 && precision != GW_PREC_MIXED) return fail(GW_EINVAL, "unknown precision");
    const bool mixed = precision == GW_PREC_MIXED;
    if (ws->device != rb->device) return fail(GW_EINVAL, "workspace and handle are on different devices");
    if (n_samples == 0) return GW_OK;
    if (!theta || !lnl_out) return fail(GW_EINVAL, "theta or lnl_out is NULL");
    DeviceGuard g(ws->device);
    if (!g.ok) return fail(GW_EDEVICE, "cannot select the workspace device");
    const int n_chunks = gw::rb::lnl_chunks(n_samples, rb->n_rb, rb->n_det, mixed, ws->n_cu);
    if ((n_samples + gw::kBlock - 1) / gw::kBlock * n_chunks > 0x7fffffffLL)
        return fail(GW_EINVAL, "too many samples for one launch");
    drop_ragged_graph(ws);               // the arena is about to be laid out for this pass
    Carver c;
    const size_t orec = c.take(sizeof(double) * gw::record_fields(rb->n_det) * n_samples);
    const size_t opart = c.take(sizeof(double) * n_chunks * n_samples);
    if (int rc = ensure_capacity(ws, c.offset, stream)) return rc;
    ws->tables_valid = false;
    auto *rec = at<double>(ws, orec);
    auto *part = at<double>(ws, opart);
    hipError_t e;
    if ((e = gw::launch_sample_prep(rb->grid, n_samples, rb->n_param, rb->n_det, false, false, rb->geom, theta, rec,
                                    stream)) != hipSuccess)
        return hip_fail(e, "sample prep");
    hipEvent_t t_start, t_stop;
    if (int rc = timer_pair(ws, stream, &t_start, &t_stop)) return rc;
    if ((e = gw::rb::launch_lnl(rb->n_det, mixed, n_samples, rb->n_rb, n_chunks, rb->edges, rb->coef, rb->ends,
                                rb->fid, rec, part, t_start, t_stop, stream)) != hipSuccess)
        return hip_fail(e, "relative-binning pass");
    if (t_stop) ++ws->timed;
    if ((e = gw::rb::launch_finalize(n_samples, n_chunks, part, rec, rb->totals, (rb->flags & GW_FLAG_ADD_NORM) != 0,
                                     lnl_out, stream)) != hipSuccess)
        return hip_fail(e, "relative-binning finalize");
    return GW_OK;
}

int gw_lnl_plan(gw_workspace *ws, int64_t n_bins, int n_det, int64_t n_samples, int precision, unsigned flags,
                int *tile_bins, int *n_chunks, int *rounds)
{
    if (!ws) return fail(GW_EINVAL, "workspace is NULL");
    if (n_bins < 1 || n_det < 1 || n_det > gw::kMaxDet || n_samples < 1) return fail(GW_EINVAL, "bad plan sizes");
    if (precision != GW_PREC_FP64 && precision != GW_PREC_MIXED) return fail(GW_EINVAL, "unknown precision");
    if (flags & ~kLnlFlags) return fail(GW_EINVAL, "unknown flag bits");
    DeviceGuard g(ws->device);
    if (!g.ok) return fail(GW_EDEVICE, "cannot select the workspace device");
    const gw::TilePlan p = plan_tiles(ws, n_bins, n_det, n_samples, precision == GW_PREC_MIXED, gw::tile_form(flags));
    if (tile_bins) *tile_bins = p.tile_bins;
    if (n_chunks) *n_chunks = p.n_chunks;
    if (rounds) *rounds = p.rounds;
    return GW_OK;
}

int gw_workspace_set_plan(gw_workspace *ws, int64_t n_bins, int n_det, int64_t n_samples, int precision,
                          unsigned flags, int tile_bins, int rounds)
{
    if (!ws) return fail(GW_EINVAL, "workspace is NULL");
    if (n_bins < 1 || n_det < 1 || n_det > gw::kMaxDet || n_samples < 1) return fail(GW_EINVAL, "bad plan sizes");
    if (precision != GW_PREC_FP64 && precision != GW_PREC_MIXED) return fail(GW_EINVAL, "unknown precision");
    if (flags & ~kLnlFlags) return fail(GW_EINVAL, "unknown flag bits");
    const bool mixed = precision == GW_PREC_MIXED;
    const int form = gw::tile_form(flags);
    const auto key = tuning_key(n_bins, n_det, n_samples, mixed, form);
    if (tile_bins == 0 && rounds == 0) {
        ws->single_tuning.erase(key);
        return GW_OK;
    }
    if (tile_bins < 64 || tile_bins % 64 != 0 || tile_bins > gw::tile_bins_for(n_det, form, mixed))
        return fail(GW_EINVAL, "tile_bins must be a multiple of 64 within the LDS budget");
    if (rounds < 0 || rounds > 16) return fail(GW_EINVAL, "rounds must be within 0..16");
    ws->single_tuning[key] = {tile_bins, rounds};
    return GW_OK;
}

int gw_ragged_tuning(const gw_workspace *ws, int *tile_bins, int64_t *chunk_bins)
{
    if (!ws || !tile_bins || !chunk_bins) return fail(GW_EINVAL, "NULL argument");
    *tile_bins = ws->last_tile_bins;
    *chunk_bins = ws->last_chunk_bins;
    return GW_OK;
}

}  // extern "C"
