// C ABI of the batched TaylorF2 likelihood library (see include/gwlnl.h).
// Validates arguments on the host, sizes the library-owned workspace, plans
// the launch and enqueues the kernels of gw_kernels.hip on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "gw_internal.h"
#include "gwlnl.h"

struct gw_workspace {
    int device = 0;
    int n_cu = 0;
    int blocks_per_cu[gw::kMaxDet + 1] = {0};   // tile-kernel occupancy by detector count (0 = unknown)
    void *base = nullptr;
    size_t capacity = 0;
    bool timing = false;
    std::vector<hipEvent_t> events;   // start/stop pairs of the hot kernel
    int64_t timed = 0;                 // pairs recorded since timing was enabled
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

int ensure_capacity(gw_workspace *ws, size_t bytes)
{
    if (bytes <= ws->capacity) return GW_OK;
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
    if (n_param == 5) return GW_OK;          // optimally oriented: geometry unused
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

int tile_bins_for(int n_det)
{
    const size_t budget = 40 * 1024;   // bytes of LDS per block: several blocks per CU fit in 160 KB
    int t = 512;
    while (t > 64 && gw::lnl_tile_lds_bytes(n_det, t) > budget) t /= 2;
    return t;
}

gw::TilePlan plan_tiles(gw_workspace *ws, int64_t n_bins, int n_det, int64_t n_samples)
{
    gw::TilePlan p;
    p.tile_bins = tile_bins_for(n_det);
    p.n_groups = (int)((n_samples + gw::kBlock - 1) / gw::kBlock);
    if (ws->blocks_per_cu[n_det] == 0) ws->blocks_per_cu[n_det] = gw::lnl_tile_blocks_per_cu(n_det, p.tile_bins);
    const int64_t target = (int64_t)ws->n_cu * ws->blocks_per_cu[n_det];
    int64_t chunks = (target + p.n_groups - 1) / p.n_groups;
    const int64_t max_chunks = std::max<int64_t>(1, n_bins / 64);     // at least 64 bins per chunk
    chunks = std::max<int64_t>(1, std::min(chunks, max_chunks));
    p.chunk_bins = (n_bins + chunks - 1) / chunks;
    p.n_chunks = (int)((n_bins + p.chunk_bins - 1) / p.chunk_bins);
    return p;
}

struct LnlLayout {
    size_t tab1, tab2, dcoef, prep_partials, event_sums, records, partials, total;
    int prep_blocks;
};

LnlLayout lnl_layout(int64_t n_bins, int n_det, int64_t n_samples, const gw::TilePlan &plan)
{
    LnlLayout l;
    Carver c;
    l.prep_blocks = (int)std::min<int64_t>(1024, (n_bins + gw::kBlock - 1) / gw::kBlock);
    l.tab1 = c.take(sizeof(gw::Tab1) * n_bins);
    l.tab2 = c.take(sizeof(gw::Tab2) * n_bins);
    l.dcoef = c.take(sizeof(double2) * n_bins * n_det);
    l.prep_partials = c.take(sizeof(double) * 2 * n_det * l.prep_blocks);
    l.event_sums = c.take(sizeof(double) * (1 + gw::kMaxDet));
    l.records = c.take(sizeof(double) * gw::record_fields(n_det) * std::max<int64_t>(n_samples, 1));
    l.partials = c.take(sizeof(double2) * (size_t)plan.n_chunks * n_samples * n_det);
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
    if (n_param != 5 && n_param != 9) return fail(GW_EINVAL, "n_param must be 5 or 9");
    if (n_samples < 0) return fail(GW_EINVAL, "n_samples must be >= 0");
    return GW_OK;
}

int lnl_one_event(gw_workspace *ws, const gw_grid &grid, int n_det, const gw::DetGeom &geom, const gw_c128 *data,
                  const double *psd, const double *theta, int n_param, int64_t n_samples, double *lnl_out,
                  hipStream_t stream)
{
    const gw::TilePlan plan = plan_tiles(ws, grid.n_bins, n_det, n_samples);
    const LnlLayout l = lnl_layout(grid.n_bins, n_det, n_samples, plan);
    if (int rc = ensure_capacity(ws, l.total)) return rc;
    auto *tab1 = at<gw::Tab1>(ws, l.tab1);
    auto *tab2 = at<gw::Tab2>(ws, l.tab2);
    auto *dcoef = at<double2>(ws, l.dcoef);
    auto *prep = at<double>(ws, l.prep_partials);
    auto *sums = at<double>(ws, l.event_sums);
    auto *rec = at<double>(ws, l.records);
    auto *part = at<double2>(ws, l.partials);
    hipError_t e;
    if ((e = gw::launch_event_tables(grid, tab1, tab2, stream)) != hipSuccess) return hip_fail(e, "event tables");
    if ((e = gw::launch_event_data(grid, n_det, data, psd, tab2, dcoef, prep, l.prep_blocks, sums, stream)) != hipSuccess)
        return hip_fail(e, "event data");
    if ((e = gw::launch_sample_prep(n_samples, n_param, n_det, false, geom, theta, rec, stream)) != hipSuccess)
        return hip_fail(e, "sample prep");
    hipEvent_t stop_event = nullptr;
    if (ws->timing) {
        if ((size_t)(2 * ws->timed + 2) > ws->events.size()) {
            for (int i = 0; i < 2; ++i) {
                hipEvent_t ev;
                if ((e = hipEventCreate(&ev)) != hipSuccess) return hip_fail(e, "hipEventCreate");
                ws->events.push_back(ev);
            }
        }
        if ((e = hipEventRecord(ws->events[2 * ws->timed], stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
        stop_event = ws->events[2 * ws->timed + 1];
    }
    if ((e = gw::launch_lnl_tiles(grid, n_det, n_samples, plan, tab1, dcoef, rec, part, stream)) != hipSuccess)
        return hip_fail(e, "lnl tiles");
    if (stop_event) {
        if ((e = hipEventRecord(stop_event, stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
        ++ws->timed;
    }
    if ((e = gw::launch_lnl_finalize(n_samples, n_det, plan, part, rec, sums, lnl_out, stream)) != hipSuccess)
        return hip_fail(e, "lnl finalize");
    return GW_OK;
}

}  // namespace

extern "C" {

int gw_version(void) { return 100; }

const char *gw_last_error(void) { return g_last_error.c_str(); }

int gw_workspace_create(gw_workspace **ws, int device)
{
    if (!ws) return fail(GW_EINVAL, "ws is NULL");
    *ws = nullptr;
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
    const gw::TilePlan plan = plan_tiles(ws, n_bins, n_det, n_samples);
    const LnlLayout l = lnl_layout(n_bins, n_det, n_samples, plan);
    size_t wave = align_up(sizeof(gw::Tab1) * n_bins) + align_up(sizeof(gw::Tab2) * n_bins) +
                  align_up(sizeof(double) * gw::record_fields(std::max(n_det, 2)) * std::max<int64_t>(n_samples, 1));
    return ensure_capacity(ws, std::max(l.total, wave));
}

int64_t gw_workspace_bytes(const gw_workspace *ws) { return ws ? (int64_t)ws->capacity : 0; }

int gw_lnl_batch(gw_workspace *ws, const gw_grid *grid, int n_det, const gw_detector *dets, const gw_c128 *data,
                 const double *psd, const double *theta, int n_param, int64_t n_samples, double *lnl_out,
                 int precision, unsigned flags, hipStream_t stream)
{
    if (int rc = check_common(ws, grid, 1, n_det, n_param, n_samples)) return rc;
    if (!data || !psd) return fail(GW_EINVAL, "data or psd is NULL");
    if (n_samples > 0 && (!theta || !lnl_out)) return fail(GW_EINVAL, "theta or lnl_out is NULL");
    if (precision != GW_PREC_FP64 && precision != GW_PREC_MIXED) return fail(GW_EINVAL, "unknown precision");
    if (precision == GW_PREC_MIXED) return fail(GW_EUNSUPPORTED, "mixed precision is not built yet");
    if (flags != 0) return fail(GW_EINVAL, "flags must be 0");
    gw::DetGeom geom;
    if (int rc = check_dets(n_det, dets, n_param, &geom)) return rc;
    if (n_samples == 0) return GW_OK;
    DeviceGuard g(ws->device);
    if (!g.ok) return fail(GW_EDEVICE, "cannot select the workspace device");
    return lnl_one_event(ws, *grid, n_det, geom, data, psd, theta, n_param, n_samples, lnl_out, stream);
}

int gw_waveform_batch(gw_workspace *ws, const gw_grid *grid, int n_det, const gw_detector *dets,
                      const double *theta, int n_param, int64_t n_samples, gw_c128 *h_out, hipStream_t stream)
{
    if (int rc = check_common(ws, grid, 0, n_det, n_param, n_samples)) return rc;
    if (n_samples > 0 && (!theta || !h_out)) return fail(GW_EINVAL, "theta or h_out is NULL");
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
    Carver c;
    const size_t o1 = c.take(sizeof(gw::Tab1) * grid->n_bins);
    const size_t o2 = c.take(sizeof(gw::Tab2) * grid->n_bins);
    const size_t orec = c.take(sizeof(double) * gw::record_fields(n_out) * n_samples);
    if (int rc = ensure_capacity(ws, c.offset)) return rc;
    auto *tab1 = at<gw::Tab1>(ws, o1);
    auto *tab2 = at<gw::Tab2>(ws, o2);
    auto *rec = at<double>(ws, orec);
    hipError_t e;
    if ((e = gw::launch_event_tables(*grid, tab1, tab2, stream)) != hipSuccess) return hip_fail(e, "event tables");
    if ((e = gw::launch_sample_prep(n_samples, n_param, n_out, polar, geom, theta, rec, stream)) != hipSuccess)
        return hip_fail(e, "sample prep");
    if ((e = gw::launch_waveform(*grid, n_out, n_samples, tab1, tab2, rec, h_out, stream)) != hipSuccess)
        return hip_fail(e, "waveform");
    return GW_OK;
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
    if (precision == GW_PREC_MIXED) return fail(GW_EUNSUPPORTED, "mixed precision is not built yet");
    if (flags != 0) return fail(GW_EINVAL, "flags must be 0");
    for (int i = 0; i < n_events; ++i) {
        const gw_event &ev = events[i];
        if (int rc = check_common(ws, &ev.grid, 1, ev.n_det, n_param, ev.n_samples)) return rc;
        if (ev.data_offset < 0 || ev.theta_offset < 0) return fail(GW_EINVAL, "negative event offset");
        if (ev.n_samples > 0 && (!theta_packed || !lnl_out_packed)) return fail(GW_EINVAL, "theta or lnl_out is NULL");
        gw::DetGeom geom;
        if (int rc = check_dets(ev.n_det, ev.dets, n_param, &geom)) return rc;
    }
    DeviceGuard g(ws->device);
    if (!g.ok) return fail(GW_EDEVICE, "cannot select the workspace device");
    for (int i = 0; i < n_events; ++i) {
        const gw_event &ev = events[i];
        if (ev.n_samples == 0) continue;
        gw::DetGeom geom;
        check_dets(ev.n_det, ev.dets, n_param, &geom);
        if (int rc = lnl_one_event(ws, ev.grid, ev.n_det, geom, data_packed + ev.data_offset,
                                   psd_packed + ev.data_offset, theta_packed + ev.theta_offset * n_param, n_param,
                                   ev.n_samples, lnl_out_packed + ev.theta_offset, stream))
            return rc;
    }
    return GW_OK;
}

}  // extern "C"
