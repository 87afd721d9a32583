// Internal interface between the C ABI (gw_api.hip) and the kernels
// (gw_kernels.hip).  Not installed; not part of the ABI.
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

#include "gwlnl.h"

namespace gw {

constexpr int kBlock = 256;          // threads per block of every kernel; one sample per thread
constexpr int kMaxDet = GW_MAX_DET;
constexpr int kQueues = 8;      // work queues of the single-event tile kernel, one per XCD

// Per-sample record, stored field-major ([field][n_samples]) so that a block
// reads it with coalesced loads.  The ten phase coefficients are those of
// Phi_0 / (2 pi), the phase at detector 0 in turns:
//   Phi_0/(2 pi) = u^-5 (c0 + u^2 (c2 + u (c3 + u (c4 + u ((c5 + c5l L)
//                      + u ((c6 + c6l L) + u (c7 + u c8)))))))
// with u = f^(1/3), L = ln u, and c8 = tau_0 (the time shift f tau_0 in turns
// written as u^8 u^-5).
enum RecordField : int {
    kRecC8 = 0, kRecC7, kRecC6, kRecC6L, kRecC5, kRecC5L, kRecC4, kRecC3, kRecC2, kRecC0,
    kRecStatus,                 // 0 evaluate, 1 out of domain (-inf), 2 non-finite (NaN)
    kRecKcut,                   // last bin of the template: n_bins - 1, or below with the ISCO end (-1: none)
    kRecDet,                    // then per output channel d: P re, P im, delta (s)
    kRecFieldsPerDet = 3,
};
constexpr int record_fields(int n_out) { return kRecDet + kRecFieldsPerDet * n_out; }

// Parameter rows: 5 (optimally oriented), 7 (the same with aligned spins
// chi1, chi2 appended), 9 (with sky position, polarisation, inclination),
// 11 (9 with chi1, chi2 appended).
__host__ __device__ constexpr bool valid_n_param(int n) { return n == 5 || n == 7 || n == 9 || n == 11; }
__host__ __device__ constexpr bool param_has_sky(int n) { return n == 9 || n == 11; }
__host__ __device__ constexpr bool param_has_spins(int n) { return n == 7 || n == 11; }
constexpr int kMaxParam = 11;

// Per event-preparation block and detector: sums of |d|^2/S, a^2/S, ln(2 pi S)
// over the block's 256 consecutive bins.  The event sums hold the same three
// quantities summed over all bins, at [kPrepPerDet d + 0, 1, 2].
constexpr int kPrepPerDet = 3;
constexpr int kEventSums = kPrepPerDet * kMaxDet;

// What the tile kernel accumulates.
enum TileForm : int {
    kFormSplit = 0,       // Z_det = sum_k D_det,k e^{-i Phi_det,k} over every bin
    kFormSplitIsco = 1,   // the same over each sample's bins k <= K_s (template end)
    kFormDirect = 2,      // sum_det sum_k a_k^2/S |d/a - P e^{-i Phi}|^2, zero template above K_s
};
constexpr int kForms = 3;
inline int tile_form(unsigned flags)
{
    return (flags & GW_FLAG_DIRECT) ? kFormDirect : (flags & GW_FLAG_TERM_ISCO) ? kFormSplitIsco : kFormSplit;
}

// Detector geometry passed by value to the sample-preparation kernel.
struct DetGeom {
    double tensor[kMaxDet][9];
    double vertex[kMaxDet][3];
};

// Tables per bin: tab1 = (u, u^2, u^-5, ln u), tab2 = (f, f^-7/6).
struct Tab1 { double u, u2, um5, lnu; };
struct Tab2 { double f, amp; };

// One event of a ragged batch as the device sees it (pointers into the
// caller's packed arrays and into the workspace).
struct RaggedEvent {
    int64_t n_bins, n_samples;
    double f_low, df;
    int n_det, n_chunks, prep_blocks, pad_;
    int64_t chunk_bins;
    const double2 *data;
    const double *psd;
    const double *theta;
    double *lnl;
    Tab1 *tab1;
    Tab2 *tab2;
    double2 *dcoef;
    double2 *edir;        // direct form: d / a per detector and bin
    double *vdir;         // direct form: a^2 / S per detector and bin
    double *qprefix;      // ISCO end: prefix sums of a^2 / S per detector
    double *qoffsets;     // ISCO end: a^2 / S totals of the preceding 256-bin blocks [n_det][prep_blocks]
    double *rec;
    double2 *partials;    // double [chunk][n_samples]: the chunk totals the finalize adds
    double *prep;
    double *sums;
};

// One unit of the persistent ragged kernel: one sample group of one event
// against one chunk of its bins.
struct WorkItem {
    int event, group, chunk, bins;   // bins: the item's cost, used to sort the list
};

// The persistent kernel of one detector count within a ragged batch.
struct RaggedClass {
    int n_det;
    int n_items;
    int grid;                 // persistent blocks
    const WorkItem *items;    // device, sorted by decreasing cost
    unsigned *counter;        // device
};

// Everything one ragged pass launches (device pointers into the workspace).
struct RaggedLaunch {
    const RaggedEvent *events;
    int n_events;
    const int2 *block_map;    // per prep block: (event, block within event)
    int n_prep_blocks;
    const int2 *groups;       // per sample group: (event, group within event)
    int n_groups;
    const DetGeom *geoms;     // per event
    int n_param;
    unsigned *counters;       // kMaxDet counters
    RaggedClass classes[kMaxDet];
    int n_classes;
    int tile_bins;
    bool mixed;
    unsigned flags;           // GW_FLAG_* of the call
};

// Launch plan of the tile kernel for one event.
struct TilePlan {
    int n_groups;        // ceil(n_samples / kBlock)
    int n_chunks;        // bin chunks per sample group
    int64_t chunk_bins;  // bins per chunk (the last may be shorter); static launch only
    int tile_bins;       // bins staged in LDS at a time
    int rounds;          // 0: one block per (group, chunk); >= 1: work queue, chunks in this many rounds
    int blocks;          // blocks launched
};

// Sizes of workspace sections for one event.
struct EventSizes {
    int64_t n_bins;
    int n_det;
    int64_t n_samples;
    int prep_blocks;
};

// Device buffers of one event's preparation (workspace sections).
struct EventBuffers {
    Tab1 *tab1;
    Tab2 *tab2;
    double2 *dcoef;       // [n_det][n_bins]
    double2 *edir;        // [n_det][n_bins], direct form only
    double *vdir;         // [n_det][n_bins], direct form only
    double *qprefix;      // [n_det][n_bins], ISCO end only
    double *qoffsets;     // [n_det][prep_blocks], ISCO end only
    double *prep;         // [prep_blocks][kPrepPerDet * n_det]
    int prep_blocks;      // ceil(n_bins / kBlock)
    double *sums;         // [kEventSums]
    int64_t *k_limit;     // ISCO end: 1 + the largest K_s of the batch
    unsigned *queue;      // [kQueues] work-queue counters of the tile kernel (zeroed by the event sums), or null
};

// ---- launchers (gw_kernels.hip); all enqueue on `stream` and return the launch status ----
hipError_t launch_event_tables(const gw_grid &grid, Tab1 *tab1, Tab2 *tab2, hipStream_t stream);

// The sample records of a likelihood call (one detector channel each), when
// launch_event_data prepares them in its own launch; isco: K_s from the
// template end (else n_bins - 1).
struct SamplePrep {
    int64_t n_samples;
    int n_param;
    int isco;
    DetGeom geom;
    const double *theta;
    double *records;
};

// D, the event sums and, as `flags` ask, the direct-form tables and the
// prefix sums of a^2/S; with sp, the sample records too, in the launch that
// computes D (the two share no data).
hipError_t launch_event_data(const gw_grid &grid, int n_det, const gw_c128 *data, const double *psd,
                             const EventBuffers &eb, unsigned flags, const SamplePrep *sp, hipStream_t stream);

// Per-sample records; with isco, K_s from the template end (else n_bins - 1).
hipError_t launch_sample_prep(const gw_grid &grid, int64_t n_samples, int n_param, int n_out, bool polarisations,
                              bool isco, const DetGeom &geom, const double *theta, double *records,
                              hipStream_t stream);

// *k_limit = 1 + max over samples of K_s (ISCO end).
hipError_t launch_isco_limit(int64_t n_samples, const double *records, int64_t *k_limit, hipStream_t stream);

hipError_t launch_lnl_tiles(const gw_grid &grid, int n_det, int64_t n_samples, const TilePlan &plan, bool mixed,
                            int form, const EventBuffers &eb, const double *records, double2 *partials,
                            hipStream_t stream);

hipError_t launch_lnl_finalize(const gw_grid &grid, int64_t n_samples, int n_det, const TilePlan &plan,
                               const double2 *partials, const double *records, const EventBuffers &eb,
                               unsigned flags, double *lnl_out, hipStream_t stream);

hipError_t launch_waveform(const gw_grid &grid, int n_out, int64_t n_samples, const Tab1 *tab1, const Tab2 *tab2,
                           const double *records, gw_c128 *h_out, hipStream_t stream);
hipError_t launch_fill_c128(int64_t n, double re, double im, gw_c128 *out, int n_cu, hipStream_t stream);

hipError_t launch_ragged(const RaggedLaunch &r, hipStream_t stream);
int lnl_ragged_blocks_per_cu(int n_det, int tile_bins, bool mixed, int form);

// Population likelihood (gw_pop.hip): workspace bytes, weight-kernel blocks
// and the launch of the hyper-parameter, weights and finalize kernels.
namespace pop {
size_t workspace_bytes(int64_t n_events, int64_t n_per, int64_t n_hyper);
int64_t weight_blocks(int64_t n_events, int64_t n_per);
hipError_t prepare(int64_t n_events, int64_t n_per, const double *samples, double *prepared, hipStream_t stream);
// samples raw [7][N][n] or, with `prepared`, from prepare [8][N][n];
// t_start / t_stop (either may be null): events recorded around the weights kernel.
hipError_t launch(int64_t n_events, int64_t n_per, const double *samples, bool prepared, int64_t n_hyper,
                  const double *hyper, void *work, double *lnl, hipEvent_t t_start, hipEvent_t t_stop,
                  hipStream_t stream);
}  // namespace pop

// Relative binning (gw_relbin.hip).  Device layout of one prepared event:
//   edges  [B + 1] RbEdge           the tables of every edge frequency;
//   coef   [B + 1][n_det] RbCoef    what the per-sample loop needs at each edge;
//   ends   [B + 1][n_det] RbEnds    the one-sided coefficients of chunk ends;
//   raw    [B][n_det][7]            A0 re, A0 im, A1 re, A1 im, B0, B1, B2;
//   bin_dd [B][2]                   per bin: sum w |d|^2 and sum ln(2 pi S) over detectors;
//   totals [2]                      <d, d> and sum ln(2 pi S) over the whole grid;
//   fid    record of the fiducial sample (record_fields(n_det) doubles).
namespace rb {
struct RbEdge {
    Tab1 t1;
    double f;
    double pad[3];
};
// Bin b, with edges f_lo < f_hi, w = f_hi - f_lo and the ratio r_lo, r_hi at
// its edges, adds to <d, h> - <h, h>/2
//   Re(Llo conj r_lo) + Re(Lhi conj r_hi) + alpha |r_lo|^2 + beta |r_hi|^2 + X Re(r_lo conj r_hi),
//   Llo = A0/2 - A1/w, Lhi = A0/2 + A1/w,  alpha = -B0/8 - B2/(2w^2) + B1/(2w),
//   beta = -B0/8 - B2/(2w^2) - B1/(2w),    X = -B0/4 + B2/w^2
// (the linear model r = r0 + r1 (f - fm) written in the two edge values).
// At an edge e inside a chunk the two bins that meet there are combined:
// L = Lhi(e-1) + Llo(e), q = beta(e-1) + alpha(e); xb = X(e-1) is the cross
// term of the bin that ends at e.  (lr, li, xb first: the per-sample pass
// reads those three at every edge, q only through its prefix sums.)
struct RbCoef {
    double lr, li, xb, q;
};
// The same per bin side: hi = the bin that ends at e (e - 1), lo = the bin that
// starts there (e); used at the last and first edge of a chunk.  qcum = the
// sum of RbCoef::q over the edges below e (an exclusive prefix sum).
struct RbEnds {
    double hi_r, hi_i, hi_q, lo_r, lo_i, lo_q, qcum, pad1;
};
constexpr int kRawPerDet = 7;

hipError_t launch_edges(const gw_grid &grid, int64_t n_edges, const int64_t *edge_idx, RbEdge *edges,
                        hipStream_t stream);
// Summary data, per-bin totals and then the edge coefficients.
hipError_t launch_summary(const gw_grid &grid, int n_det, int64_t n_rb, const int64_t *edge_idx, const Tab1 *tab1,
                          const Tab2 *tab2, const double *fid, const gw_c128 *data, const double *psd,
                          const RbEdge *edges, double *raw, RbCoef *coef, RbEnds *ends, double *bin_dd,
                          double *totals, hipStream_t stream);
// Chunks of bins per sample group for n_samples samples over n_rb bins.
int lnl_chunks(int64_t n_samples, int64_t n_rb, int n_det, bool mixed, int n_cu);
// mixed: FP32 hardware phasor of the ratio (the phase and every sum FP64).
hipError_t launch_lnl(int n_det, bool mixed, int64_t n_samples, int64_t n_rb, int n_chunks, const RbEdge *edges,
                      const RbCoef *coef, const RbEnds *ends, const double *fid, const double *rec,
                      double *partials, hipEvent_t t_start, hipEvent_t t_stop, hipStream_t stream);
hipError_t launch_finalize(int64_t n_samples, int n_chunks, const double *partials, const double *rec,
                           const double *totals, bool add_norm, double *lnl_out, hipStream_t stream);
}  // namespace rb

// LDS bytes of the tile kernel and its occupancy.
size_t lnl_tile_lds_bytes(int n_det, int tile_bins, int form, bool mixed);
int lnl_tile_blocks_per_cu(int n_det, int tile_bins, bool mixed, int form);

}  // namespace gw
