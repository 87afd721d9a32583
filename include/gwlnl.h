/*
 * gwlnl.h -- C ABI of the MI355X (gfx950) batched TaylorF2 likelihood library.
 *
 * The library evaluates, for a batch of compact-binary parameter samples, the
 * Gaussian single-event log-likelihood of Talbot, Smith, Thrane & Poole 2019
 * (arXiv:1904.02863), Eq. (cbclike) in Sec. III:
 *
 *     lnL(theta) = -(2/T) sum_det sum_bins |d - h(theta)|^2 / S,   T = 1/delta_f,
 *
 * without the theta-independent factor prod (2 pi S)^-1 of that equation
 * (GW_FLAG_ADD_NORM adds its logarithm).
 * h is the response of each detector to a non-spinning TaylorF2 inspiral
 * (Sec. II: Newtonian amplitude, 3.5PN phase), projected with the detector's
 * antenna pattern and shifted by exp(-2 pi i f dt_det), the time translation
 * described after Eq. (cbclike).
 *
 * Conventions
 *  - Frequency bins: f_k = f_low + k * delta_f, k = 0 .. n_bins-1.  Every bin
 *    is evaluated (no upper cut-off) unless GW_FLAG_TERM_ISCO is given.
 *  - Complex arrays are interleaved (re, im) double pairs, the layout of
 *    torch.complex128 / numpy complex128.
 *  - theta is row-major [n_samples][n_param], n_param 5, 7, 9 or 11, columns
 *      0 Mc   chirp mass, solar masses      1 q     m2/m1 in (0, 1]
 *      2 dL   luminosity distance, Mpc      3 phic  coalescence phase, rad
 *      4 tc   coalescence time at the geocentre relative to the segment, s
 *      5 ra   right ascension, rad (Greenwich sidereal time taken as 0)
 *      6 dec  declination, rad              7 psi   polarisation angle, rad
 *      8 iota inclination, rad
 *    With n_param 5 or 7 the source is optimally oriented (F+ = 1, Fx = 0,
 *    iota = 0, no delay) and the detector geometry is not used.  With
 *    n_param 7 or 11 the last two columns are the dimensionless spins chi1
 *    (of the heavier body m1) and chi2, along the orbital angular momentum,
 *    in [-1, 1].
 *  - h_plus = A (1 + cos^2 iota)/2 e^{-i Psi}, h_cross = -i A cos iota e^{-i Psi},
 *    A = sqrt(5/24) pi^(-2/3) Mc^(5/6) f^(-7/6) / dL (geometric units),
 *    Psi = 2 pi f tc - phic - pi/4 + 3/(128 eta v^5) sum_k (phi_k + phi_k^l ln v) v^k,
 *    v = (pi M f)^(1/3), coefficients of Buonanno et al. 2009, Eq. (3.18).
 *    Rows with spins add the aligned-spin terms to phi_k: spin-orbit at 1.5,
 *    2.5 (as phi_5 (1 + 3 ln v)), 3 and 3.5PN, spin-spin at 2PN with the
 *    black-hole quadrupole-monopole term (Kidder 1995; Poisson 1998;
 *    Blanchet 2014; Bohe et al. 2013); the amplitude stays Newtonian.
 *    Response h_det = (F+ h_plus + Fx h_cross) e^{-2 pi i f dt_det},
 *    F = D : e with the polarisation tensors of the sky basis, dt_det = -n.r/c.
 *  - Per-sample domain: any non-finite parameter gives lnL = NaN; Mc <= 0,
 *    q outside (0, 1], dL <= 0 or |chi| > 1 give lnL = -infinity.  These are
 *    not errors.
 *
 * Calls and ownership
 *  - Every pointer marked "device" is a device pointer (e.g. a PyTorch tensor's
 *    data_ptr()); the caller owns it and the library never frees it.  Pointers
 *    marked "host" are read during the call only.
 *  - Computing calls are asynchronous and ordered on `stream` (0 = the null
 *    stream); they return once the work is enqueued.  Results are valid after
 *    the stream has reached that point.
 *  - The workspace is library-owned device memory (the reusable pre-allocated
 *    buffer of Sec. II).  A call grows it when it is too small (hipMalloc);
 *    after gw_workspace_reserve covers a shape, calls of that shape allocate
 *    nothing.  One workspace must not be used by two calls at once (calls on
 *    different streams with the same workspace race).
 *  - Graph capture: gw_lnl_batch, gw_waveform_batch, gw_pop_lnl(_prepared)
 *    and gw_rb_lnl may be captured into a HIP graph on `stream`.  The graph
 *    holds every kernel that fills what it reads (the bin tables included),
 *    so calls of other shapes on the same workspace between its replays do
 *    not change its results; but it keeps pointing at the workspace's device
 *    memory.  A call under capture therefore never grows the workspace (it
 *    returns GW_EINVAL when the workspace is too small: reserve it first),
 *    and once a call has been captured the workspace is pinned: any later
 *    call that would grow it returns GW_EINVAL (use another workspace).
 *    Destroying the workspace while a graph captured from it lives leaves the
 *    graph pointing at freed memory.  Calls under capture record no
 *    timing events (gw_workspace_set_timing).
 *
 * Errors
 *  - Every function returns GW_OK (0) or a negative code; gw_last_error()
 *    returns a thread-local message about the last failing call.  Structural
 *    problems are reported synchronously and enqueue nothing: null pointers,
 *    n_bins < 1, delta_f <= 0 or non-finite, f_low <= 0 or non-finite,
 *    n_det outside 1..8, n_param not 5, 7, 9 or 11, n_samples < 0.
 *  - A PSD value that is <= 0 or non-finite cannot be seen without waiting
 *    for the device: the call then writes NaN to every lnL of that call.
 */
#ifndef GWLNL_H
#define GWLNL_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GW_MAX_DET 8

typedef struct { double re, im; } gw_c128;

/* The frequency grid of one segment: bins f_low + k delta_f, delta_f = 1/T. */
typedef struct {
    double f_low;     /* Hz, > 0 */
    double delta_f;   /* Hz, > 0 */
    int64_t n_bins;   /* M >= 1 */
} gw_grid;

/* One detector, Earth-fixed: tensor D (row-major 3x3, symmetric) and vertex
 * position r in metres from the geocentre. */
typedef struct {
    double tensor[9];
    double vertex[3];
} gw_detector;

typedef struct gw_workspace gw_workspace;

enum {
    GW_OK = 0,
    GW_EINVAL = -1,        /* invalid argument */
    GW_ENOMEM = -2,        /* device allocation failed */
    GW_EDEVICE = -3,       /* a HIP runtime call failed */
    GW_EUNSUPPORTED = -4,  /* valid request the library does not implement */
    GW_EABI = -5           /* the library's objects come from different builds (see gw_abi_layout) */
};

enum {
    GW_PREC_FP64 = 0,      /* every step in FP64 */
    GW_PREC_MIXED = 1      /* FP64 phase, reduction and sums; FP32 hardware phasor */
};

/* Options of the likelihood and waveform calls (bitwise or). */
enum {
    /* Accumulate the literal residual sum of Eq. (cbclike),
     * sum_det sum_k |d - h|^2 / S, for every (sample, bin, detector), instead of
     * the default split form -<d,d>/2 + sum_det [Re <d,h> - <h,h>/2] (an exact
     * identity that needs no per-bin template magnitude).  Same value up to
     * rounding; slower.  Likelihood calls only. */
    GW_FLAG_DIRECT = 1u,
    /* End every template at the gravitational-wave frequency of the
     * Schwarzschild innermost stable circular orbit of its total mass M,
     * f_isco = c^3 / (6^(3/2) pi G M): h = 0 on bins with f_k > f_isco.
     * The paper prints no cut-off (Sec. II names TaylorF2 only); this is the
     * usual end of an inspiral template.  Likelihood and waveform calls. */
    GW_FLAG_TERM_ISCO = 2u,
    /* Add the logarithm of the prefactor prod 1/(2 pi S) of Eq. (cbclike),
     * -sum_det sum_k ln(2 pi S_det,k), to every lnL.  Likelihood calls only. */
    GW_FLAG_ADD_NORM = 4u
};

/* Create a workspace bound to HIP device `device` (the current device when
 * device < 0).  *ws receives the handle.  Allocates no device memory yet. */
int gw_workspace_create(gw_workspace **ws, int device);

/* Free a workspace and its device memory.  Waits for the device first.
 * NULL is accepted and ignored. */
int gw_workspace_destroy(gw_workspace *ws);

/* Size the workspace for events of up to n_bins bins and n_det detectors and
 * batches of up to n_samples samples, so that later calls within these sizes
 * allocate nothing (under the default plans, the plans already tuned and any
 * plan the autotuner may pick; a plan set with gw_workspace_set_plan may need
 * more). */
int gw_workspace_reserve(gw_workspace *ws, int64_t n_bins, int n_det, int64_t n_samples);

/* Bytes of device memory the workspace currently holds. */
int64_t gw_workspace_bytes(const gw_workspace *ws);

/* Plan autotuning of gw_lnl_batch on this workspace.  While it is on (the
 * default), the first call of a size class (detector count, precision,
 * template end, floor(log2 n_bins), floor(log2 n_samples)) with at least 2^24
 * (sample, bin) pairs times the call under each candidate plan (the largest
 * LDS tile and half of it; 0, 4, 6 or 8 work-queue rounds, 0 only with the
 * ISCO end), writing lnl_out once per candidate and waiting for the stream,
 * and later calls of the class use the fastest (the default plan unless the
 * fastest beats it by 3%, so that plans of equal speed do not flip with
 * timing noise from one process to the next).  Calls under stream capture
 * and on a workspace that has been captured are never tuned; they use a
 * class's tuned plan when there is one, else the default.
 *   enable  1: on; 0: off (tuned plans are kept and still used);
 *           -1: off, and the tuned plans are forgotten (the default plans
 *           are used again).
 * Returns GW_OK or GW_EINVAL (ws NULL). */
int gw_workspace_set_tuning(gw_workspace *ws, int enable);

/* Measurement support.  While timing is enabled (enable != 0), every
 * gw_lnl_batch, gw_waveform_batch, gw_pop_lnl(_prepared) and gw_rb_lnl call
 * made with this workspace records a pair of HIP events on its own stream around its
 * hot kernel: the tile kernel that forms Z for every sample, bin and
 * detector; the kernel that writes the templates; the kernel that forms the
 * population weights; the per-sample relative-binning kernel.  Enabling (or disabling) clears earlier records. */
int gw_workspace_set_timing(gw_workspace *ws, int enable);

/* Sum of the recorded hot-kernel durations in milliseconds and the number of
 * launches recorded since timing was enabled.  Waits for the last recorded
 * event. */
int gw_workspace_kernel_time(gw_workspace *ws, double *total_ms, int64_t *launches);

/*
 * gw_waveform_batch -- the template of Sec. II for every sample.
 *   grid      host, the frequency grid.
 *   n_det     number of detectors (1..8), or 0 for the two polarisations.
 *   dets      host [n_det] detectors; ignored (may be NULL) when n_det == 0 or
 *             n_param == 5.
 *   theta     device [n_samples][n_param] doubles.
 *   h_out     device [n_samples][max(n_det,2 if n_det==0)][n_bins] complex:
 *             the detector responses h_det, or (h_plus, h_cross) when n_det == 0.
 *             Rows of out-of-domain or non-finite samples are NaN.
 *   flags     0 or GW_FLAG_TERM_ISCO; any other bit is GW_EINVAL.
 */
int gw_waveform_batch(gw_workspace *ws, const gw_grid *grid, int n_det, const gw_detector *dets,
                      const double *theta, int n_param, int64_t n_samples,
                      gw_c128 *h_out, unsigned flags, hipStream_t stream);

/* out[i] = re + i im for i < n (device complex array): a plain store stream
 * with the store pattern of gw_waveform_batch, e.g. to clear a template
 * buffer; it is also the write ceiling that call is measured against. */
int gw_fill_c128(gw_c128 *out, int64_t n, double re, double im, hipStream_t stream);

/*
 * gw_lnl_batch -- Eq. (cbclike) for every sample of one event.
 *   grid      host, the frequency grid shared by all detectors.
 *   n_det     detectors 1..8;  dets host [n_det] (ignored when n_param == 5).
 *   data      device [n_det][n_bins] complex, frequency-domain strain d~.
 *   psd       device [n_det][n_bins] doubles, one-sided PSD S(f) (1/Hz).
 *   theta     device [n_samples][n_param].
 *   lnl_out   device [n_samples] doubles.
 *   precision GW_PREC_FP64 or GW_PREC_MIXED.
 *   flags     any combination of GW_FLAG_DIRECT, GW_FLAG_TERM_ISCO and
 *             GW_FLAG_ADD_NORM; any other bit is GW_EINVAL.
 */
int gw_lnl_batch(gw_workspace *ws, const gw_grid *grid, int n_det, const gw_detector *dets,
                 const gw_c128 *data, const double *psd,
                 const double *theta, int n_param, int64_t n_samples,
                 double *lnl_out, int precision, unsigned flags, hipStream_t stream);

/*
 * gw_lnl_batch_static -- gw_lnl_batch without a workspace, allocating nothing.
 * For callers that cannot allocate device memory during a call: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Arguments, results and kernels are those of gw_lnl_batch; it always runs
 * the default plan, so its values equal bit for bit those of gw_lnl_batch on
 * a workspace with plan autotuning off (gw_workspace_set_tuning), and those
 * of a tuned plan to the rounding of FP64 sums taken in another order.  Its
 * intermediate buffers live in one static device array of
 * GW_STATIC_SCRATCH_BYTES per GPU, which the library holds on every GPU it
 * runs on until the process ends.  The call uses the array of the current
 * device.  Every call on a GPU shares that array: two calls that overlap on
 * one GPU (different streams, or host threads without ordering) race and
 * give wrong results; calls ordered on one stream are safe.  A call whose
 * buffers exceed the array (gw_lnl_batch_static_bytes > GW_STATIC_SCRATCH_BYTES)
 * returns GW_EINVAL and enqueues nothing; 64 MiB covers, for example, 3
 * detectors x 259,585 bins x 4096 samples.  No bin tables are kept between
 * calls, so each call costs one more short pass over the bins than a
 * repeated gw_lnl_batch on a workspace.
 */
#define GW_STATIC_SCRATCH_BYTES (64ll << 20)
int gw_lnl_batch_static(const gw_grid *grid, int n_det, const gw_detector *dets,
                        const gw_c128 *data, const double *psd,
                        const double *theta, int n_param, int64_t n_samples,
                        double *lnl_out, int precision, unsigned flags, hipStream_t stream);

/* Bytes of the static array a gw_lnl_batch_static call of this shape on the
 * current device needs (a negative error code for bad arguments), and the
 * array's size. */
int64_t gw_lnl_batch_static_bytes(const gw_grid *grid, int n_det, int64_t n_samples, int precision, unsigned flags);
int64_t gw_lnl_batch_static_capacity(void);

/* One event of a ragged batch: its own grid, detectors, and rows. */
typedef struct {
    gw_grid grid;
    int n_det;
    gw_detector dets[GW_MAX_DET];
    int64_t data_offset;    /* element offset of this event's [n_det][n_bins] block in data/psd */
    int64_t theta_offset;   /* first row of this event in theta and lnl_out */
    int64_t n_samples;      /* rows of this event */
} gw_event;

/*
 * gw_lnl_ragged -- Eq. (cbclike) for many events of different durations
 * (Sec. III: different signals have different numbers of bins), each with its
 * own samples, in one persistent launch.  The pass (event preparation, sample
 * preparation, the persistent kernel per detector count, final reduction) is
 * captured once in a HIP graph and replayed while the events, pointers and
 * precision stay the same; any other call on the workspace, or a change of
 * those, rebuilds it (waiting for `stream`).  Events with n_samples == 0 are
 * skipped.
 *   events          host [n_events].
 *   data_packed     device complex, event e at data_offset_e, [n_det_e][n_bins_e].
 *   psd_packed      device doubles, same offsets as data_packed.
 *   theta_packed    device [sum n_samples][n_param]; event e uses rows
 *                   theta_offset_e .. theta_offset_e + n_samples_e - 1.
 *   lnl_out_packed  device, one double per row of theta_packed that an event uses.
 *   precision, flags  as for gw_lnl_batch, applied to every event.
 */
int gw_lnl_ragged(gw_workspace *ws, int n_events, const gw_event *events,
                  const gw_c128 *data_packed, const double *psd_packed,
                  const double *theta_packed, int n_param,
                  double *lnl_out_packed, int precision, unsigned flags, hipStream_t stream);

/*
 * gw_pop_lnl -- the recycled population likelihood of Eq. (poplike), Sec. IV:
 *     ln L(Lambda) = sum_i ln[ (1/n) sum_j p(theta_ij | Lambda) / p(theta_ij | 0) ]
 * for each of n_hyper hyper-parameter points, over n posterior samples of
 * each of n_events events, without the rate and selection factors
 * R^N e^{-R VT(Lambda)} (the paper leaves VT out of its timings).
 * The population model (named, not printed, in Sec. IV): primary mass a
 * power law m1^-alpha plus a Gaussian peak N(mu_m, sigma_m), mixed with
 * weight lam, on [m_min, m_max]; q = m2/m1 a power law q^beta on
 * [m_min/m1, 1]; spin magnitudes a1, a2 Beta(alpha_chi, beta_chi); spin tilt
 * cosines (1 - xi)/4 + xi N_T(c1; 1, sigma_1) N_T(c2; 1, sigma_2) on
 * [-1, 1]^2 (N_T a Gaussian truncated to [-1, 1]).  Every factor is
 * normalised in closed form.
 *   samples  device, field-major [7][n_events][n]: m1 (solar masses), q, a1,
 *            a2, cos t1, cos t2, and ln p(theta | 0), the log density of the
 *            prior the samples were drawn under.  A sample outside the
 *            supports (q not in (0, 1], a or cos t outside their ranges,
 *            non-finite ln prior) has weight 0.
 *   hyper    device [n_hyper][12]: alpha, beta, m_min, m_max, lam, mu_m,
 *            sigma_m, alpha_chi, beta_chi, xi, sigma_1, sigma_2.
 *   lnl_out  device [n_hyper].  A point outside its domain (m_min >= m_max or
 *            <= 0, a width <= 0, lam or xi outside [0, 1], alpha_chi or
 *            beta_chi <= 0) gives -infinity; a non-finite one NaN; an event
 *            whose samples all have weight 0 gives -infinity.
 * Uses the workspace (a call with other shapes relays it out).
 */
int gw_pop_lnl(gw_workspace *ws, int64_t n_events, int64_t n_per_event, const double *samples, int64_t n_hyper,
               const double *hyper, double *lnl_out, hipStream_t stream);

/* The recycled likelihood reuses the same posterior samples for every
 * Lambda, so the per-sample logarithms can be taken once:
 * gw_pop_prepare writes prepared_out (device, caller-owned, [8][n_events][n]
 * doubles: m1, ln m1, ln q, ln a1 + ln a2, ln(1 - a1) + ln(1 - a2),
 * cos t1 - 1, cos t2 - 1, ln p(theta | 0); m1 = -1 marks a sample outside
 * the supports), and gw_pop_lnl_prepared takes that array in place of
 * `samples`, with results identical to gw_pop_lnl on the raw samples. */
int gw_pop_prepare(int64_t n_events, int64_t n_per_event, const double *samples, double *prepared_out,
                   hipStream_t stream);
int gw_pop_lnl_prepared(gw_workspace *ws, int64_t n_events, int64_t n_per_event, const double *prepared,
                        int64_t n_hyper, const double *hyper, double *lnl_out, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Relative binning: Eq. (cbclike) from about 10^3 frequencies.
 *
 * Secs. I and V name relative binning (Zackay, Dai & Venumadhav 2018,
 * arXiv:1806.08792) as the other route to long signals.  Around a fiducial
 * template h0 (parameters theta0) the ratio r = h(theta) / h0 is smooth in
 * frequency, so the grid is cut into B bins by edges e_0 = 0 < ... < e_B =
 * n_bins - 1 (bin b holds grid bins e_b .. e_{b+1} - 1, the last bin also
 * e_B), r is taken as linear in each bin between its values at the two
 * edges, and a sample needs the template only at the B + 1 edge frequencies
 * plus summary data formed once per event (w = 4 delta_f / S, fm the bin
 * centre, r0 and r1 the ratio's value at fm and its slope):
 *   A0 = sum w d conj(h0),  A1 = sum w d conj(h0) (f - fm),
 *   B0 = sum w |h0|^2,      B1 = sum w |h0|^2 (f - fm),  B2 = sum w |h0|^2 (f - fm)^2,
 *   lnL = Re sum [A0 conj(r0) + A1 conj(r1)]
 *         - 1/2 sum [B0 |r0|^2 + 2 B1 Re(r0 conj(r1)) + B2 |r1|^2] - <d,d>/2.
 * The |r1|^2 B2 term, which Zackay et al. drop, is kept: the estimate is then
 * exact where r is linear in every bin (an edge at every grid bin) and at
 * theta0.  Elsewhere it approximates gw_lnl_batch with an error that falls as
 * the bins narrow.  Templates are never ended at f_isco here.
 */

/* Bin edges by the phase-bound rule of Zackay et al. (their Sec. III):
 *   dPsi(f) = 2 pi chi sum_i sgn(g_i) (f / f*_i)^g_i,  g = (-5/3, -2/3, 1, 5/3, 7/3),
 *   f*_i = f_min for g_i < 0 and f_max otherwise (first and last grid frequency);
 * edges at grid bin 0, at every bin k where floor((dPsi(f_k) - dPsi(f_0)) / eps)
 * steps up, and at n_bins - 1.  Host computation; no device is used.
 *   grid       host; n_bins >= 2.
 *   chi, eps   finite and > 0.
 *   edges_out  host [capacity] int64, or NULL to ask for the count only.
 *   n_edges    receives the number of edges (B + 1).
 * Returns GW_EINVAL when edges_out is not NULL and capacity < *n_edges
 * (*n_edges is set all the same). */
int gw_rb_edges(const gw_grid *grid, double chi, double eps, int64_t *edges_out, int64_t capacity,
                int64_t *n_edges);

typedef struct gw_relbin gw_relbin;

/* Prepare one event: the edge tables, the summary data of every detector and
 * bin, <d,d> and sum ln(2 pi S).  Synchronous: returns once the work it
 * enqueued on `stream` has finished, so data and psd may be released then.
 *   ws       workspace; the handle lives on its device and the call uses its
 *            arena for the grid tables.
 *   grid, n_det, dets, data, psd  as for gw_lnl_batch, with n_bins >= 2.
 *   theta0   host [n_param]: the fiducial parameters.  They must be in the
 *            domain (finite, Mc > 0, q in (0, 1], d_L > 0, |chi| <= 1) and give a non-zero
 *            response on every detector, else GW_EINVAL.
 *   n_param  5, 7, 9 or 11; rows passed to gw_rb_lnl use the same layout.
 *   edges    host [n_edges], n_edges >= 2, strictly increasing from 0 to
 *            n_bins - 1 (for instance from gw_rb_edges).
 *   flags    0 or GW_FLAG_ADD_NORM (every lnL then carries -sum ln(2 pi S));
 *            any other bit is GW_EINVAL.
 *   rb       receives the handle, which owns about (72 + 96 n_det) (B + 1)
 *            + (56 n_det + 16) B bytes of device memory until gw_rb_destroy. */
int gw_rb_create(gw_workspace *ws, const gw_grid *grid, int n_det, const gw_detector *dets, const gw_c128 *data,
                 const double *psd, const double *theta0, int n_param, const int64_t *edges, int64_t n_edges,
                 unsigned flags, gw_relbin **rb, hipStream_t stream);

/* Free a handle and its device memory (waits for the device).  NULL is ignored. */
int gw_rb_destroy(gw_relbin *rb);

/* Relative-binning lnL of every row of theta.
 *   ws        workspace on the handle's device: scratch for the sample records
 *             and partial sums, and the hot-kernel timer (gw_workspace_set_timing).
 *   theta     device [n_samples][n_param of the handle]; lnl_out device [n_samples].
 *   precision GW_PREC_FP64, or GW_PREC_MIXED: the ratio's phasor from the FP32
 *             hardware sine and cosine of the FP64 phase reduced to a
 *             fractional turn; the ratio and every sum stay FP64.
 * Per-row domain rules as for gw_lnl_batch. */
int gw_rb_lnl(gw_workspace *ws, const gw_relbin *rb, const double *theta, int64_t n_samples, double *lnl_out,
              int precision, hipStream_t stream);

/* Number of bins B and of detectors of a handle. */
int gw_rb_shape(const gw_relbin *rb, int64_t *n_rb, int *n_det);

/* Copies of the summary data as formed (inspection and test support; waits
 * for the device):
 *   raw_out     host [B][n_det][7]: A0 re, A0 im, A1 re, A1 im, B0, B1, B2;
 *   totals_out  host [2]: <d,d> and sum ln(2 pi S).  Either may be NULL. */
int gw_rb_summary(const gw_relbin *rb, double *raw_out, double *totals_out);

/* How gw_lnl_batch splits a call of this shape on the workspace's device:
 * the plan tuned for its size class when there is one, else the default
 * (inspection and test support; no device work):
 *   tile_bins  bins staged in LDS at a time;
 *   n_chunks   bin chunks per group of 256 samples (partial sums per chunk);
 *   rounds     0: one block per (sample group, chunk) item, in one wave of
 *              resident blocks; R >= 1: a persistent grid over one work queue
 *              per XCD, the chunks in R rounds, each covering half the bins
 *              the earlier rounds left (the last round the rest).
 * n_bins >= 1, 1 <= n_det <= GW_MAX_DET, n_samples >= 1, precision and flags
 * as for gw_lnl_batch; any output pointer may be NULL.  Returns GW_OK,
 * GW_EINVAL or GW_EDEVICE. */
int gw_lnl_plan(gw_workspace *ws, int64_t n_bins, int n_det, int64_t n_samples, int precision, unsigned flags,
                int *tile_bins, int *n_chunks, int *rounds);

/* Set the plan gw_lnl_batch uses on this workspace for the size class of
 * (n_bins, n_det, n_samples, precision, flags), as the autotuner records it:
 * for reproducing a plan read with gw_lnl_plan on another workspace or in
 * another process (plans differ only in the order of FP64 additions) or for
 * comparing plans.
 *   tile_bins  bins staged in LDS per tile: a multiple of 64, at most the
 *              largest tile the LDS budget allows for the size class;
 *   rounds     work-queue rounds, 0..16 (0: one block per item; a size that
 *              cannot take R rounds, and the ISCO end, use 0).
 * tile_bins == 0 and rounds == 0 remove the class's plan (the default is used
 * again, or the autotuner's choice once it has timed the class anew).  Sizes,
 * precision and flags as for gw_lnl_plan.  Returns GW_OK or GW_EINVAL. */
int gw_workspace_set_plan(gw_workspace *ws, int64_t n_bins, int n_det, int64_t n_samples, int precision,
                          unsigned flags, int tile_bins, int rounds);

/* Tile shape the last gw_lnl_ragged call used: bins staged in LDS per tile and
 * bins per work item.  The first call for a new size class times every
 * candidate shape once (several passes, results overwritten) and keeps the
 * fastest for later calls of that class on this workspace. */
int gw_ragged_tuning(const gw_workspace *ws, int *tile_bins, int64_t *chunk_bins);

/* ------------------------------------------------------------------------
 * Learned proposal and many-chain Metropolis-Hastings
 *
 * The paper (Sec. I) observes that the sampling algorithm itself is hard to
 * parallelise while the likelihood is embarrassingly parallel.  These calls
 * run many chains at once on the GPU, with the exact likelihood above as the
 * Metropolis-Hastings judge, and a normalising flow trained on the chains'
 * own samples as an independence proposal.
 *
 * Sampler coordinates: x in R^dim (dim 9 or 11), x_i = logit(u_i) with u_i the
 * position of parameter i in a uniform prior box [lo_i, hi_i]; the parameters
 * are, in order, Mc, q, d_L, phi_c, t_c, RA, sin Dec, psi, cos iota and, for
 * dim 11, two aligned spins that the non-spinning waveform does not use.
 * ------------------------------------------------------------------------ */

/* Philox4x32-10 (Salmon et al., SC 2011) block `i` of counter
 * (i mod 2^32, i div 2^32, step, stream_id) and key (seed mod 2^32, seed div 2^32),
 * for i = first .. first + n_blocks - 1 (mod 2^64): out (device) [n_blocks][4],
 * row j holding block first + j. */
int gw_philox_raw(uint64_t seed, uint32_t stream_id, uint32_t step, uint64_t first, int64_t n_blocks,
                  uint32_t *out, hipStream_t stream);

/* out (device) [n]: kind 0 uniforms in (0,1) (53 random bits; numbers 2i and
 * 2i+1 from block i), kind 1 standard normals (Box-Muller of that pair). */
int gw_philox_fill(uint64_t seed, uint32_t stream_id, uint32_t step, int kind, int64_t n, double *out,
                   hipStream_t stream);

/* out (device) [n_chains][dim]: normal i of chain c is member i mod 2 of the
 * Box-Muller pair of block c ceil(dim/2) + i div 2. */
int gw_philox_chain_normals(int dim, int64_t n_chains, uint64_t seed, uint32_t stream_id, uint32_t step,
                            double *out, hipStream_t stream);

/* theta_out (device) [n][theta_cols] in the layout of gw_lnl_batch, and the
 * log prior density of x, sum_i log u_i (1 - u_i) (logprior_out may be NULL).
 * box_lo, box_hi: host [dim]; the sin Dec and cos iota boxes lie in [-1, 1].
 * theta_cols 9: the nine non-spinning columns (with dim 11 the two spin
 * coordinates stay sampler-only); theta_cols 11 (dim 11 only): the spin
 * coordinates become chi1, chi2 in columns 9 and 10, their boxes within
 * [-1, 1]. */
int gw_mcmc_to_theta(int dim, int64_t n, const double *box_lo, const double *box_hi, const double *x,
                     int theta_cols, double *theta_out, double *logprior_out, hipStream_t stream);

/* Random-walk proposals x_prop = x + L z, z from Philox stream 1 at `step`
 * (chain c uses the normals of gw_philox_chain_normals).  chol: device [dim][dim],
 * lower triangular.  With mode non-NULL only chains whose mode is 1 (random
 * walk) are written. */
int gw_mcmc_rw_propose(int dim, int64_t n, const double *x, const double *chol, uint64_t seed, uint32_t step,
                       const int *mode, double *x_prop, hipStream_t stream);

/* Metropolis-Hastings decision for every chain, with the uniform from Philox
 * stream 2 at `step`:
 *   log alpha = lnl_prop + lp_prop - lnp  [+ logq - logq_prop for chains in mode 0]
 * On acceptance x and lnp (= lnl + lp) take the proposal's values, and for
 * chains in mode 0 so does logq.  mode NULL means every chain used a symmetric
 * proposal (logq, logq_prop may then be NULL).  Each acceptance adds 1 to
 * window_accepts[c] and total_accepts[c] (device int32, either may be NULL). */
int gw_mcmc_accept(int dim, int64_t n, uint64_t seed, uint32_t step, double *x, double *lnp, double *logq,
                   const double *x_prop, const double *lnl_prop, const double *lp_prop, const double *logq_prop,
                   const int *mode, int *window_accepts, int *total_accepts, hipStream_t stream);

/* mode[c] = 1 (random walk) when window_accepts[c] < threshold * window, else
 * 0 (flow proposals); window_accepts restarts at zero. */
int gw_mcmc_update_mode(int64_t n, int *window_accepts, int window, double threshold, int *mode,
                        hipStream_t stream);

/* Random-walk adaptation from the chains themselves (Haario, Saksman &
 * Tamminen 2001, with the 2.38^2/d scaling of Roberts, Gelman & Gilks 1997):
 * chol_out (device [dim][dim], lower triangular, upper part written zero) is
 * the Cholesky factor of (2.38^2 / dim) scale^2 Cov(x) + eps I, Cov the sample
 * covariance of the n rows of x (device [n][dim]), eps = floor max(1, tr/dim)
 * with tr the trace of the scaled covariance.  A non-positive pivot (a
 * degenerate chain set) is replaced by sqrt(eps).  One block; n >= 2,
 * scale > 0, floor >= 0. */
int gw_mcmc_adapt_chol(int dim, int64_t n, const double *x, double scale, double floor, double *chol_out,
                       hipStream_t stream);

/* Sample mean (mean_out, device [dim]) and covariance (cov_out, device
 * [dim][dim], divisor n - 1) of the n rows of x (device [n][dim]); either
 * output may be NULL, not both.  n >= 2. */
int gw_mcmc_moments(int dim, int64_t n, const double *x, double *mean_out, double *cov_out, hipStream_t stream);

/* out (device int64 [1]) = sum of counts (device int32 [n]), e.g. the
 * acceptance counters of gw_mcmc_accept. */
int gw_mcmc_count(int64_t n, const int *counts, int64_t *out, hipStream_t stream);

/* Rows drawn with replacement: dst[i] = src[floor(u_i n_src)] for i < n_out,
 * u_i uniform number i of Philox (seed, stream_id, step) as in
 * gw_philox_fill.  src device [n_src][dim], dst device [n_out][dim]
 * (minibatches for gw_flow_train_step). */
int gw_gather_rows(int dim, int64_t n_out, const double *src, int64_t n_src, uint64_t seed, uint32_t stream_id,
                   uint32_t step, double *dst, hipStream_t stream);

/* Affine-coupling flow (RealNVP): x = mu + sigma * f_{L-1}(... f_0(z)), z ~ N(0, I).
 * Layer l keeps the dimensions whose bit is set in cond_masks[l] and maps the
 * others as y = a exp(s) + t, s = 3 tanh(r/3), (r, t) = MLP_l(masked a),
 * MLP = Linear(dim, H) ReLU Linear(H, H) ReLU Linear(H, 2 dim) (r first).
 * The MLPs run on BF16 matrix cores with FP32 accumulation; the coupling, the
 * state and the log densities are FP64.  Parameters are FP32, per layer in
 * the order W1 [H][dim], b1 [H], W2 [H][H], b2 [H], W3 [2 dim][H], b3 [2 dim].
 * A flow object is bound to one device; it is not thread-safe. */
typedef struct gw_flow gw_flow;

int gw_flow_create(gw_flow **flow, int device, int dim, int n_layers, int hidden, const unsigned *cond_masks);
int gw_flow_destroy(gw_flow *flow);
int64_t gw_flow_num_params(const gw_flow *flow);

/* Host copies in/out of the parameters, mu and log sigma; setting resets the
 * optimiser state.  Both wait for the device. */
int gw_flow_set_params(gw_flow *flow, const float *params, const double *mu, const double *log_sigma);
int gw_flow_get_params(const gw_flow *flow, float *params, double *mu, double *log_sigma);

/* z (device) [n][dim] -> x_out [n][dim] (may be z itself) and log q(x)
 * (logq_out may be NULL). */
int gw_flow_forward(gw_flow *flow, const double *z, int64_t n, double *x_out, double *logq_out,
                    hipStream_t stream);

/* x (device) [n][dim] -> z_out (may be NULL) and log q(x) (may be NULL). */
int gw_flow_inverse(gw_flow *flow, const double *x, int64_t n, double *z_out, double *logq_out,
                    hipStream_t stream);

/* Gradient (device, [num_params] FP32) of the mean of -log q over the rows
 * of x, and that mean (device scalar, may be NULL), without updating. */
int gw_flow_gradients(gw_flow *flow, const double *x, int64_t n, float *grad_out, double *loss_out,
                      hipStream_t stream);

/* One Adam step (beta 0.9, 0.999, eps 1e-8, learning rate lr) on the mean of
 * -log q over the rows of x; the loss before the step goes to loss_out. */
int gw_flow_train_step(gw_flow *flow, const double *x, int64_t n, float lr, double *loss_out, hipStream_t stream);

/* Message about the last failing call on this thread ("" if none). */
const char *gw_last_error(void);

/* Library version as major*10000 + minor*100 + patch. */
int gw_version(void);

/* Layout check for bindings, which must not call into a library whose
 * structures they describe differently.  sizes_out (host, `capacity`
 * entries, may be NULL when capacity is 0) receives, in order:
 * sizeof(gw_c128), sizeof(gw_grid), sizeof(gw_detector), sizeof(gw_event),
 * offsetof(gw_event, dets) and GW_MAX_DET.  Returns the number of entries
 * the library reports (6, of which the first min(6, capacity) are written),
 * or GW_EABI when the library's translation units were compiled from
 * different sources (a link of objects from different builds, whose internal
 * structures need not agree).  gw_workspace_create and gw_flow_create refuse
 * to work in such a library with the same code.  No device is used. */
int gw_abi_layout(int64_t *sizes_out, int capacity);

/* SHA-256 (64 hex digits) over the sources and public header the library was
 * compiled from; a binding can compare it with its own source tree to detect
 * a library left over from older sources.  Static storage; no device is used. */
const char *gw_source_hash(void);

#ifdef __cplusplus
}
#endif

#endif /* GWLNL_H */
