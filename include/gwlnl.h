/*
 * gwlnl.h -- C ABI of the MI355X (gfx950) batched TaylorF2 likelihood library.
 *
 * The library evaluates, for a batch of compact-binary parameter samples, the
 * Gaussian single-event log-likelihood of Talbot, Smith, Thrane & Poole 2019
 * (arXiv:1904.02863), Eq. (cbclike) in Sec. III:
 *
 *     lnL(theta) = -(2/T) sum_det sum_bins |d - h(theta)|^2 / S,   T = 1/delta_f,
 *
 * without the theta-independent factor prod (2 pi S)^-1 of that equation.
 * h is the response of each detector to a non-spinning TaylorF2 inspiral
 * (Sec. II: Newtonian amplitude, 3.5PN phase), projected with the detector's
 * antenna pattern and shifted by exp(-2 pi i f dt_det), the time translation
 * described after Eq. (cbclike).
 *
 * Conventions
 *  - Frequency bins: f_k = f_low + k * delta_f, k = 0 .. n_bins-1.  Every bin
 *    is evaluated (no upper cut-off).
 *  - Complex arrays are interleaved (re, im) double pairs, the layout of
 *    torch.complex128 / numpy complex128.
 *  - theta is row-major [n_samples][n_param], n_param 5 or 9, columns
 *      0 Mc   chirp mass, solar masses      1 q     m2/m1 in (0, 1]
 *      2 dL   luminosity distance, Mpc      3 phic  coalescence phase, rad
 *      4 tc   coalescence time at the geocentre relative to the segment, s
 *      5 ra   right ascension, rad (Greenwich sidereal time taken as 0)
 *      6 dec  declination, rad              7 psi   polarisation angle, rad
 *      8 iota inclination, rad
 *    With n_param == 5 the source is optimally oriented (F+ = 1, Fx = 0,
 *    iota = 0, no delay) and the detector geometry is not used.
 *  - h_plus = A (1 + cos^2 iota)/2 e^{-i Psi}, h_cross = -i A cos iota e^{-i Psi},
 *    A = sqrt(5/24) pi^(-2/3) Mc^(5/6) f^(-7/6) / dL (geometric units),
 *    Psi = 2 pi f tc - phic - pi/4 + 3/(128 eta v^5) sum_k (phi_k + phi_k^l ln v) v^k,
 *    v = (pi M f)^(1/3), coefficients of Buonanno et al. 2009, Eq. (3.18).
 *    Response h_det = (F+ h_plus + Fx h_cross) e^{-2 pi i f dt_det},
 *    F = D : e with the polarisation tensors of the sky basis, dt_det = -n.r/c.
 *  - Per-sample domain: any non-finite parameter gives lnL = NaN; Mc <= 0,
 *    q outside (0, 1] or dL <= 0 give lnL = -infinity.  These are not errors.
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
 *
 * Errors
 *  - Every function returns GW_OK (0) or a negative code; gw_last_error()
 *    returns a thread-local message about the last failing call.  Structural
 *    problems are reported synchronously and enqueue nothing: null pointers,
 *    n_bins < 1, delta_f <= 0 or non-finite, f_low <= 0 or non-finite,
 *    n_det outside 1..8, n_param not 5 or 9, n_samples < 0.
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
    GW_EUNSUPPORTED = -4   /* valid request this build does not implement */
};

enum {
    GW_PREC_FP64 = 0,      /* every step in FP64 */
    GW_PREC_MIXED = 1      /* FP64 phase and final sums, FP32 phasors and tile sums */
};

/* Create a workspace bound to HIP device `device` (the current device when
 * device < 0).  *ws receives the handle.  Allocates no device memory yet. */
int gw_workspace_create(gw_workspace **ws, int device);

/* Free a workspace and its device memory.  Waits for the device first.
 * NULL is accepted and ignored. */
int gw_workspace_destroy(gw_workspace *ws);

/* Size the workspace for events of up to n_bins bins and n_det detectors and
 * batches of up to n_samples samples, so that later calls within these sizes
 * allocate nothing. */
int gw_workspace_reserve(gw_workspace *ws, int64_t n_bins, int n_det, int64_t n_samples);

/* Bytes of device memory the workspace currently holds. */
int64_t gw_workspace_bytes(const gw_workspace *ws);

/* Measurement support.  While timing is enabled (enable != 0), every
 * likelihood call made with this workspace records a pair of HIP events on
 * its own stream around its hot kernel (the tile kernel that forms Z for
 * every sample, bin and detector).  Enabling clears earlier records. */
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
 */
int gw_waveform_batch(gw_workspace *ws, const gw_grid *grid, int n_det, const gw_detector *dets,
                      const double *theta, int n_param, int64_t n_samples,
                      gw_c128 *h_out, hipStream_t stream);

/*
 * gw_lnl_batch -- Eq. (cbclike) for every sample of one event.
 *   grid      host, the frequency grid shared by all detectors.
 *   n_det     detectors 1..8;  dets host [n_det] (ignored when n_param == 5).
 *   data      device [n_det][n_bins] complex, frequency-domain strain d~.
 *   psd       device [n_det][n_bins] doubles, one-sided PSD S(f) (1/Hz).
 *   theta     device [n_samples][n_param].
 *   lnl_out   device [n_samples] doubles.
 *   precision GW_PREC_FP64 or GW_PREC_MIXED.
 *   flags     must be 0 (reserved).
 */
int gw_lnl_batch(gw_workspace *ws, const gw_grid *grid, int n_det, const gw_detector *dets,
                 const gw_c128 *data, const double *psd,
                 const double *theta, int n_param, int64_t n_samples,
                 double *lnl_out, int precision, unsigned flags, hipStream_t stream);

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
 * own samples, in one persistent launch.
 *   events          host [n_events].
 *   data_packed     device complex, event e at data_offset_e, [n_det_e][n_bins_e].
 *   psd_packed      device doubles, same offsets as data_packed.
 *   theta_packed    device [sum n_samples][n_param]; event e uses rows
 *                   theta_offset_e .. theta_offset_e + n_samples_e - 1.
 *   lnl_out_packed  device, one double per row of theta_packed that an event uses.
 */
int gw_lnl_ragged(gw_workspace *ws, int n_events, const gw_event *events,
                  const gw_c128 *data_packed, const double *psd_packed,
                  const double *theta_packed, int n_param,
                  double *lnl_out_packed, int precision, unsigned flags, hipStream_t stream);

/* Message about the last failing call on this thread ("" if none). */
const char *gw_last_error(void);

/* Library version as major*10000 + minor*100 + patch. */
int gw_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GWLNL_H */
