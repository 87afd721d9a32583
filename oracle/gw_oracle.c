/*
 * Plain FP64 CPU oracle for the batched TaylorF2 single-event likelihood.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may include, link,
 * load or call this file; only the test-suite, the smoke check and the CPU
 * baseline of the benchmark use it.  It shares no code with the HIP library.
 *
 * What it computes (Talbot, Smith, Thrane & Poole 2019, arXiv:1904.02863):
 *   lnL(theta) = -(2/T) sum_det sum_bins |d - h(theta)|^2 / S
 * i.e. the exponent of the Gaussian likelihood of Eq. (cbclike) (Sec. III),
 * with T = 1/delta_f the segment duration, h the response of each detector to
 * a TaylorF2 inspiral (Sec. II) including its time translation
 * exp(-2 pi i f dt_det) (Sec. III, the paragraph after Eq. (cbclike)).
 * The theta-independent factor prod 1/(2 pi S) of Eq. (cbclike) is left out.
 *
 * The paper does not print the waveform; it names TaylorF2 and cites Ajith
 * (2011).  This file writes out the standard non-spinning form:
 *   Newtonian amplitude  A(f) = sqrt(5/24) pi^(-2/3) Mc^(5/6) f^(-7/6) / D
 *   3.5PN phase          Psi(f) = 2 pi f t_c - phi_c - pi/4
 *                               + 3/(128 eta v^5) sum_k (phi_k + phi_k^l ln v) v^k,
 *                        v = (pi M f)^(1/3)
 * with the phase coefficients of Buonanno, Iyer, Ochsner, Pan & Sathyaprakash,
 * PRD 80, 084043 (2009), Eq. (3.18), ln v convention.  Geometric units use
 * GM_sun = 1.3271244e20 m^3 s^-2 (IAU 2015 B3 nominal), c = 299792458 m/s and
 * 1 Mpc = 3.0856775814913673e22 m.
 *
 * Readings where the paper is silent (each listed in the design notes):
 *  - h_plus  = A (1 + cos^2 iota)/2 e^{-i Psi},  h_cross = -i A cos(iota) e^{-i Psi};
 *  - detector response h_det = (F+ h_plus + Fx h_cross) e^{-2 pi i f dt_det},
 *    F = D : e (antenna tensors below), dt_det = -n.r_det / c, GMST = 0;
 *  - no upper frequency cut-off by default: h is evaluated on every bin; on
 *    request (isco != 0) h = 0 above the gravitational-wave frequency of the
 *    Schwarzschild innermost stable circular orbit of the total mass M,
 *    f_isco = c^3 / (6^(3/2) pi G M), the usual end of an inspiral template;
 *  - 5-parameter rows are an optimally oriented source: h = A e^{-i Psi};
 *  - 7- and 11-parameter rows are the 5- and 9-parameter rows followed by
 *    the aligned spins chi1 (of the heavier body) and chi2, which add the
 *    spin terms of oracle_pn_spin_terms to the phase (the amplitude stays
 *    Newtonian); |chi| > 1 gives -infinity;
 *  - any non-finite parameter gives NaN; Mc <= 0, q outside (0, 1] or
 *    d_L <= 0 give -infinity.
 * Sums use Neumaier compensation per (sample, detector), then across
 * detectors in order.  On request (add_norm != 0) lnL also carries the
 * logarithm of the prefactor of Eq. (cbclike), -sum_det sum_bins ln(2 pi S).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stddef.h>

#define ORACLE_PI 3.14159265358979323846
#define ORACLE_EULER_GAMMA 0.57721566490153286061
#define ORACLE_GM_SUN 1.3271244e20            /* m^3 s^-2 */
#define ORACLE_C_SI 299792458.0               /* m s^-1 */
#define ORACLE_MPC_SI 3.0856775814913673e22   /* m */

/* Solar mass in seconds, G M_sun / c^3. */
static double msun_s(void) { return ORACLE_GM_SUN / (ORACLE_C_SI * ORACLE_C_SI * ORACLE_C_SI); }

/* TaylorF2 phase coefficients phi_k and their ln v partners phi_k^l, k = 0..7,
 * for symmetric mass ratio eta; Buonanno et al. 2009, Eq. (3.18). */
int oracle_pn_coefficients(double eta, double phi[8], double phi_log[8])
{
    const double pi = ORACLE_PI, pi2 = ORACLE_PI * ORACLE_PI;
    const double e2 = eta * eta, e3 = eta * eta * eta;
    for (int k = 0; k < 8; ++k) { phi[k] = 0.0; phi_log[k] = 0.0; }
    phi[0] = 1.0;
    phi[1] = 0.0;
    phi[2] = 3715.0 / 756.0 + 55.0 / 9.0 * eta;
    phi[3] = -16.0 * pi;
    phi[4] = 15293365.0 / 508032.0 + 27145.0 / 504.0 * eta + 3085.0 / 72.0 * e2;
    phi[5] = pi * (38645.0 / 756.0 - 65.0 / 9.0 * eta);
    phi_log[5] = 3.0 * phi[5];
    phi[6] = 11583231236531.0 / 4694215680.0 - 640.0 / 3.0 * pi2 - 6848.0 / 21.0 * ORACLE_EULER_GAMMA
           - 6848.0 / 21.0 * log(4.0)
           + (-15737765635.0 / 3048192.0 + 2255.0 / 12.0 * pi2) * eta
           + 76055.0 / 1728.0 * e2 - 127825.0 / 1296.0 * e3;
    phi_log[6] = -6848.0 / 21.0;
    phi[7] = pi * (77096675.0 / 254016.0 + 378515.0 / 1512.0 * eta - 74045.0 / 756.0 * e2);
    return 0;
}

/* Aligned-spin additions to phi_k (and to phi_5^l) for dimensionless spins
 * chi1 (heavier body, m1) and chi2 (lighter, m2) along the orbital angular
 * momentum, written with chi_s = (chi1 + chi2)/2, chi_a = (chi1 - chi2)/2 and
 * delta = (m1 - m2)/M:
 *   1.5PN spin-orbit (Kidder 1995; Arun, Buonanno, Faye & Ochsner 2009),
 *   2PN spin-spin with the black-hole quadrupole-monopole term, kappa = 1
 *     (Kidder 1995; Poisson 1998),
 *   2.5PN spin-orbit, entering as phi_5 (1 + 3 ln v) like the non-spinning
 *     2.5PN term (Blanchet, Buonanno & Faye 2006),
 *   3PN spin-orbit including its tail (Blanchet 2014, Living Rev. Relativ. 17, 2),
 *   3.5PN spin-orbit (Bohe, Marsat, Faye & Blanchet 2013).
 * Spin-spin terms beyond 2PN and cubic-in-spin terms are not included. */
void oracle_pn_spin_terms(double eta, double delta, double chi1, double chi2, double phi[8], double phi_log[8])
{
    const double pi = ORACLE_PI, e2 = eta * eta, e3 = eta * eta * eta;
    const double cs = 0.5 * (chi1 + chi2), ca = 0.5 * (chi1 - chi2);
    phi[3] += 113.0 / 3.0 * delta * ca + (113.0 / 3.0 - 76.0 / 3.0 * eta) * cs;
    phi[4] += -(405.0 / 8.0 - 200.0 * eta) * ca * ca - 405.0 / 4.0 * delta * cs * ca
              - (405.0 / 8.0 - 5.0 / 2.0 * eta) * cs * cs;
    const double gamma = (732985.0 / 2268.0 - 24260.0 / 81.0 * eta - 340.0 / 9.0 * e2) * cs
                       + (732985.0 / 2268.0 + 140.0 / 9.0 * eta) * delta * ca;
    phi[5] -= gamma;
    phi_log[5] -= 3.0 * gamma;
    phi[6] += pi * (2270.0 / 3.0 * delta * ca + (2270.0 / 3.0 - 520.0 * eta) * cs);
    phi[7] += (-25150083775.0 / 3048192.0 + 10566655595.0 / 762048.0 * eta - 1042165.0 / 3024.0 * e2
               + 5345.0 / 36.0 * e3) * cs
            + delta * (-25150083775.0 / 3048192.0 + 26804935.0 / 6048.0 * eta - 1985.0 / 48.0 * e2) * ca;
}

/* The post-Newtonian part of the TaylorF2 phase at v = (pi M f)^(1/3):
 *   3/(128 eta v^5) sum_k (phi_k + phi_k^l ln v) v^k. */
static double pn_series_phase(double eta, const double phi[8], const double phi_log[8], double v)
{
    const double lnv = log(v);
    double series = 0.0, vk = 1.0;
    for (int k = 0; k < 8; ++k) {
        series += (phi[k] + phi_log[k] * lnv) * vk;
        vk *= v;
    }
    return 3.0 / (128.0 * eta * pow(v, 5)) * series;
}

/* Symmetric mass ratio and total mass (seconds) from chirp mass (solar
 * masses) and q = m2/m1. */
static void masses(double mc, double q, double *eta, double *mtot_s)
{
    *eta = q / ((1.0 + q) * (1.0 + q));
    *mtot_s = mc * pow(*eta, -0.6) * msun_s();
}

/* The post-Newtonian part of the phase at frequency f (Hz) for chirp mass mc
 * (solar masses) and q = m2/m1; the waveform adds 2 pi f t_c - phi_c - pi/4. */
double oracle_pn_phase(double mc, double q, double f)
{
    double eta, mtot_s, phi[8], phi_log[8];
    masses(mc, q, &eta, &mtot_s);
    oracle_pn_coefficients(eta, phi, phi_log);
    return pn_series_phase(eta, phi, phi_log, cbrt(ORACLE_PI * mtot_s * f));
}

/* Unit vectors of the source frame for right ascension ra and declination dec
 * (GMST = 0): n points from the geocentre to the source, e_ra and e_dec span
 * the plane of the sky. */
static void sky_basis(double ra, double dec, double n[3], double e_ra[3], double e_dec[3])
{
    n[0] = cos(dec) * cos(ra);  n[1] = cos(dec) * sin(ra);  n[2] = sin(dec);
    e_ra[0] = -sin(ra);         e_ra[1] = cos(ra);          e_ra[2] = 0.0;
    e_dec[0] = -sin(dec) * cos(ra); e_dec[1] = -sin(dec) * sin(ra); e_dec[2] = cos(dec);
}

/* Antenna patterns F+ = D : e+, Fx = D : ex of a detector with tensor D
 * (row-major 3x3), polarisation tensors e+ = X X^T - Y Y^T, ex = X Y^T + Y X^T
 * with X = cos psi e_ra + sin psi e_dec, Y = -sin psi e_ra + cos psi e_dec. */
void oracle_antenna(const double tensor[9], double ra, double dec, double psi, double *fplus, double *fcross)
{
    double n[3], ea[3], ed[3], x[3], y[3];
    sky_basis(ra, dec, n, ea, ed);
    for (int i = 0; i < 3; ++i) {
        x[i] = cos(psi) * ea[i] + sin(psi) * ed[i];
        y[i] = -sin(psi) * ea[i] + cos(psi) * ed[i];
    }
    double fp = 0.0, fx = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            fp += tensor[3 * i + j] * (x[i] * x[j] - y[i] * y[j]);
            fx += tensor[3 * i + j] * (x[i] * y[j] + y[i] * x[j]);
        }
    *fplus = fp;
    *fcross = fx;
}

/* Arrival time at a detector at `vertex` (metres) minus arrival time at the
 * geocentre for a plane wave from (ra, dec): -n . r / c. */
double oracle_delay(const double vertex[3], double ra, double dec)
{
    double n[3], ea[3], ed[3];
    sky_basis(ra, dec, n, ea, ed);
    return -(n[0] * vertex[0] + n[1] * vertex[1] + n[2] * vertex[2]) / ORACLE_C_SI;
}

/* Rows with aligned spins carry chi1, chi2 as their last two columns. */
static int has_spins(int n_param) { return n_param == 7 || n_param == 11; }
/* Rows with a sky position, polarisation and inclination (columns 5-8). */
static int has_sky(int n_param) { return n_param == 9 || n_param == 11; }

/* Classification of one parameter row: 1 = evaluate, 0 = out of domain
 * (-infinity), -1 = non-finite (NaN). */
static int classify(const double *th, int n_param)
{
    for (int i = 0; i < n_param; ++i)
        if (!isfinite(th[i])) return -1;
    if (!(th[0] > 0.0) || !(th[1] > 0.0 && th[1] <= 1.0) || !(th[2] > 0.0)) return 0;
    if (has_spins(n_param) && (fabs(th[n_param - 2]) > 1.0 || fabs(th[n_param - 1]) > 1.0)) return 0;
    return 1;
}

/* Everything about one parameter row that does not depend on frequency. */
typedef struct {
    double eta, mtot_s, amp0, phic, tc, cos_iota;
    double f_cut;                 /* h = 0 at f > f_cut (infinity without the cut-off) */
    double phi[8], phi_log[8];
    int n_det;
    double fplus[8], fcross[8], dt[8];
} source;

/* Gravitational-wave frequency (twice the orbital one) at the innermost
 * stable circular orbit of a test mass around a Schwarzschild black hole of
 * mass M (seconds): r = 6 M, orbital angular frequency M^(1/2) r^(-3/2). */
static double isco_frequency(double mtot_s)
{
    return 1.0 / (pow(6.0, 1.5) * ORACLE_PI * mtot_s);
}

static void make_source(const double *th, int n_param, int n_det, int isco,
                        const double *tensors, const double *vertices, source *src)
{
    const double mc = th[0], q = th[1], dl = th[2];
    masses(mc, q, &src->eta, &src->mtot_s);
    src->f_cut = isco ? isco_frequency(src->mtot_s) : INFINITY;
    const double mc_s = mc * msun_s();
    const double dist_s = dl * ORACLE_MPC_SI / ORACLE_C_SI;
    src->amp0 = sqrt(5.0 / 24.0) * pow(ORACLE_PI, -2.0 / 3.0) * pow(mc_s, 5.0 / 6.0) / dist_s;
    src->phic = th[3];
    src->tc = th[4];
    src->cos_iota = has_sky(n_param) ? cos(th[8]) : 1.0;
    oracle_pn_coefficients(src->eta, src->phi, src->phi_log);
    if (has_spins(n_param)) {
        const double q = th[1];
        const double delta = (1.0 - q) / (1.0 + q);
        oracle_pn_spin_terms(src->eta, delta, th[n_param - 2], th[n_param - 1], src->phi, src->phi_log);
    }
    src->n_det = n_det;
    for (int d = 0; d < n_det; ++d) {
        if (has_sky(n_param)) {
            oracle_antenna(tensors + 9 * d, th[5], th[6], th[7], &src->fplus[d], &src->fcross[d]);
            src->dt[d] = oracle_delay(vertices + 3 * d, th[5], th[6]);
        } else {   /* optimally oriented, overhead source */
            src->fplus[d] = 1.0; src->fcross[d] = 0.0; src->dt[d] = 0.0;
        }
    }
}

/* The two TaylorF2 polarisations at frequency f. */
static void polarisations(const source *src, double f, double complex *hp, double complex *hx)
{
    if (f > src->f_cut) { *hp = 0.0; *hx = 0.0; return; }
    const double v = cbrt(ORACLE_PI * src->mtot_s * f);
    const double psi = 2.0 * ORACLE_PI * f * src->tc - src->phic - ORACLE_PI / 4.0
                     + pn_series_phase(src->eta, src->phi, src->phi_log, v);
    const double complex h = src->amp0 * pow(f, -7.0 / 6.0) * cexp(-I * psi);
    *hp = 0.5 * (1.0 + src->cos_iota * src->cos_iota) * h;
    *hx = -I * src->cos_iota * h;
}

/* Response of detector d at frequency f given the polarisations there. */
static double complex response(const source *src, int d, double f, double complex hp, double complex hx)
{
    return (src->fplus[d] * hp + src->fcross[d] * hx) * cexp(-2.0 * ORACLE_PI * I * f * src->dt[d]);
}

static int check_args(double delta_f, int64_t n_bins, int n_det, int n_param, int64_t n_samples)
{
    if (!(delta_f > 0.0) || n_bins < 0 || n_det < 0 || n_det > 8 || n_samples < 0) return -1;
    if (n_param != 5 && n_param != 7 && n_param != 9 && n_param != 11) return -1;
    return 0;
}

/* Waveforms of n_samples parameter rows on bins f_low + k delta_f.
 * n_det > 0: detector responses, out[(s * n_det + d) * n_bins + k].
 * n_det == 0: polarisations, out[(s * 2 + p) * n_bins + k], p = 0 plus, 1 cross.
 * isco != 0 ends every template at its f_isco.
 * Rows that are out of domain or non-finite produce NaN. */
int oracle_waveform(double f_low, double delta_f, int64_t n_bins, int n_det,
                    const double *tensors, const double *vertices,
                    const double *theta, int n_param, int64_t n_samples, int isco, double complex *out)
{
    if (check_args(delta_f, n_bins, n_det, n_param, n_samples)) return -1;
    const int n_out = n_det > 0 ? n_det : 2;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < n_samples; ++s) {
        const double *th = theta + s * n_param;
        const int ok = classify(th, n_param);
        source src;
        if (ok == 1) make_source(th, n_param, n_det, isco, tensors, vertices, &src);
        for (int64_t k = 0; k < n_bins; ++k) {
            const double f = f_low + (double)k * delta_f;
            double complex hp = NAN, hx = NAN;
            if (ok == 1) polarisations(&src, f, &hp, &hx);
            for (int d = 0; d < n_out; ++d) {
                double complex *o = out + ((size_t)s * n_out + d) * n_bins + k;
                if (ok != 1) *o = NAN;
                else if (n_det > 0) *o = response(&src, d, f, hp, hx);
                else *o = d == 0 ? hp : hx;
            }
        }
    }
    return 0;
}

/* Detector responses of n_samples parameter rows at an arbitrary list of
 * n_freq frequencies (the unevenly spaced frequencies of relative binning):
 * out[(s * n_det + d) * n_freq + j] = h_det(freqs[j]), n_det >= 1.  Rows that
 * are out of domain or non-finite produce NaN. */
int oracle_waveform_at(const double *freqs, int64_t n_freq, int n_det,
                       const double *tensors, const double *vertices,
                       const double *theta, int n_param, int64_t n_samples, double complex *out)
{
    if (check_args(1.0, n_freq, n_det, n_param, n_samples) || n_det < 1) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < n_samples; ++s) {
        const double *th = theta + s * n_param;
        const int ok = classify(th, n_param);
        source src;
        if (ok == 1) make_source(th, n_param, n_det, 0, tensors, vertices, &src);
        for (int64_t j = 0; j < n_freq; ++j) {
            double complex hp = NAN, hx = NAN;
            if (ok == 1) polarisations(&src, freqs[j], &hp, &hx);
            for (int d = 0; d < n_det; ++d)
                out[((size_t)s * n_det + d) * n_freq + j] = ok == 1 ? response(&src, d, freqs[j], hp, hx) : NAN;
        }
    }
    return 0;
}

/* Neumaier's compensated summation step. */
static void neumaier_add(double *sum, double *comp, double x)
{
    const double t = *sum + x;
    if (fabs(*sum) >= fabs(x)) *comp += (*sum - t) + x;
    else *comp += (x - t) + *sum;
    *sum = t;
}

/* lnL of Eq. (cbclike) without its theta-independent factor, for each of the
 * n_samples parameter rows:  lnl[s] = -2 delta_f sum_d sum_k |d_dk - h_dk|^2 / S_dk.
 * data: (n_det, n_bins) complex; psd: (n_det, n_bins).  isco != 0 ends every
 * template at its f_isco; add_norm != 0 adds the log of the factor
 * prod 1/(2 pi S_dk), -sum_d sum_k ln(2 pi S_dk), to every finite value.
 * n_threads <= 0 uses the OpenMP default. */
int oracle_lnl(double f_low, double delta_f, int64_t n_bins, int n_det,
               const double *tensors, const double *vertices,
               const double complex *data, const double *psd,
               const double *theta, int n_param, int64_t n_samples, int isco, int add_norm,
               double *lnl, int n_threads)
{
    if (check_args(delta_f, n_bins, n_det, n_param, n_samples) || n_det < 1) return -1;
    double norm = 0.0;
    if (add_norm) {
        double per[8] = {0}, per_c[8] = {0}, nc = 0.0;
        for (int d = 0; d < n_det; ++d)
            for (int64_t k = 0; k < n_bins; ++k)
                neumaier_add(&per[d], &per_c[d], log(2.0 * ORACLE_PI * psd[(size_t)d * n_bins + k]));
        for (int d = 0; d < n_det; ++d) neumaier_add(&norm, &nc, per[d] + per_c[d]);
        norm += nc;
    }
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    extern int omp_get_max_threads(void);
    const int saved = omp_get_max_threads();
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < n_samples; ++s) {
        const double *th = theta + s * n_param;
        const int ok = classify(th, n_param);
        if (ok < 0) { lnl[s] = NAN; continue; }
        if (ok == 0) { lnl[s] = -INFINITY; continue; }
        source src;
        make_source(th, n_param, n_det, isco, tensors, vertices, &src);
        double sum[8] = {0}, comp[8] = {0};
        for (int64_t k = 0; k < n_bins; ++k) {
            const double f = f_low + (double)k * delta_f;
            double complex hp, hx;
            polarisations(&src, f, &hp, &hx);
            for (int d = 0; d < n_det; ++d) {
                const double complex r = data[(size_t)d * n_bins + k] - response(&src, d, f, hp, hx);
                const double r2 = creal(r) * creal(r) + cimag(r) * cimag(r);
                neumaier_add(&sum[d], &comp[d], r2 / psd[(size_t)d * n_bins + k]);
            }
        }
        double total = 0.0, total_c = 0.0;
        for (int d = 0; d < n_det; ++d) neumaier_add(&total, &total_c, sum[d] + comp[d]);
        lnl[s] = -2.0 * delta_f * (total + total_c) - norm;
    }
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(saved);
#endif
    return 0;
}

/* Number of OpenMP threads a parallel region would use (1 without OpenMP). */
int oracle_max_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
