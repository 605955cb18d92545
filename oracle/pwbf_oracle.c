/* FP64 reference plane-wave receive beamformer.
 *
 * TEST INFRASTRUCTURE ONLY: this file is the oracle against which the GPU path
 * is checked. Only the test suite, the smoke check and the benchmark's CPU
 * baseline may load it; the product path never does. It shares no code, header
 * or constant with the GPU library.
 *
 * Plain, slow and literal: double precision, libm sqrt/cos, no blocking, no
 * reordering. Every pixel value is evaluated straight from the definition, one
 * pixel, one angle and one element at a time. Built as is, it runs on one
 * thread; built with -fopenmp, the loop over the requested pixels is shared
 * among threads (each pixel is still computed by one thread in the same
 * order, so the values are bitwise those of the single-threaded build).
 *
 * What is computed (paper section II-B):
 *  - Eq. (1): y[p] = sum_i w_i[p] u_i[dn_p], the conventional delay-and-sum.
 *  - The delay dn_p: the paper prints the round trip of a synthetic-aperture
 *    shot, 2 fs/c * |r_i - r_p|, while its acquisition is a plane-wave transmit
 *    (section II-C, abstract). Read here as transmit plane-wave delay plus receive
 *    path: s = fs * ((x sin t + z cos t - d_t)/c + |r_i - r_p|/c - t0), with
 *    d_t = min_e(x_e sin t) so the first-firing element fires at time 0. At
 *    t = 0 and x = x_i it reduces to the printed 2 z fs / c.
 *  - u_i[s] at a fractional delay: linear interpolation between the two
 *    neighbouring samples, the record being zero outside [0, Ns).
 *  - w_i[p]: "predefined" in the paper; here Hann over the aperture z / F#
 *    centred on the pixel, w = 0.5 (1 + cos(pi d / a)) with d = |x - x_e| and
 *    a = z / (2 F#), zero for d >= a or z <= 0 (boxcar and "none" also offered).
 *  - Coherent compounding: the unweighted sum of the per-angle DAS images.
 *  - DMAS on RF with signed square-root compression, the weight outside the
 *    root as in Eq. (2): s_e = w_e sign(v_e) sqrt|v_e|, y = sum_{e<f} s_e s_f,
 *    the squared-sum structure of Eq. (4) without its 1/N. Computed both as
 *    the O(N^2) pair sum and as ((sum s)^2 - sum s^2) / 2; compounding sums the
 *    per-angle results.
 *  - pDAS, Eqs. (2)-(3): each delayed sample compressed to sign(v)|v|^(1/p),
 *    weighted and summed (the weight outside the root), then the sum restored
 *    by the signed p-th power; compounding sums the per-angle results, as for
 *    DMAS. p = 1 is DAS.
 *  - On IQ data (baseband channel records q[n] = a[n] exp(-2 pi i fd n / fs),
 *    a the analytic signal; the demodulation itself is in oracle/__init__.py):
 *    the delay-compensated IQ sample is q interpolated linearly (real and
 *    imaginary parts, zero outside [0, Ns)) at the delay s and rotated back by
 *    exp(2 pi i fd s / fs). IQ-DAS sums w q_delayed as Eq. (1) does; BB-DMAS,
 *    Eq. (4), squares the sum of w sqrt(|q|) exp(i arg q) (the weight outside
 *    the root as in Eq. (2), the constant 1/N dropped). Compounding sums the
 *    complex per-angle values.
 *
 * Pins (tests marked "not gpu"): impulse response of a single RF sample
 * (triangle-weighted iso-delay arc), point scatterer simulated independently
 * peaking at its own pixel, special-case delays (on-axis round trip, 3-4-5
 * triangle, steered first-firing element), linearity, channel superposition,
 * mirror symmetry, compound = sum of angles, DMAS pairs = identity, DMAS of
 * equal signals and of two channels in closed form, and a 4x4-pixel
 * brute-force re-implementation that interpolates with numpy.interp.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
  int32_t n_angles, n_channels, n_samples;
  const double *elem_x; /* [n_channels] element centres, m (array on z = 0) */
  const double *angle;  /* [n_angles] steering angles, rad */
  const double *t0;     /* [n_angles] time of sample 0, s */
  double c, fs;         /* m/s, Hz */
  int32_t nx, nz;
  double x0, dx, z0, dz; /* centre of pixel (0, 0) and pitches, m */
  double f_number;
  int32_t apod; /* 0 = Hann, 1 = boxcar, 2 = none (w = 1) */
} ora_geom;

enum { ORA_OK = 0, ORA_BAD = -1 };

/* Threads a call of this build shares its pixel loop among (1 unless built
 * with -fopenmp). */
int ora_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Every requested flat pixel index lies in [0, total). */
static int check_pixels(const int64_t *pix, int64_t npix, int64_t total) {
  if (npix < 0) return ORA_BAD;
  if (pix)
    for (int64_t k = 0; k < npix; ++k)
      if (pix[k] < 0 || pix[k] >= total) return ORA_BAD;
  return ORA_OK;
}

/* min_e(x_e sin th): the lateral term of the first-firing element for angle a. */
static double first_fire(const ora_geom *g, int32_t a) {
  double th = g->angle[a];
  double first = g->elem_x[0] * sin(th);
  for (int32_t k = 1; k < g->n_channels; ++k) {
    double v = g->elem_x[k] * sin(th);
    if (v < first) first = v;
  }
  return first;
}

static double tof(const ora_geom *g, int32_t a, double first, int32_t e, double x, double z) {
  double th = g->angle[a];
  double t_tx = (x * sin(th) + z * cos(th) - first) / g->c;
  double dxe = x - g->elem_x[e];
  double t_rx = sqrt(dxe * dxe + z * z) / g->c;
  return (t_tx + t_rx - g->t0[a]) * g->fs;
}

/* Time of flight in samples from transmit to the echo of (x, z) reaching element e. */
double ora_tof_samples(const ora_geom *g, int32_t a, int32_t e, double x, double z) {
  return tof(g, a, first_fire(g, a), e, x, z);
}

/* Receive apodization weight of element e for the pixel at (x, z). */
double ora_apod_weight(const ora_geom *g, int32_t e, double x, double z) {
  if (g->apod == 2) return 1.0;
  if (z <= 0.0) return 0.0;
  double half_aperture = z / (2.0 * g->f_number);
  double d = fabs(x - g->elem_x[e]);
  if (!(d < half_aperture)) return 0.0;
  if (g->apod == 1) return 1.0;
  return 0.5 * (1.0 + cos(M_PI * d / half_aperture));
}

/* u at fractional sample s: linear interpolation, u taken as zero outside [0, ns). */
double ora_interp(const double *u, int32_t ns, double s) {
  double n0 = floor(s);
  double f = s - n0;
  double a = 0.0, b = 0.0;
  if (n0 >= 0.0 && n0 < (double)ns) a = u[(int64_t)n0];
  if (n0 + 1.0 >= 0.0 && n0 + 1.0 < (double)ns) b = u[(int64_t)n0 + 1];
  return (1.0 - f) * a + f * b;
}

#define ORA_MAX_ANGLES 256

static int check(const ora_geom *g, int32_t angle) {
  if (!g || g->n_angles < 1 || g->n_channels < 1 || g->n_samples < 1) return ORA_BAD;
  if (g->n_angles > ORA_MAX_ANGLES) return ORA_BAD;
  if (angle < -1 || angle >= g->n_angles) return ORA_BAD;
  return ORA_OK;
}

static void pixel_xz(const ora_geom *g, int64_t p, double *x, double *z) {
  int64_t ix = p / g->nz, iz = p % g->nz;
  *x = g->x0 + (double)ix * g->dx;
  *z = g->z0 + (double)iz * g->dz;
}

/* Delayed, interpolated sample of element e for angle a at pixel (x, z). */
static double delayed(const ora_geom *g, const double *rf, int32_t a, double first, int32_t e,
                      double x, double z) {
  const double *u = rf + ((int64_t)a * g->n_channels + e) * g->n_samples;
  return ora_interp(u, g->n_samples, tof(g, a, first, e, x, z));
}

/* Eq. (1) for one angle. */
static double das_one_angle(const ora_geom *g, const double *rf, int32_t a, double first,
                            double x, double z) {
  double y = 0.0;
  for (int32_t e = 0; e < g->n_channels; ++e)
    y += ora_apod_weight(g, e, x, z) * delayed(g, rf, a, first, e, x, z);
  return y;
}

static double sgn(double v) { return (v > 0.0) - (v < 0.0); }

/* RF DMAS for one angle; form 0 = pair sum, form 1 = squared-sum identity. */
static double dmas_one_angle(const ora_geom *g, const double *rf, int32_t a, double first,
                             double x, double z, int32_t form) {
  int32_t n = g->n_channels;
  double s[1024];
  if (n > 1024) return NAN;
  for (int32_t e = 0; e < n; ++e) {
    double v = delayed(g, rf, a, first, e, x, z);
    s[e] = ora_apod_weight(g, e, x, z) * sgn(v) * sqrt(fabs(v));
  }
  if (form == 0) {
    double y = 0.0;
    for (int32_t i = 0; i < n; ++i)
      for (int32_t j = i + 1; j < n; ++j) y += s[i] * s[j];
    return y;
  }
  double sum = 0.0, sq = 0.0;
  for (int32_t e = 0; e < n; ++e) {
    sum += s[e];
    sq += s[e] * s[e];
  }
  return 0.5 * (sum * sum - sq);
}

/* pDAS, Eqs. (2)-(3), for one angle: the sum of w_e sign(v_e) |v_e|^(1/p), then
 * its signed p-th power. */
static double pdas_one_angle(const ora_geom *g, const double *rf, int32_t a, double first,
                             double x, double z, double p) {
  double yt = 0.0;
  for (int32_t e = 0; e < g->n_channels; ++e) {
    double v = delayed(g, rf, a, first, e, x, z);
    yt += ora_apod_weight(g, e, x, z) * sgn(v) * pow(fabs(v), 1.0 / p);
  }
  return sgn(yt) * pow(fabs(yt), p);
}

/* DAS image values. angle >= 0: that angle alone; angle == -1: the compound sum
 * over all angles. pix == NULL evaluates every pixel in [nx][nz] order; otherwise
 * pix[k] is a flat pixel index ix * nz + iz. rf is [n_angles][n_channels][n_samples]. */
int ora_das(const ora_geom *g, const double *rf, int32_t angle, const int64_t *pix, int64_t npix,
            double *out) {
  if (check(g, angle) != ORA_OK || !rf || !out) return ORA_BAD;
  int64_t total = (int64_t)g->nx * g->nz;
  if (!pix) npix = total;
  if (check_pixels(pix, npix, total) != ORA_OK) return ORA_BAD;
  double first[ORA_MAX_ANGLES];
  for (int32_t a = 0; a < g->n_angles; ++a) first[a] = first_fire(g, a);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < npix; ++k) {
    int64_t p = pix ? pix[k] : k;
    double x, z;
    pixel_xz(g, p, &x, &z);
    double y = 0.0;
    if (angle >= 0) {
      y = das_one_angle(g, rf, angle, first[angle], x, z);
    } else {
      for (int32_t a = 0; a < g->n_angles; ++a) y += das_one_angle(g, rf, a, first[a], x, z);
    }
    out[k] = y;
  }
  return ORA_OK;
}

int ora_dmas(const ora_geom *g, const double *rf, int32_t angle, int32_t form, const int64_t *pix,
             int64_t npix, double *out) {
  if (check(g, angle) != ORA_OK || !rf || !out || (form != 0 && form != 1)) return ORA_BAD;
  int64_t total = (int64_t)g->nx * g->nz;
  if (!pix) npix = total;
  if (check_pixels(pix, npix, total) != ORA_OK) return ORA_BAD;
  double first[ORA_MAX_ANGLES];
  for (int32_t a = 0; a < g->n_angles; ++a) first[a] = first_fire(g, a);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < npix; ++k) {
    int64_t p = pix ? pix[k] : k;
    double x, z;
    pixel_xz(g, p, &x, &z);
    double y = 0.0;
    if (angle >= 0) {
      y = dmas_one_angle(g, rf, angle, first[angle], x, z, form);
    } else {
      for (int32_t a = 0; a < g->n_angles; ++a)
        y += dmas_one_angle(g, rf, a, first[a], x, z, form);
    }
    out[k] = y;
  }
  return ORA_OK;
}

/* pDAS image values (Eqs. (2)-(3)) with root order p >= 1; angle and pix as for
 * ora_das; compounding sums the per-angle pDAS values. */
int ora_pdas(const ora_geom *g, const double *rf, int32_t angle, double p, const int64_t *pix,
             int64_t npix, double *out) {
  if (check(g, angle) != ORA_OK || !rf || !out || !(p >= 1.0)) return ORA_BAD;
  int64_t total = (int64_t)g->nx * g->nz;
  if (!pix) npix = total;
  if (check_pixels(pix, npix, total) != ORA_OK) return ORA_BAD;
  double first[ORA_MAX_ANGLES];
  for (int32_t a = 0; a < g->n_angles; ++a) first[a] = first_fire(g, a);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < npix; ++k) {
    int64_t q = pix ? pix[k] : k;
    double x, z;
    pixel_xz(g, q, &x, &z);
    double y = 0.0;
    if (angle >= 0) {
      y = pdas_one_angle(g, rf, angle, first[angle], x, z, p);
    } else {
      for (int32_t a = 0; a < g->n_angles; ++a) y += pdas_one_angle(g, rf, a, first[a], x, z, p);
    }
    out[k] = y;
  }
  return ORA_OK;
}

/* Delay-compensated IQ sample of element e for angle a at pixel (x, z):
 * linear interpolation of the baseband record, then the carrier phase of the
 * delay restored. */
static void iq_delayed(const ora_geom *g, const double *iq_re, const double *iq_im, double fd,
                       int32_t a, double first, int32_t e, double x, double z, double *re,
                       double *im) {
  const int64_t row = ((int64_t)a * g->n_channels + e) * g->n_samples;
  const double s = tof(g, a, first, e, x, z);
  const double vr = ora_interp(iq_re + row, g->n_samples, s);
  const double vi = ora_interp(iq_im + row, g->n_samples, s);
  const double ph = 2.0 * M_PI * fd * s / g->fs;
  const double c = cos(ph), sn = sin(ph);
  *re = vr * c - vi * sn;
  *im = vr * sn + vi * c;
}

/* IQ-DAS (form 0) or BB-DMAS (form 1), Eq. (4), for one angle; complex result. */
static void iq_one_angle(const ora_geom *g, const double *iq_re, const double *iq_im, double fd,
                         int32_t form, int32_t a, double first, double x, double z, double *yr,
                         double *yi) {
  double sr = 0.0, si = 0.0;
  for (int32_t e = 0; e < g->n_channels; ++e) {
    double vr, vi;
    iq_delayed(g, iq_re, iq_im, fd, a, first, e, x, z, &vr, &vi);
    const double w = ora_apod_weight(g, e, x, z);
    if (form == 1) {
      /* sqrt(amplitude) with the phase kept: v / sqrt|v| */
      const double amp = sqrt(vr * vr + vi * vi);
      const double k = amp > 0.0 ? 1.0 / sqrt(amp) : 0.0;
      vr *= k;
      vi *= k;
    }
    sr += w * vr;
    si += w * vi;
  }
  if (form == 1) {
    *yr = sr * sr - si * si;
    *yi = 2.0 * sr * si;
  } else {
    *yr = sr;
    *yi = si;
  }
}

/* IQ-DAS (form 0) or BB-DMAS (form 1) image values from baseband channel data
 * iq = iq_re + i iq_im, [n_angles][n_channels][n_samples], demodulated at fd;
 * angle and pix as for ora_das; complex output in out_re, out_im. */
int ora_iq(const ora_geom *g, const double *iq_re, const double *iq_im, double fd, int32_t form,
           int32_t angle, const int64_t *pix, int64_t npix, double *out_re, double *out_im) {
  if (check(g, angle) != ORA_OK || !iq_re || !iq_im || !out_re || !out_im) return ORA_BAD;
  if (form != 0 && form != 1) return ORA_BAD;
  int64_t total = (int64_t)g->nx * g->nz;
  if (!pix) npix = total;
  if (check_pixels(pix, npix, total) != ORA_OK) return ORA_BAD;
  double first[ORA_MAX_ANGLES];
  for (int32_t a = 0; a < g->n_angles; ++a) first[a] = first_fire(g, a);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < npix; ++k) {
    int64_t q = pix ? pix[k] : k;
    double x, z;
    pixel_xz(g, q, &x, &z);
    double yr = 0.0, yi = 0.0;
    for (int32_t a = 0; a < g->n_angles; ++a) {
      if (angle >= 0 && a != angle) continue;
      double ar, ai;
      iq_one_angle(g, iq_re, iq_im, fd, form, a, first[a], x, z, &ar, &ai);
      yr += ar;
      yi += ai;
    }
    out_re[k] = yr;
    out_im[k] = yi;
  }
  return ORA_OK;
}
