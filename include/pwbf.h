/* pwbf.h - plane-wave receive beamformer for MI355X (gfx950), C ABI.
 *
 * The library computes, for every pixel of a 2-D grid, the delay-and-sum of
 * the paper's Eq. (1) over the receive channels of a linear array insonified by
 * steered plane waves, and the RF delay-multiply-and-sum variant built on the
 * squared-sum structure of Eq. (4) with the signed-root compression of Eq. (2);
 * optional depth-wise post-processing gives the band-passed image, the envelope
 * (magnitude of the analytic signal) and the log-compressed image displayed at
 * -70 dB (Fig. 3).
 *
 * Conventions shared by every entry point
 *  - RF is one contiguous device buffer RF[n_angles][n_channels][n_samples],
 *    sample index fastest, stored as int16, IEEE binary16 or float32
 *    (pwbf_dtype). Sample n of angle a was acquired at time t0[a] + n / fs.
 *  - Elements lie on z = 0 at elem_x[e]. A steered plane wave of angle theta
 *    leaves the first-firing element at time 0. The sample position of pixel
 *    (x, z) for element e and angle a is
 *       s = fs * ((x sin th + z cos th - min_k x_k sin th) / c
 *                 + sqrt((x - x_e)^2 + z^2) / c - t0[a]),
 *    which at th = 0 is the transmit depth plus the receive path; the paper's
 *    delay text after Eq. (1) is the same receive path.
 *  - The delayed sample is the linear interpolation between samples floor(s)
 *    and floor(s) + 1, with the record taken as zero outside [0, n_samples).
 *  - Receive apodization (the paper's predefined weights w_i[p]): Hann over a
 *    half-aperture z / (2 F#), w = 0.5 (1 + cos(pi |x - x_e| / a)) for
 *    |x - x_e| < a and z > 0, else 0; or boxcar, or none (w = 1).
 *  - Images are float32 [nx][nz], depth fastest. Pixel (ix, iz) is centred at
 *    (x0 + ix dx, z0 + iz dz).
 *  - All arithmetic on the GPU is float32 (no float64 on the device). Geometry
 *    is taken in float64 on the host and rounded once to float32 in sample units.
 *  - Every call validates its arguments on the host before any HIP call; on a
 *    validation error nothing is enqueued and nothing is written. Work is
 *    enqueued on the caller's HIP stream (NULL = the null stream) and the call
 *    returns once it is enqueued. Device faults surface at the caller's next
 *    synchronisation. No single-frame call allocates or frees device memory,
 *    keeps a pointer after it returns, prints (unless PWBF_DEBUG is set), or
 *    throws (the batch, tuning and serving objects below own memory and say
 *    so). Calls on different streams from different threads may overlap; calls
 *    that share a workspace must not.
 *  - Return value: PWBF_OK (0) or a negative PWBF_E_* code; pwbf_last_error()
 *    gives a thread-local description of the last failure on the calling thread.
 *
 * Environment (read once, at first use)
 *  - PWBF_DEBUG=1: every launch shape the planner picks (and whether it came
 *    from the caller, the tuning table, the default or the fallback search) and
 *    every error a call returns are printed to stderr as "pwbf: ..." lines.
 *    Unset or "0": the library prints nothing.
 *  - PWBF_TUNE_CACHE=<path>: the tuning table starts from that file (the format
 *    of pwbf_tune_save) when it exists, and each shape pwbf_tune measures is
 *    written back to it at once (through a side file and a rename).
 *  - PWBF_BATCH_BRANCHES=1..4: the branches of a batch graph (default 3).
 *  - PWBF_SERVE_INFLIGHT=1..4: the batches a server keeps on the device at
 *    once (default 4), read when the server is created.
 */
#ifndef PWBF_H
#define PWBF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PWBF_ABI_VERSION 6u

#ifndef PWBF_API
#define PWBF_API __attribute__((visibility("default")))
#endif

#define PWBF_OK 0
#define PWBF_E_INVALID (-1)     /* bad pointer, size, enum or geometry */
#define PWBF_E_UNSUPPORTED (-2) /* valid but outside what the kernels handle */
#define PWBF_E_NOMEM (-3)       /* host or device allocation failed (batch objects only) */
#define PWBF_E_DEVICE (-4)      /* a HIP runtime call failed */

/* Storage type of the RF samples. */
#define PWBF_I16 0
#define PWBF_F16 1
#define PWBF_F32 2
#define PWBF_C32 3 /* complex float32 (re, im interleaved): baseband IQ samples */

/* Beamformer. */
#define PWBF_DAS 0
#define PWBF_DMAS 1
#define PWBF_PDAS 2
#define PWBF_IQDAS 3  /* DAS on IQ data (input PWBF_C32) */
#define PWBF_BBDMAS 4 /* BB-DMAS on IQ data, Eq. (4) (input PWBF_C32) */

/* Apodization. */
#define PWBF_APOD_HANN 0
#define PWBF_APOD_BOXCAR 1
#define PWBF_APOD_NONE 2

/* Library limits. */
#define PWBF_MAX_ANGLES 32
#define PWBF_MAX_CHANNELS 256
#define PWBF_MAX_NZ_POST 4096 /* longest depth column the post-processing handles */
/* Longest LDS window per (channel, angle) of a launch shape, in samples. The
 * DAS, IQ-DAS and BB-DMAS kernels hold every per-gather delay as a float32
 * offset centred on its tile's window, so the delay's rounding grows with the
 * window. 64 entries keep those offsets under 32 samples (2^-19 of a sample
 * resolution), which holds them within 1e-5 of the float64 definition
 * (max-normalised). In the IQ modes a delay rounding of d samples also turns
 * the carrier's phase by 2 pi r d, r = f0 / fs in cycles per record sample
 * (f0 D / fs for records decimated by D), so there the limit is
 * min(64, 16 / r) entries, rounded down to a multiple of 4: 32 at D = 2 and
 * 16 at D = 4 for f0 = fs / 4. DMAS and pDAS measure delays from their
 * wavefront's centre pixel (below). A tile's window spans
 * about |sin th| TX DX + |cos th| TZ DZ + hypot(TX DX, TZ DZ) + 6 samples (DX,
 * DZ: pixel pitches times fs / c); explicit shapes needing more are refused
 * with PWBF_E_UNSUPPORTED, and default plans pick a smaller tile. A grid whose
 * pixels are so coarse that no shape fits (a tile of one 2 x 2-pixel lane
 * group needs DZ + hypot(DX, DZ) + 6 within the limit) is refused the same
 * way. */
#define PWBF_MAX_WINDOW 64
/* DMAS and pDAS take each delay relative to their wavefront's centre pixel.
 * The shapes the library picks itself (default, fallback, tuner) keep every
 * gather within 4 samples of that pixel's delay whenever some shape does:
 * 2 (lz / 2) DZ + (lx / 2) DX (max |sin th| + 1 / sqrt(1 + 4 F#^2)) <= 4 for
 * lane groups of lz x lx pixels (halves rounded down; the last term 1 without
 * apodization), which bounds the float32 rounding of their delays. Explicit
 * shapes are taken as given. */

/* Acquisition and grid. Host pointers are read during the call only. */
typedef struct pwbf_geometry {
  uint32_t abi_version;     /* must be PWBF_ABI_VERSION */
  int32_t n_angles;         /* 1 .. PWBF_MAX_ANGLES */
  int32_t n_channels;       /* 1 .. PWBF_MAX_CHANNELS (>= 2 for DMAS) */
  int32_t n_samples;        /* 2 .. 2^24 - 1; n_angles * n_channels * n_samples < 2^31 */
  const double *elem_x;     /* host [n_channels], element centres, m */
  const double *angle_rad;  /* host [n_angles], steering angles, |th| < pi/2 */
  const double *t0;         /* host [n_angles], s, time of sample 0; NULL = all 0 */
  double c;                 /* speed of sound, m/s, > 0 */
  double fs;                /* sampling rate, Hz, > 0 */
  double f0;                /* centre frequency, Hz (band-pass only) */
  int32_t nx, nz;           /* grid size, >= 1 each */
  double x0, dx;            /* centre of column 0 and lateral pitch, m (dx > 0) */
  double z0, dz;            /* centre of row 0 and depth pitch, m (dz > 0) */
  double f_number;          /* > 0 for Hann and boxcar */
  int32_t apod;             /* PWBF_APOD_* */
  int32_t bandpass;         /* 1: keep round-trip band [f0, 3 f0] along depth before
                               the envelope (needs dz <= c / (12 f0)); 0: none */
  double log_floor_db;      /* floor of the log image, dB, < 0 (e.g. -70) */
  double pdas_p;            /* root order p of pDAS, 1 .. 2 (PWBF_PDAS only; else ignored) */
  int32_t iq_decimation;    /* baseband records keep every D-th sample: 0 or 1 (none), 2, 4
                               or 8; n_samples divisible by D (IQ calls only; else ignored) */
  int32_t reserved;         /* 0 */
} pwbf_geometry;

/* Output planes, each a device float32 [nx][nz] buffer owned by the caller.
 * rf is required; the others may be NULL. filtered needs bandpass = 1. The
 * envelope and the log image are taken from the band-passed image when
 * bandpass = 1, else from rf. For the IQ modes the image is complex: rf holds
 * its real part, imag its imaginary part, env its magnitude (the displayed
 * image of Eq. (4)); filtered must be NULL. */
typedef struct pwbf_outputs {
  float *rf;       /* beamformed image: DAS sum, raw DMAS or pDAS; real part (IQ modes) */
  float *filtered; /* band-passed image */
  float *env;      /* envelope along depth; |image| (IQ modes) */
  float *logimg;   /* 20 log10(env / max env), clipped at log_floor_db */
  float *imag;     /* imaginary part of the image (IQ modes only), or NULL */
} pwbf_outputs;

/* Launch shape of the beamforming kernel. Zeros select the library default.
 * A wavefront (64 lanes) holds cpw lane groups; each group covers the same
 * lz (depth) x (64 / cpw / lz) (lateral) pixels and sums its share of the
 * channels, and the groups are reduced in-wave. A tile (one block) is wz x wx
 * wavefronts, i.e. lz * wz pixels along depth by (64 / cpw / lz) * wx along x.
 * Its LDS windows must fit PWBF_MAX_WINDOW entries (PWBF_E_UNSUPPORTED
 * otherwise). */
typedef struct pwbf_tile {
  int32_t cpw;   /* lane groups per wavefront: 1, 2, 4, 8 or 16 */
  int32_t lz;    /* lanes of a group along depth: a power of two <= 64 / cpw */
  int32_t wz;    /* wavefronts stacked along depth in a tile */
  int32_t wx;    /* wavefronts side by side along x in a tile; wz * wx in 1..8 */
  int32_t chunk; /* channels staged in LDS at a time (0 = as many as fit) */
} pwbf_tile;

/* ABI version of the loaded library (PWBF_ABI_VERSION). */
PWBF_API uint32_t pwbf_abi_version(void);

/* Thread-local text of the last error on this thread ("" if none). Valid until
 * the next pwbf_* call on the same thread. */
PWBF_API const char *pwbf_last_error(void);

/* Bytes of device workspace the calls below need for these outputs (0 when no
 * log image is requested). Returns 0 and sets the last error on invalid input. */
PWBF_API size_t pwbf_workspace_bytes(const pwbf_geometry *g, const pwbf_outputs *out);

/* Delay-and-sum for one steering angle: Eq. (1), y[p] = sum_e w_e[p] u_e(s_e[p]).
 *  rf        device RF[n_angles][n_channels][n_samples] of rf_dtype; slab `angle` is used
 *  angle     0 .. n_angles - 1
 *  out       output planes (see pwbf_outputs)
 *  workspace device buffer of at least pwbf_workspace_bytes(g, out) bytes, or NULL
 *            when that is 0; the call overwrites it
 *  stream    hipStream_t as void*, NULL for the null stream
 * Errors: PWBF_E_INVALID, PWBF_E_UNSUPPORTED, PWBF_E_DEVICE. */
PWBF_API int pwbf_beamform_das(const pwbf_geometry *g, const void *rf, int32_t rf_dtype, int32_t angle,
                      const pwbf_outputs *out, void *workspace, size_t workspace_bytes,
                      void *stream);

/* RF delay-multiply-and-sum for one angle: with s_e = w_e sign(v_e) sqrt|v_e| for
 * the delayed samples v_e (the weight outside the root, as in Eq. (2)),
 * y = sum_{e<f} s_e s_f, computed as ((sum_e s_e)^2 - sum_e s_e^2) / 2 (the
 * squared-sum form of Eq. (4) without its 1/N). Arguments and errors as for
 * pwbf_beamform_das; needs n_channels >= 2. */
PWBF_API int pwbf_beamform_dmas(const pwbf_geometry *g, const void *rf, int32_t rf_dtype,
                       int32_t angle, const pwbf_outputs *out, void *workspace,
                       size_t workspace_bytes, void *stream);

/* pDAS for one angle, Eqs. (2)-(3): the delayed samples are compressed to
 * w_e sign(v_e) |v_e|^(1/p) (p = g->pdas_p), summed, and the sum restored by
 * its signed p-th power, y = sign(t) |t|^p. p = 1 is DAS. The paper gives no p;
 * the kernels take 1 <= p <= 2 (PWBF_E_INVALID below 1 or not finite,
 * PWBF_E_UNSUPPORTED above 2: a root steeper than the square root amplifies the
 * float32 delay rounding near zero crossings of the delayed samples past 1e-5
 * of the definition). Arguments and other errors as for pwbf_beamform_das. */
PWBF_API int pwbf_beamform_pdas(const pwbf_geometry *g, const void *rf, int32_t rf_dtype,
                                int32_t angle, const pwbf_outputs *out, void *workspace,
                                size_t workspace_bytes, void *stream);

/* Baseband (IQ) channel data, the demodulation and decimation of the IQ path
 * of Section II-B: for every record RF[a][e][:], the analytic signal (one-sided
 * spectrum along samples: 1 at DC and Nyquist, 2 on positive bins, 0 on
 * negative ones) times exp(-2 pi i f0 n / fs), sample n of the record. With
 * g->iq_decimation = D > 1 the analytic spectrum first keeps only the positive
 * bins within fs / (2 D) of f0 (an ideal low-pass of the baseband signal to the
 * decimated rate's band), and the record keeps samples n = 0, D, 2D, ...
 *  rf   device RF[n_angles][n_channels][n_samples] of rf_dtype (int16, FP16, FP32)
 *  iq   device complex float32 [n_angles][n_channels][n_samples / D] (8 bytes
 *       per sample, re then im), owned by the caller, 8-byte aligned; overwritten
 * Needs n_samples a power of two in 2..4096 and f0 > 0 (PWBF_E_UNSUPPORTED /
 * PWBF_E_INVALID). No workspace; enqueued on stream. The IQ beamformers read
 * such records with the same geometry (D included). */
PWBF_API int pwbf_iq_demodulate(const pwbf_geometry *g, const void *rf, int32_t rf_dtype,
                                void *iq, void *stream);

/* DAS on IQ data for one angle: with q_e the baseband record of element e
 * interpolated linearly at the delay s_e and rotated back by exp(2 pi i f0 s_e / fs)
 * (a record decimated by D is read at s_e / D, its own sample rate),
 * y = sum_e w_e q_e (Eq. (1) on the delay-compensated IQ signals). iq from
 * pwbf_iq_demodulate (rf_dtype PWBF_C32). Outputs: rf = Re y, imag = Im y,
 * env = |y|, logimg from env; bandpass must be 0 and filtered NULL. */
PWBF_API int pwbf_beamform_iqdas(const pwbf_geometry *g, const void *iq, int32_t angle,
                                 const pwbf_outputs *out, void *workspace,
                                 size_t workspace_bytes, void *stream);

/* BB-DMAS for one angle, Eq. (4): y = (sum_e w_e sqrt(a_e) exp(i phi_e))^2 with
 * a_e exp(i phi_e) = q_e the delay-compensated IQ sample (the weight outside the
 * root as in Eq. (2); the constant 1/N of Eq. (4) is dropped). The image is |y|
 * (env). Arguments and outputs as for pwbf_beamform_iqdas. */
PWBF_API int pwbf_beamform_bbdmas(const pwbf_geometry *g, const void *iq, int32_t angle,
                                  const pwbf_outputs *out, void *workspace,
                                  size_t workspace_bytes, void *stream);

/* Image metrics of the evaluation (Section II-D) on an envelope image env,
 * device float32 [nx][nz] of the grid in g (any plane of the calls above).
 * Regions are discs (centre x, z and radius r in m); a pixel belongs to a disc
 * when ((ix - cx) sx)^2 + ((iz - cz) sz)^2 <= 1 in separately rounded float32
 * operations, with cx = (x - x0)/dx, cz = (z - z0)/dz, sx = dx/r, sz = dz/r
 * rounded to float32 once. Results go to caller-owned device memory; at most
 * PWBF_MAX_METRIC_REGIONS cysts or targets per call. */
#define PWBF_MAX_METRIC_REGIONS 32

typedef struct pwbf_disc {
  double x, z, r; /* centre and radius, m (r > 0) */
} pwbf_disc;

typedef struct pwbf_cyst {
  pwbf_disc in;  /* inside the cyst */
  pwbf_disc out; /* background */
} pwbf_cyst;

typedef struct pwbf_contrast {
  float mu_in, mu_out;       /* mean envelope inside / background */
  float sigma_in, sigma_out; /* population standard deviations */
  float cr_db;               /* Eq. (5): 20 log10(mu_in / mu_out) */
  float cnr;                 /* Eq. (6), denominator read as sqrt((sigma_in^2 + sigma_out^2) / 2) */
  int32_t n_in, n_out;       /* pixels in each disc (NaN statistics when 0) */
} pwbf_contrast;

typedef struct pwbf_resolution {
  float peak;           /* envelope maximum in the target disc (first flat index on ties) */
  float fwhm_x, fwhm_z; /* full widths at half the peak (-6.02 dB) of the lateral and axial
                           profiles through the peak, m, crossings interpolated linearly
                           between pixels; NaN when a side never falls below half */
  int32_t ix, iz;       /* pixel of the peak; -1 when the disc holds no pixel */
} pwbf_resolution;

/* CR and CNR (Eqs. (5)-(6)) for n cysts; out: device pwbf_contrast[n]. */
PWBF_API int pwbf_contrast_metrics(const pwbf_geometry *g, const float *env,
                                   const pwbf_cyst *cysts, int32_t n, pwbf_contrast *out,
                                   void *stream);

/* FWHM of n point targets (the peak is searched inside each target disc);
 * out: device pwbf_resolution[n]. */
PWBF_API int pwbf_resolution_metrics(const pwbf_geometry *g, const float *env,
                                     const pwbf_disc *targets, int32_t n, pwbf_resolution *out,
                                     void *stream);

/* f-k migrations of steered plane waves: Stolt's (reflector model) and Lu's
 * (scattering model), both listed among the beamformers of Section II-B without
 * formulas, so what follows is the reading the library implements. Per angle th,
 * with Nt = n_samples, p the (uniform) element pitch, k = f / c and all
 * wavenumbers in cycles per metre:
 *  1. temporal spectrum of every trace (e^{-2 pi i f t}), bins f_k = k fs / Nt for
 *     0 <= k <= Nt / 2, times exp(2 pi i f_k (tau - t0[a])); Stolt: tau = tau_e,
 *     the element's firing delay (x_e sin th - min_k x_k sin th) / c; Lu: tau =
 *     tau_0, the moment the wave crosses the first element, for every trace;
 *  2. spectrum along the array zero-padded to Nx, the power of two >= 2 N
 *     (Stolt) or >= 4 N (Lu, whose remap reads it at fractional bins);
 *     kx_m = m / (Nx p), signed;
 *  3. remap onto the image spectrum, the one-sided data spectrum extended by zeros
 *     past bin Nt / 2 and read by linear interpolation:
 *     Stolt: v = c / (sqrt2 cos^2 th); the image spectrum at (kx, kz_j =
 *     j fs / (Nt v)) is the data at f = v sqrt(kx^2 + kz^2), times
 *     kz / sqrt(kx^2 + kz^2) (0 at the origin);
 *     Lu: the image spectrum at (kx', kz'_j = 2 j fs / (Nt c)) is the data at
 *     k = (kx'^2 + kz'^2) / (2 (kx' sin th + kz' cos th)), kx = kx' - k sin th
 *     (bilinear, periodic in the spatial bin), times kz_r / (kx' sin th +
 *     kz' cos th) with kz_r = kz' - k cos th; zero where kz_r < 0 or the
 *     denominator is <= 0;
 *  4. inverse transforms along kx (Nx) and along kz with the one-sided spectrum
 *     zero-filled to Nt, scaled by 1 / (Nx Nt): the complex migrated image on
 *     x1 = elem_x[0] + e' p and z1 = l v / fs (Stolt) or l c / (2 fs) (Lu);
 *  5. output pixel (x, z) takes that image bilinearly (zero outside) at
 *     (x + z tan th, sqrt2 z / cos th) (Stolt: v and this map put the migrated
 *     point where the plane-wave travel-time curve has its apex, with matching
 *     curvature) or at (x, z) (Lu); angles add (complex).
 *  rf        device RF[n_angles][n_channels][n_samples] (int16, FP16 or FP32)
 *  method    PWBF_FK_STOLT or PWBF_FK_LU
 *  angle     0..n_angles-1, or -1 for the sum over all angles
 *  out       rf = real part, imag = imaginary part, env = magnitude (the image),
 *            logimg from env; filtered must be NULL and bandpass 0
 *  workspace device, 256-byte aligned, >= pwbf_fk_workspace_bytes(g, method,
 *            angle, out) bytes: the spectra and migrated images of every angle
 *            of the call (8 N Kb + 16 (Nt/2 + 1) Nx + 8 Nx Nt bytes per angle,
 *            Kb = Nt/2 + 1 rounded up to a multiple of 4096 / Nx: 19 MB (Stolt)
 *            or 36 MB (Lu) per angle at 128 channels x 4096 samples)
 * Needs n_channels >= 2 with a uniform pitch (within 1e-6 p; the element
 * positions used are elem_x[0] + e p), n_samples a power of two in 2..4096, and
 * nx, nz <= 2^24 (PWBF_E_UNSUPPORTED otherwise). apod and f_number are unused. Work is enqueued
 * on stream. pwbf_fk_workspace_bytes returns 0 (and sets the last error) when the
 * call is not supported. */
#define PWBF_FK_STOLT 0
#define PWBF_FK_LU 1
PWBF_API size_t pwbf_fk_workspace_bytes(const pwbf_geometry *g, int32_t method, int32_t angle,
                                        const pwbf_outputs *out);
PWBF_API int pwbf_fk_migrate(const pwbf_geometry *g, const void *rf, int32_t rf_dtype,
                             int32_t method, int32_t angle, const pwbf_outputs *out,
                             void *workspace, size_t workspace_bytes, void *stream);

/* Coherent compounding: the unweighted sum over all n_angles of the per-angle
 * DAS (mode PWBF_DAS), DMAS (PWBF_DMAS), pDAS (PWBF_PDAS) images, or of the
 * complex IQ-DAS (PWBF_IQDAS) or BB-DMAS (PWBF_BBDMAS) values, in one pass that shares
 * each pixel's receive delays and weights across the angles. Before
 * post-processing, compound(mode) equals the sum of beamform_<mode>(a) over a
 * (up to float32 summation order). Other arguments and errors as above. */
PWBF_API int pwbf_compound(const pwbf_geometry *g, const void *rf, int32_t rf_dtype, int32_t mode,
                  const pwbf_outputs *out, void *workspace, size_t workspace_bytes,
                  void *stream);

/* pwbf_compound without a workspace argument, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation. The same kernels and results as pwbf_compound; the
 * scratch they need (the frame maximum for the log image, and the envelope
 * plane when logimg is requested without env) lives in a device array of the
 * library, one per GPU, held until the process ends: 8 KiB plus
 * PWBF_NOALLOC_ENV_PIXELS * 4 bytes (16 MiB). Its device address is looked up
 * once per device on the first call that needs it (with that device current).
 * A log image without env on a grid of more than PWBF_NOALLOC_ENV_PIXELS pixels
 * returns PWBF_E_UNSUPPORTED. The call allocates and frees nothing. Every call
 * on one GPU shares that GPU's array, which keeps the last call's contents (the
 * kernels clear what must start at zero): calls that overlap on one GPU (other
 * streams, other threads) race and must be ordered by the caller. Other
 * arguments and errors as for pwbf_compound. */
#define PWBF_NOALLOC_ENV_PIXELS (1 << 22)
PWBF_API int pwbf_compound_noalloc(const pwbf_geometry *g, const void *rf, int32_t rf_dtype,
                                   int32_t mode, const pwbf_outputs *out, void *stream);

/* pwbf_compound (angle == -1) or the single-angle call (angle >= 0) with an explicit
 * launch shape; tile == NULL behaves as the plain calls. Used by the tuner and
 * by tests that sweep launch shapes. */
PWBF_API int pwbf_beamform_ex(const pwbf_geometry *g, const void *rf, int32_t rf_dtype, int32_t mode,
                     int32_t angle, const pwbf_tile *tile, const pwbf_outputs *out,
                     void *workspace, size_t workspace_bytes, void *stream);

/* Every host-side check of pwbf_beamform_ex with the same arguments, without
 * enqueuing anything: returns what that call would return before it reaches the
 * device (PWBF_OK when the call would be enqueued). Pointers are only checked
 * for NULL and alignment, never dereferenced. */
PWBF_API int pwbf_validate_call(const pwbf_geometry *g, const void *rf, int32_t rf_dtype,
                                int32_t mode, int32_t angle, const pwbf_tile *tile,
                                const pwbf_outputs *out, const void *workspace,
                                size_t workspace_bytes);

/* The resolved launch of a beamforming call and the float32 constants its kernel
 * uses (all lengths in samples: metres * fs / c). Diagnostic: lets a caller see
 * the LDS use and tile grid, and lets tests re-derive the kernel's window bounds
 * on the CPU. */
typedef struct pwbf_plan_info {
  int32_t cpw, lz, wz, wx, chunk; /* resolved launch shape */
  int32_t tile_z, tile_x;     /* pixels of a tile along depth and x */
  int32_t win;                /* LDS entries per (channel, angle) window */
  int32_t off_t, off_r;       /* window-delay centring offsets (entries) */
  int32_t tiles_z, tiles_x;   /* tile grid */
  int32_t threads_per_block;
  int32_t blocks;             /* blocks launched (a multiple of 8) */
  int32_t n_angles_used;      /* angles the kernel sums (1 for single-angle calls) */
  int64_t lds_bytes;          /* LDS per block */
  /* Geometry constants as float-float pairs: value = hi + lo. */
  float X0, DX, Z0, DZ;       /* pixel (0, 0) centre and pitches (hi) */
  float X0l, DXl, Z0l, DZl;   /* ... lo parts */
  float ap_k;                 /* 2 F# (0 when apod is none) */
  float sa[PWBF_MAX_ANGLES], sal[PWBF_MAX_ANGLES]; /* sin(theta) per angle used */
  float ca[PWBF_MAX_ANGLES], cal[PWBF_MAX_ANGLES]; /* cos(theta) */
  float to[PWBF_MAX_ANGLES], tol[PWBF_MAX_ANGLES]; /* first-firing term + t0 * fs */
  float xe[PWBF_MAX_CHANNELS], xel[PWBF_MAX_CHANNELS]; /* element x */
} pwbf_plan_info;

/* Fill *info for a call with this geometry, mode, angle (-1 = compound) and tile
 * (NULL = default). No device work; returns PWBF_OK or a validation error. */
PWBF_API int pwbf_describe_plan(const pwbf_geometry *g, int32_t mode, int32_t angle,
                       const pwbf_tile *tile, pwbf_plan_info *info);

/* ------------------------------------------------------------------ batches
 * Frames of uneven size, channel count, angle count, storage type and mode go
 * into one graph launch: the frames are split into up to four branches of about
 * equal estimated cost, each running one beamform kernel per class of its
 * frames (one block per (frame, pixel tile) item, largest tiles first), then
 * the depth post-processing and the log image of its frames; the branches run
 * side by side. The launch sequence is captured once in a HIP graph and
 * replayed.
 * The batch keeps the frames' device pointers until it is updated or
 * destroyed; creating it allocates the graph, the descriptor tables and a
 * small per-frame workspace (PWBF_E_NOMEM on failure). Launch and update must
 * be enqueued on the same stream (or the caller orders them). */
typedef struct pwbf_frame {
  const pwbf_geometry *geom; /* host; read during create / update */
  const void *rf;            /* device RF of rf_dtype */
  int32_t rf_dtype;          /* PWBF_I16, PWBF_F16, PWBF_F32 */
  int32_t mode;              /* PWBF_DAS, PWBF_DMAS or PWBF_PDAS (the IQ modes are
                                single-frame only: PWBF_E_UNSUPPORTED) */
  int32_t angle;             /* -1: compound over all angles; else that angle */
  int32_t reserved;          /* 0 */
  pwbf_outputs out;          /* device planes, as for the single-frame calls (imag NULL) */
  pwbf_tile tile;            /* zeros: tuned entry if present, else default;
                                wz * wx must be 8 (batch blocks are 8 wavefronts) */
} pwbf_frame;

typedef struct pwbf_batch pwbf_batch;

#define PWBF_BATCH_TUNE 1 /* create: tune every shape without a tuned entry first */

typedef struct pwbf_batch_info {
  int32_t n_frames;
  int32_t n_items;          /* (frame, tile) work items */
  int32_t n_columns;        /* depth columns post-processed */
  int32_t blocks;           /* blocks launched (one per item), summed over the kernels */
  int32_t blocks_per_cu;    /* the smallest occupancy among the kernels */
  int32_t lds_bytes;        /* LDS per block of the beamform kernels */
  int32_t graph_nodes;
  int32_t kernels;          /* beamform kernel launches: one per class of frames
                               (beamformer, lane grouping, angle count 1/5/11/other)
                               in each branch */
  int32_t branches;         /* parallel branches of the graph (frames balanced by cost) */
} pwbf_batch_info;

/* Build a batch of n >= 1 frames; *out receives the handle. flags: 0 or
 * PWBF_BATCH_TUNE (tuning runs the frames on `stream`, overwriting their rf
 * outputs, and blocks until done). */
PWBF_API int pwbf_batch_create(const pwbf_frame *frames, int32_t n, int32_t flags, void *stream,
                               pwbf_batch **out);

/* Point an existing batch at new buffers: the frames must have the same
 * geometry, storage type, mode, angle selection and requested planes as at
 * creation (PWBF_E_INVALID otherwise). The new descriptors are copied on
 * `stream`, ordered before later launches on it. */
PWBF_API int pwbf_batch_update(pwbf_batch *b, const pwbf_frame *frames, int32_t n, void *stream);

/* Enqueue one execution of the batch graph on `stream`. */
PWBF_API int pwbf_batch_launch(pwbf_batch *b, void *stream);

/* Shape of the batch launch. */
PWBF_API int pwbf_batch_describe(const pwbf_batch *b, pwbf_batch_info *info);

/* Release the batch (waits for its outstanding work). NULL is ignored. */
PWBF_API int pwbf_batch_destroy(pwbf_batch *b);

/* ------------------------------------------------------------------ tuning
 * Time candidate launch shapes (lane groups, lanes along depth, wavefront
 * arrangement) for this frame and keep the fastest in the process-wide tuning
 * table, which single-frame calls with a NULL or all-zero tile and batch frames
 * consult. waves = 8 restricts to shapes the batch kernel can run; 0 allows
 * 1..8 wavefronts. Overwrites out->rf; blocks until the timing runs finish.
 * *best / *best_ms (may be NULL) receive the winner and its time. */
PWBF_API int pwbf_tune(const pwbf_geometry *g, const void *rf, int32_t rf_dtype, int32_t mode,
                       int32_t angle, const pwbf_outputs *out, int32_t waves, void *stream,
                       pwbf_tile *best, float *best_ms);

/* Persist / restore / clear the tuning table (a small JSON file of
 * shape key -> tile). Load merges into the table. */
PWBF_API int pwbf_tune_save(const char *path);
PWBF_API int pwbf_tune_load(const char *path);
PWBF_API int pwbf_tune_clear(void);

/* ------------------------------------------------------------------ serving
 * A request loop over fixed probes. Each probe (geometry, mode, angle
 * selection, output planes) owns ring slots resident in HBM: its RF stored as
 * FP16 and its output planes. submit() queues a frame of int16 RF from pinned
 * host memory; a scheduler thread admits queued requests into free slots while
 * the HBM budget ledger allows (the bytes of the slots in use), uploads them on
 * one of two copy streams (the one with fewer bytes outstanding) and converts
 * them to FP16 on the device, and, whenever fewer than four batches
 * (PWBF_SERVE_INFLIGHT) are on the GPU, launches every uploaded request as one
 * batch (continuous batching:
 * requests that arrive while others run join the next batch). A frame runs the
 * same kernels with the same plan whether it is alone or in a mix, so its
 * planes do not depend on the mix. The decisions (ledger, admission, deadlines,
 * batching) are a device-free core that the CPU tests drive with a fake clock. */
typedef struct pwbf_probe {
  const pwbf_geometry *geom; /* host; copied at creation */
  int32_t mode;              /* PWBF_DAS / PWBF_DMAS / PWBF_PDAS */
  int32_t angle;             /* -1: compound; else that angle */
  int32_t want_env;          /* 1: envelope plane */
  int32_t want_log;          /* 1: log image (implies the envelope) */
  int32_t slots;             /* ring slots (0 = 4) */
  int32_t want_quality;      /* 1: a quality check of every served frame (implies the
                                envelope): its envelope maximum and the CR and CNR
                                (Eqs. (5)-(6), Section II-D) of quality_region, with
                                quality_ok = frame maximum > 0 and CR <= quality_max_cr_db */
  pwbf_cyst quality_region;  /* inside and background discs (m), as for pwbf_contrast_metrics */
  double quality_max_cr_db;  /* e.g. -10 for an anechoic cyst */
} pwbf_probe;

typedef struct pwbf_server pwbf_server;

typedef struct pwbf_result {
  uint64_t id;            /* as returned by submit */
  int32_t probe, slot;    /* slot -1 when the request expired */
  double t_arrival;       /* seconds on the server clock (pwbf_server_now) */
  double t_admit;         /* slot assigned, upload enqueued */
  double t_launch;        /* batch enqueued */
  double t_done;          /* output planes complete on the device (or the expiry time) */
  const float *rf;        /* device planes of the slot, valid until released (NULL when
                             the request expired) */
  const float *env;
  const float *logimg;
  int32_t status;         /* PWBF_OK, or PWBF_E_TIMEOUT: not admitted by its deadline */
  int32_t quality_ok;     /* want_quality: the frame passed the probe's check (else 0) */
  float frame_max;        /* want_quality: maximum of the envelope */
  float cr_db, cnr;       /* want_quality: Eqs. (5)-(6) over the probe's quality_region */
} pwbf_result;

typedef struct pwbf_server_stats {
  int64_t submitted, rejected, completed, batches;
  int64_t queued, in_flight;   /* right now */
  double mean_batch;           /* requests per batch */
  size_t budget_bytes, budget_in_use, budget_peak;
  int64_t expired;             /* dropped at their deadline before admission */
} pwbf_server_stats;

#define PWBF_E_BUSY (-5)    /* serving: the probe's queue is full */
#define PWBF_E_TIMEOUT (-6) /* serving: the request was not admitted by its deadline */

/* Create a server for n probes. A slot of a probe costs its FP16 RF
 * (2 n_angles n_channels n_samples bytes), its float32 planes (rf, plus env
 * when want_env or want_log, plus the log image) and 256 bytes for the frame
 * maximum. hbm_budget_bytes caps the bytes of slots in use at once (0 = no cap
 * beyond the allocated rings; PWBF_E_INVALID when one slot of some probe
 * exceeds it); max_queue bounds each probe's queue of waiting requests
 * (0 = 1024). Probes are validated like single-frame calls before anything is
 * allocated (at most 16 summed angles per frame); then the rings are allocated
 * on the current device (PWBF_E_NOMEM on failure) and the scheduler thread
 * starts. The functions below may be called from any thread. */
PWBF_API int pwbf_server_create(const pwbf_probe *probes, int32_t n, size_t hbm_budget_bytes,
                                int32_t max_queue, pwbf_server **out);

/* Queue a frame for probe `probe`: host_rf is int16 RF[n_angles][n_channels][n_samples]
 * in pinned host memory, read asynchronously until the request completes.
 * t_arrival < 0 stamps the current server time. *id receives the request id.
 * PWBF_E_BUSY when the probe's queue is full (the request is dropped). */
PWBF_API int pwbf_server_submit(pwbf_server *s, int32_t probe, const int16_t *host_rf,
                                double t_arrival, uint64_t *id);

/* pwbf_server_submit with a deadline: deadline >= 0 is the server time (seconds,
 * pwbf_server_now) by which the request must be admitted; one still queued then
 * is dropped, and poll returns it with status PWBF_E_TIMEOUT and no planes (its
 * release frees nothing). deadline < 0: none. */
PWBF_API int pwbf_server_submit_ex(pwbf_server *s, int32_t probe, const int16_t *host_rf,
                                   double t_arrival, double deadline, uint64_t *id);

/* Collect up to max completed requests into results (*n receives the count),
 * waiting up to wait_ms for at least one. Their slots stay reserved until
 * pwbf_server_release. */
PWBF_API int pwbf_server_poll(pwbf_server *s, pwbf_result *results, int32_t max, int32_t *n,
                              int32_t wait_ms);

/* Free the slot of a completed request. */
PWBF_API int pwbf_server_release(pwbf_server *s, uint64_t id);

PWBF_API int pwbf_server_stats_get(pwbf_server *s, pwbf_server_stats *st);

/* Seconds on the server's steady clock. */
PWBF_API double pwbf_server_now(const pwbf_server *s);

/* Stop the scheduler, wait for the device, free everything. NULL is ignored. */
PWBF_API int pwbf_server_destroy(pwbf_server *s);

#ifdef __cplusplus
}
#endif

#endif /* PWBF_H */
