// Host-side validation and plan construction (no HIP calls).
//
// Everything a kernel needs is derived here in double precision and rounded
// once to float32 in sample units. The LDS window length per (channel, angle)
// comes from a bound on how far a tile's delays can spread:
//   - the transmit term X sin(th) + Z cos(th) is linear, so over a tile of
//     TX x TZ pixels it spans |sin th| (TX-1) DX + |cos th| (TZ-1) DZ;
//   - the receive term is a Euclidean distance, 1-Lipschitz in the pixel
//     position, so it spans at most the tile diagonal.
// The kernel starts each window at floor(min transmit) - 1 plus
// floor(min receive) - 1, so every interpolation pair of every pixel of the
// tile lies inside ceil(spread) + 6 entries (rounded up to a multiple of 4).
#include "frame_max_layout.h"
#include "plan_host.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>

namespace pwbf {

namespace {

bool finite(double v) { return std::isfinite(v); }

int fail(std::string *err, int code, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
int fail(std::string *err, int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (err) *err = buf;
  return code;
}

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// v as a float-float pair: hi = v rounded to float, lo = the rest rounded.
void split(double v, float *hi, float *lo) {
  *hi = (float)v;
  *lo = (float)(v - (double)*hi);
}

}  // namespace

void split_double(double v, float *hi, float *lo) { split(v, hi, lo); }

size_t dtype_bytes(int dtype) { return dtype == kC32 ? 8 : (dtype == kF32 ? 4 : 2); }

int validate_geometry(const pwbf_geometry *g, std::string *err) {
  if (!g) return fail(err, PWBF_E_INVALID, "geometry is NULL");
  if (g->abi_version != PWBF_ABI_VERSION)
    return fail(err, PWBF_E_INVALID, "geometry abi_version %u != library %u", g->abi_version,
                PWBF_ABI_VERSION);
  if (g->n_angles < 1 || g->n_angles > kMaxAngles)
    return fail(err, g->n_angles < 1 ? PWBF_E_INVALID : PWBF_E_UNSUPPORTED,
                "n_angles %d outside 1..%d", g->n_angles, kMaxAngles);
  if (g->n_channels < 1 || g->n_channels > kMaxChannels)
    return fail(err, g->n_channels < 1 ? PWBF_E_INVALID : PWBF_E_UNSUPPORTED,
                "n_channels %d outside 1..%d", g->n_channels, kMaxChannels);
  if (g->n_samples < 2) return fail(err, PWBF_E_INVALID, "n_samples %d < 2", g->n_samples);
  if (g->n_samples >= (1 << 24))
    return fail(err, PWBF_E_UNSUPPORTED, "n_samples %d > 2^24 - 1", g->n_samples);
  // sample indices into the RF array are 32-bit in the kernels
  if ((int64_t)g->n_angles * g->n_channels * g->n_samples >= ((int64_t)1 << 31))
    return fail(err, PWBF_E_UNSUPPORTED, "RF of %d x %d x %d samples exceeds 2^31 - 1",
                g->n_angles, g->n_channels, g->n_samples);
  if (!g->elem_x || !g->angle_rad) return fail(err, PWBF_E_INVALID, "elem_x or angle_rad NULL");
  for (int e = 0; e < g->n_channels; ++e)
    if (!finite(g->elem_x[e])) return fail(err, PWBF_E_INVALID, "elem_x[%d] not finite", e);
  for (int a = 0; a < g->n_angles; ++a) {
    double th = g->angle_rad[a];
    if (!finite(th) || !(std::fabs(th) < M_PI / 2))
      return fail(err, PWBF_E_INVALID, "angle_rad[%d] = %g not in (-pi/2, pi/2)", a, th);
    if (g->t0 && !finite(g->t0[a])) return fail(err, PWBF_E_INVALID, "t0[%d] not finite", a);
  }
  if (!(g->c > 0) || !finite(g->c)) return fail(err, PWBF_E_INVALID, "c must be > 0");
  if (!(g->fs > 0) || !finite(g->fs)) return fail(err, PWBF_E_INVALID, "fs must be > 0");
  if (g->nx < 1 || g->nz < 1) return fail(err, PWBF_E_INVALID, "grid %d x %d", g->nx, g->nz);
  if ((int64_t)g->nx * g->nz > (int64_t)1 << 30)
    return fail(err, PWBF_E_UNSUPPORTED, "grid larger than 2^30 pixels");
  if (!(g->dx > 0) || !(g->dz > 0) || !finite(g->dx) || !finite(g->dz) || !finite(g->x0) ||
      !finite(g->z0))
    return fail(err, PWBF_E_INVALID, "grid origin/pitch invalid (dx, dz must be > 0)");
  if (g->apod != kHann && g->apod != kBoxcar && g->apod != kNone)
    return fail(err, PWBF_E_INVALID, "apod %d unknown", g->apod);
  if (g->apod != kNone && (!(g->f_number > 0) || !finite(g->f_number)))
    return fail(err, PWBF_E_INVALID, "f_number must be > 0");
  if (g->bandpass != 0 && g->bandpass != 1)
    return fail(err, PWBF_E_INVALID, "bandpass must be 0 or 1");
  if (!(g->log_floor_db < 0) || !finite(g->log_floor_db))
    return fail(err, PWBF_E_INVALID, "log_floor_db must be < 0");
  if (g->reserved != 0) return fail(err, PWBF_E_INVALID, "reserved must be 0");
  if (g->iq_decimation != 0 && g->iq_decimation != 1 && g->iq_decimation != 2 &&
      g->iq_decimation != 4 && g->iq_decimation != 8)
    return fail(err, PWBF_E_INVALID, "iq_decimation %d not in {0, 1, 2, 4, 8}", g->iq_decimation);
  if (g->n_samples % iq_decimation(g) || g->n_samples / iq_decimation(g) < 2)
    return fail(err, PWBF_E_INVALID, "n_samples %d not a multiple of iq_decimation %d (with "
                "at least 2 decimated samples)", g->n_samples, g->iq_decimation);
  // float32 delays lose precision far from the origin: bound the largest
  // sample position any pixel can reach.
  double scale = g->fs / g->c;
  double xmax = 0, zmax = std::max(std::fabs(g->z0), std::fabs(g->z0 + (g->nz - 1) * g->dz));
  for (double x : {g->x0, g->x0 + (g->nx - 1) * g->dx})
    for (int e = 0; e < g->n_channels; ++e) xmax = std::max(xmax, std::fabs(x - g->elem_x[e]));
  double smax = (2 * zmax + 2 * xmax) * scale;
  for (int a = 0; a < g->n_angles; ++a) {
    if (g->t0) smax += std::fabs(g->t0[a]) * g->fs;
  }
  if (smax >= (double)(1 << 20))
    return fail(err, PWBF_E_UNSUPPORTED,
                "delays reach %.0f samples; float32 delays need < 2^20", smax);
  // the pitches bound the window of a tile even where the grid is one pixel
  // wide or deep (the delay bound above does not see them then)
  if (g->dx * scale >= (double)(1 << 20) || g->dz * scale >= (double)(1 << 20))
    return fail(err, PWBF_E_UNSUPPORTED, "pixel pitch of %.3g x %.3g samples exceeds 2^20",
                g->dx * scale, g->dz * scale);
  return PWBF_OK;
}

static bool post_requested(const pwbf_outputs *o) {
  return o->filtered || o->env || o->logimg;
}

size_t workspace_bytes(const pwbf_geometry *g, const pwbf_outputs *o) {
  if (!o || !o->logimg) return 0;
  size_t b = kMaxSlotBytes;  // the frame maximum's slots, then the envelope if not an output
  if (!o->env) b += (size_t)g->nx * g->nz * sizeof(float);
  return b;
}

int validate_outputs(const pwbf_geometry *g, const pwbf_outputs *o, void *ws, size_t ws_bytes,
                     std::string *err, int mode) {
  if (!o) return fail(err, PWBF_E_INVALID, "outputs is NULL");
  if (!o->rf) return fail(err, PWBF_E_INVALID, "outputs->rf is NULL");
  const float *planes[5] = {o->rf, o->filtered, o->env, o->logimg, o->imag};
  for (const float *p : planes)
    if (p && ((uintptr_t)p % 4)) return fail(err, PWBF_E_INVALID, "output plane not 4-byte aligned");
  if (is_iq_mode(mode)) {
    // the complex image's magnitude is the envelope: no depth post-processing
    if (o->filtered || g->bandpass)
      return fail(err, PWBF_E_INVALID, "band-pass applies to RF images, not to the IQ modes");
  } else if (o->imag) {
    return fail(err, PWBF_E_INVALID, "imag output is for the IQ modes only");
  }
  if (o->filtered && !g->bandpass)
    return fail(err, PWBF_E_INVALID, "filtered output requested without bandpass");
  if (!is_iq_mode(mode) && (post_requested(o) || g->bandpass)) {
    if (!is_pow2(g->nz) || g->nz > kMaxNzPost || g->nz < 2)
      return fail(err, PWBF_E_UNSUPPORTED,
                  "depth post-processing needs nz a power of two in 2..%d (nz = %d)", kMaxNzPost,
                  g->nz);
  }
  if (g->bandpass) {
    if (!(g->f0 > 0) || !finite(g->f0)) return fail(err, PWBF_E_INVALID, "bandpass needs f0 > 0");
    double dz_max = g->c / (12.0 * g->f0);
    if (g->dz > dz_max * (1 + 1e-9))
      return fail(err, PWBF_E_UNSUPPORTED,
                  "bandpass [f0, 3 f0] needs dz <= c / (12 f0) = %.4g m (dz = %.4g m)", dz_max,
                  g->dz);
  }
  size_t need = workspace_bytes(g, o);
  if (need) {
    if (!ws) return fail(err, PWBF_E_INVALID, "workspace of %zu bytes required", need);
    if (ws_bytes < need)
      return fail(err, PWBF_E_INVALID, "workspace %zu bytes < %zu required", ws_bytes, need);
    if ((uintptr_t)ws % 256) return fail(err, PWBF_E_INVALID, "workspace not 256-byte aligned");
  }
  return PWBF_OK;
}

// Default launch shape. Tiles are 16 pixels deep: the LDS window of a tile
// grows as ~2 DZ TZ + DX (1 + |sin|) TX samples, which for a fixed pixel count
// is smallest near TZ = 16 on the usual grids (dz ~ dx), and shallow tiles keep
// the per-pixel delay offsets small, which keeps float32 delays accurate. A
// wavefront covers 8 x 8 pixels (2 x 4 wavefronts per 16 x 32 tile): its lanes'
// delays then span fewer window entries per gather than a 16 x 4 column
// layout (~10% faster with an earlier kernel; with the current one the two
// shapes time within 0.5% on every benchmark workload). Small frames split channels
// across lane groups so there are enough waves.
pwbf_tile default_tile(const pwbf_geometry *g, int n_angles_used, int mode) {
  (void)mode;
  (void)n_angles_used;
  pwbf_tile t;
  int64_t pixels = (int64_t)g->nx * g->nz;
  t.cpw = pixels >= 256 * 1024 ? 1 : (pixels >= 64 * 1024 ? 2 : 4);
  // one group: 8 x 8 pixels per wavefront. A narrower tile reaches fewer
  // channels (its active aperture is the pixels' apertures widened by the
  // tile's width): from a million pixels on, 4 x 2 wavefronts (a tile 32
  // pixels deep and 16 wide; on the 11-angle 1024 x 1024 frame 4-6% faster
  // than 16 x 32: DAS 104 against 110 us, pDAS 215 against 225 us); below,
  // 2 x 2 (16 x 16, twice the blocks; on the 512 x 512 frame 3-5% faster than
  // 32 x 16: DMAS 17.2 against 17.9 us, DAS 14.8 against 15.4 us).
  t.lz = t.cpw == 1 ? 8 : 16;
  t.wz = t.cpw == 1 ? (pixels >= 1024 * 1024 ? 4 : 2) : 1;
  t.wx = t.cpw == 1 ? 2 : 8;
  t.chunk = 0;
  return t;
}

// Window length for TZ x TX tiles, and the offsets that centre the transmit and
// receive window delays on zero (the kernel reads entry n + off_t + off_r).
static int window_entries(FramePlan &p, int TZ, int TX) {
  double rt = 0;
  for (int a = 0; a < p.n_angles; ++a) {
    double v = std::fabs((double)p.sa[a]) * (TX - 1) * p.DX +
               std::fabs((double)p.ca[a]) * (TZ - 1) * p.DZ;
    rt = std::max(rt, v);
  }
  double rr = std::hypot((TX - 1) * (double)p.DX, (TZ - 1) * (double)p.DZ);
  // window delays relative to the origin lie in [1, r + 2) for each term
  p.off_t = (int)std::floor(rt / 2) + 1;
  p.off_r = (int)std::floor(rr / 2) + 1;
  // a multiple of 4: the staging threads write four entries at a time
  return ((int)std::ceil(rt + rr) + 6 + 3) & ~3;
}

// Wavefronts of a tile, without overflow for any field values.
static int64_t tile_waves(const pwbf_tile &t) { return (int64_t)t.wz * t.wx; }

// The bound on a root-mode gather's offset from its wavefront's reference
// pixel (plan.h), in samples, for lane groups of lz x lx pixels.
static double root_offset_samples(const pwbf_geometry *g, const FramePlan &P, int lz, int lx) {
  double smax = 0.0;
  for (int a = 0; a < P.n_angles; ++a) smax = std::max(smax, std::fabs((double)P.sa[a]));
  const double sphi =
      g->apod == kNone ? 1.0 : 1.0 / std::sqrt(1.0 + 4.0 * g->f_number * g->f_number);
  const double hz = (lz / 2) * std::fabs((double)P.DZ), hx = (lx / 2) * std::fabs((double)P.DX);
  return 2.0 * hz + hx * (smax + sphi);
}

bool root_compact(const pwbf_geometry *g, const FramePlan &P) {
  return !wave_ref_mode(P.mode) || root_offset_samples(g, P, P.lz, P.lx) <= kRootOffsetAuto;
}

// Apply launch shape t to plan P (geometry already filled in): window length,
// channels per LDS chunk. PWBF_E_UNSUPPORTED when even cpw channels do not fit.
static int fit_tile(const pwbf_geometry *g, pwbf_tile t, FramePlan *P, std::string *err) {
  if (t.cpw != 1 && t.cpw != 2 && t.cpw != 4 && t.cpw != 8 && t.cpw != 16)
    return fail(err, PWBF_E_INVALID, "tile.cpw %d not in {1, 2, 4, 8, 16}", t.cpw);
  const int ppw = kWave / t.cpw;
  if (t.lz < 1 || t.lz > ppw || (t.lz & (t.lz - 1)))
    return fail(err, PWBF_E_INVALID, "tile.lz %d not a power of two in 1..%d", t.lz, ppw);
  if (t.wz < 1 || t.wx < 1 || tile_waves(t) > kMaxWavesPerBlock)
    return fail(err, PWBF_E_INVALID, "tile %d x %d wavefronts outside 1..%d", t.wz, t.wx,
                kMaxWavesPerBlock);
  if (t.chunk < 0 || t.chunk % t.cpw)
    return fail(err, PWBF_E_INVALID, "tile.chunk %d not a non-negative multiple of cpw",
                t.chunk);
  P->cpw = t.cpw;
  P->lz = t.lz;
  P->lx = ppw / t.lz;
  P->wz = t.wz;
  P->wx = t.wx;
  const int TZ = P->lz * t.wz, TX = P->lx * t.wx;
  P->tile_z = TZ;
  P->tile_x = TX;
  // a tile's pixels never extend past the grid (edge lanes repeat the edge pixel)
  P->win = window_entries(*P, std::min(TZ, g->nz), std::min(TX, g->nx));
  int wmax = max_window(P->mode);
  // IQ modes: a delay rounding of d samples turns the carrier's phase by
  // 2 pi r d (r = f0 / fs in cycles per record sample), so above a quarter
  // cycle per sample (decimated records) the windows shrink to keep r times
  // the window within 16, the 64-entry limit's product at r = 1/4 (decimated
  // BB-DMAS at r = 1 with 48- and 56-entry windows measured 1.5e-5 and 2.0e-5)
  if (is_iq_mode(P->mode) && P->iq_r > 0.25f)
    wmax = std::min(wmax, std::max(4, (int)(16.0f / P->iq_r) / 4 * 4));
  if (P->win > wmax)
    return fail(err, PWBF_E_UNSUPPORTED,
                "tile of %d x %d pixels needs LDS windows of %d entries (limit %d for this "
                "beamformer, which keeps float32 delay offsets under %d samples); use a "
                "shallower or narrower tile",
                TZ, TX, P->win, wmax, wmax / 2);
  const size_t per_channel = (size_t)P->n_angles * (P->win * P->entry_bytes + 8) +
                             (is_iq_mode(P->mode) ? 24 : 16) +
                             (wave_ref_mode(P->mode) ? (size_t)t.wz * t.wx * 16 : 0);
  const size_t fixed = kLdsAngleBytes + 16;
  int chunk = t.chunk;
  if (chunk == 0) {
    // as many channels as the default budget holds (each tile walks only its
    // own active aperture, so the chunks start wherever that begins)
    const int fit = (int)((kDefaultLdsBytes - fixed) / per_channel) / t.cpw * t.cpw;
    const int nch = (g->n_channels + t.cpw - 1) / t.cpw * t.cpw;
    chunk = std::max(t.cpw, std::min(fit, nch));
  }
  P->chunk = chunk;
  if (P->chunk < t.cpw || plan_lds_bytes(*P) > (size_t)kMaxLdsBytes)
    return fail(err, PWBF_E_UNSUPPORTED,
                "tile needs %zu bytes of LDS per block (limit %d); use a smaller tile",
                plan_lds_bytes(*P), kMaxLdsBytes);
  return PWBF_OK;
}

static int plan_frame_uncached(const pwbf_geometry *g, int dtype, int mode, int angle,
                               const pwbf_tile *tile_in, FramePlan *P, std::string *err,
                               int waves) {
  int rc = validate_geometry(g, err);
  if (rc) return rc;
  // Decimated baseband records are records of the decimated rate: sample m of
  // one is at time t0 + m D / fs, so the IQ beamformers are planned with fs / D
  // and n_samples / D (delays, windows and the carrier phase per sample all
  // follow from those)
  pwbf_geometry gd;
  if (is_iq_mode(mode) && iq_decimation(g) > 1) {
    gd = *g;
    gd.fs = g->fs / iq_decimation(g);
    gd.n_samples = g->n_samples / iq_decimation(g);
    gd.iq_decimation = 1;
    g = &gd;
  }
  if (dtype != kI16 && dtype != kF16 && dtype != kF32 && dtype != kC32)
    return fail(err, PWBF_E_INVALID, "rf_dtype %d unknown", dtype);
  if (mode < kDas || mode > kBbdmas) return fail(err, PWBF_E_INVALID, "mode %d unknown", mode);
  if (is_iq_mode(mode) != (dtype == kC32))
    return fail(err, PWBF_E_INVALID, "the IQ modes take complex IQ input (PWBF_C32), the others RF");
  if (is_iq_mode(mode) && !(g->f0 > 0.0 && finite(g->f0)))
    return fail(err, PWBF_E_INVALID, "the IQ modes need f0 > 0 (the demodulation frequency)");
  if (mode == kPdas && !(g->pdas_p >= 1.0 && finite(g->pdas_p)))
    return fail(err, PWBF_E_INVALID, "pdas_p = %g must be a finite number >= 1", g->pdas_p);
  // A root steeper than the square root amplifies the float32 delay rounding
  // near zero crossings of the delayed samples past the 1e-5 agreement with the
  // definition (measured: p = 3 reaches 1.03e-5), so the kernels take 1 <= p <= 2.
  if (mode == kPdas && g->pdas_p > 2.0)
    return fail(err, PWBF_E_UNSUPPORTED, "pdas_p = %g above 2 (the kernels take 1 <= p <= 2)",
                g->pdas_p);
  if (angle < -1 || angle >= g->n_angles)
    return fail(err, PWBF_E_INVALID, "angle %d outside 0..%d", angle, g->n_angles - 1);
  if (mode == kDmas && g->n_channels < 2)
    return fail(err, PWBF_E_INVALID, "DMAS needs at least 2 channels");
  // the kernels address the RF bytes with 32-bit buffer offsets
  if ((int64_t)g->n_angles * g->n_channels * g->n_samples * (int64_t)dtype_bytes(dtype) >=
      ((int64_t)1 << 31))
    return fail(err, PWBF_E_UNSUPPORTED, "RF buffer of 2^31 bytes or more");

  std::memset(P, 0, sizeof *P);
  const double scale = g->fs / g->c;
  const int a0 = angle < 0 ? 0 : angle;
  const int na = angle < 0 ? g->n_angles : 1;
  P->dtype = dtype;
  P->mode = mode;
  P->apod = g->apod;
  P->n_angles = na;
  P->n_channels = g->n_channels;
  P->n_samples = g->n_samples;
  P->nx = g->nx;
  P->nz = g->nz;
  split(g->x0 * scale, &P->X0, &P->X0l);
  split(g->dx * scale, &P->DX, &P->DXl);
  split(g->z0 * scale, &P->Z0, &P->Z0l);
  split(g->dz * scale, &P->DZ, &P->DZl);
  P->ap_k = g->apod == kNone ? 0.0f : (float)(2.0 * g->f_number);
  P->pdas_p = mode == kPdas ? (float)g->pdas_p : 1.0f;
  P->pdas_inv_p = mode == kPdas ? (float)(1.0 / g->pdas_p) : 1.0f;
  P->entry_bytes = is_iq_mode(mode) ? 16 : 8;
  if (is_iq_mode(mode)) split(g->f0 / g->fs, &P->iq_r, &P->iq_rl);
  for (int e = 0; e < kMaxChannels; ++e)
    split(g->elem_x[std::min(e, g->n_channels - 1)] * scale, &P->xe[e], &P->xel[e]);
  for (int k = 0; k < na; ++k) {
    int a = a0 + k;
    double th = g->angle_rad[a];
    double first = g->elem_x[0] * std::sin(th);
    for (int e = 1; e < g->n_channels; ++e) first = std::min(first, g->elem_x[e] * std::sin(th));
    split(std::sin(th), &P->sa[k], &P->sal[k]);
    split(std::cos(th), &P->ca[k], &P->cal[k]);
    split(first * scale + (g->t0 ? g->t0[a] : 0.0) * g->fs, &P->to[k], &P->tol[k]);
  }

  // An explicit tile is taken as given; an absent or all-zero tile takes the
  // tuned entry for this shape if there is one and it fits, else the default;
  // when that does not fit (LDS or window length), the fitting shape with the
  // most pixels per tile, then the shortest window, then the fewest lane groups.
  pwbf_tile d = default_tile(g, na, mode);
  // Batch and serving kernels (8-wavefront plans) take their tiles in cost
  // order across frames instead of the single-frame kernel's depth-ordered,
  // XCD-balanced order; there the 16 x 32 tile is the faster one (8 compound
  // frames per launch: 9586 against 9355 frames/s for 32 x 16).
  if (waves && d.cpw == 1) {
    d.wz = 2;
    d.wx = 4;
  }
  const bool zero_tile = tile_in && !tile_in->cpw && !tile_in->lz && !tile_in->wz &&
                         !tile_in->wx && !tile_in->chunk;
  if (zero_tile) tile_in = nullptr;
  int rc_fit = PWBF_OK;
  const char *source = "explicit";
  if (tile_in) {
    pwbf_tile t = *tile_in;
    if (t.cpw == 0) t.cpw = d.cpw;
    if (t.lz == 0) t.lz = std::min(d.lz, kWave / t.cpw);
    if (t.wz == 0 && t.wx == 0) {
      t.wz = d.wz;
      t.wx = d.wx;
    }
    if (waves && tile_waves(t) != waves)
      return fail(err, PWBF_E_INVALID, "batch tiles need wz * wx = %d (got %d x %d)", waves,
                  t.wz, t.wx);
    rc_fit = fit_tile(g, t, P, err);
  } else {
    pwbf_tile tuned;
    bool done = false;
    if (tune_lookup(shape_key(g, dtype, mode, angle, waves), &tuned) &&
        (!waves || tile_waves(tuned) == waves))
      done = fit_tile(g, tuned, P, err) == PWBF_OK && root_compact(g, *P);
    source = "tuned";
    if (!done && (!waves || d.wz * d.wx == waves)) {
      done = fit_tile(g, d, P, err) == PWBF_OK && root_compact(g, *P);
      source = "default";
      if (!done && d.cpw == 1) {
        // one tile's window can pass the limit where the other orientation
        // fits (pixels much deeper or wider than each other, in samples)
        pwbf_tile other = d;
        std::swap(other.wz, other.wx);
        done = fit_tile(g, other, P, err) == PWBF_OK && root_compact(g, *P);
      }
      // DMAS and pDAS past their delay-offset bound: the same tile in lane
      // groups half as deep and twice as wide (twice the wavefronts along
      // depth, half across). 11-angle 1024 x 1024 pDAS: 8 x 1 wavefronts of
      // 4 x 16 pixels take 0.195 ms, the 16 x 32 tile of the search below
      // 0.203 ms.
      for (pwbf_tile s = d; !done && s.cpw == 1 && s.lz > 1 && s.wx % 2 == 0;) {
        s.lz /= 2;
        s.wz *= 2;
        s.wx /= 2;
        done = fit_tile(g, s, P, err) == PWBF_OK && root_compact(g, *P);
      }
    }
    if (!done) {
      source = "fallback";
      // every shape with at least the default's lane groups and the required
      // wavefront count; the choice depends on the geometry only. Groups of 8
      // or 4 pixels (cpw 8, 16) keep windows short on grids with pixels tens of
      // samples deep, such as 32 rows over 3 cm at 50 MHz.
      static const int kArr[][2] = {{2, 4}, {1, 8}, {4, 2}, {8, 1}, {1, 4}, {2, 2},
                                    {4, 1}, {1, 2}, {2, 1}, {1, 1}};
      // (DMAS and pDAS: a shape within their delay-offset bound first)
      pwbf_tile best = {0, 0, 0, 0, 0};
      int best_px = 0, best_win = 0;
      bool best_compact = false;
      for (int cpw = d.cpw; cpw <= 16; cpw *= 2)
        for (int lz = 1; lz <= kWave / cpw; lz *= 2)
          for (const auto &wa : kArr) {
            if (waves ? wa[0] * wa[1] != waves : wa[0] * wa[1] > kMaxWavesPerBlock) continue;
            const pwbf_tile t = {cpw, lz, wa[0], wa[1], 0};
            FramePlan Q = *P;
            std::string e2;
            if (fit_tile(g, t, &Q, &e2) != PWBF_OK) continue;
            const int px = std::min(Q.tile_z, g->nz) * std::min(Q.tile_x, g->nx);
            const bool compact = root_compact(g, Q);
            if ((compact && !best_compact) ||
                (compact == best_compact &&
                 (px > best_px || (px == best_px && Q.win < best_win)))) {
              best = t;
              best_px = px;
              best_win = Q.win;
              best_compact = compact;
            }
          }
      if (best_px > 0) {
        rc_fit = fit_tile(g, best, P, err);
      } else {
        rc_fit = fail(err, PWBF_E_UNSUPPORTED,
                      "no launch shape keeps the LDS windows within %d entries on this grid "
                      "(pixel pitch %.3g x %.3g samples); use a finer grid",
                      max_window(mode), (double)P->DX, (double)P->DZ);
      }
    }
  }
  if (rc_fit) return rc_fit;
  const int TZ = P->tile_z, TX = P->tile_x;
  P->tiles_z = (g->nz + TZ - 1) / TZ;
  P->tiles_x = (g->nx + TX - 1) / TX;
  P->n_tiles = P->tiles_z * P->tiles_x;
  if (debug_enabled())
    debug_log("plan mode %d dtype %d angle %d grid %d x %d: %s shape cpw %d lz %d wz %d wx %d "
              "chunk %d, window %d, %d x %d tiles, %zu B LDS",
              mode, dtype, angle, g->nx, g->nz, source, P->cpw, P->lz, P->wz, P->wx, P->chunk,
              P->win, P->tiles_z, P->tiles_x, plan_lds_bytes(*P));
  return PWBF_OK;
}

// Plans are a pure function of the geometry (scalars and arrays), the call
// shape and the tuning table, so the last few successful ones are kept, keyed
// by those bytes; a hit skips validation and planning (a few microseconds of
// host time per call, which matters when a frame takes a few hundred).
namespace {

std::string plan_key(const pwbf_geometry *g, int dtype, int mode, int angle,
                     const pwbf_tile *tile, int waves) {
  std::string k;
  if (!g || g->n_channels < 1 || g->n_channels > kMaxChannels || g->n_angles < 1 ||
      g->n_angles > kMaxAngles || !g->elem_x || !g->angle_rad)
    return k;  // not cacheable: the uncached path reports the error
  pwbf_geometry s = *g;
  s.elem_x = nullptr;
  s.angle_rad = nullptr;
  s.t0 = nullptr;
  const int32_t head[7] = {dtype, mode, angle, waves, g->t0 ? 1 : 0, tile ? 1 : 0,
                           (int32_t)tune_generation()};
  k.reserve(sizeof s + sizeof head + sizeof(pwbf_tile) +
            sizeof(double) * (g->n_channels + 2 * g->n_angles));
  k.append((const char *)&s, sizeof s);
  k.append((const char *)head, sizeof head);
  if (tile) k.append((const char *)tile, sizeof *tile);
  k.append((const char *)g->elem_x, sizeof(double) * g->n_channels);
  k.append((const char *)g->angle_rad, sizeof(double) * g->n_angles);
  if (g->t0) k.append((const char *)g->t0, sizeof(double) * g->n_angles);
  return k;
}

constexpr int kPlanCacheSize = 16;
std::mutex g_plan_mu;
std::string g_plan_keys[kPlanCacheSize];
FramePlan g_plans[kPlanCacheSize];
int g_plan_next = 0;

}  // namespace

int plan_frame(const pwbf_geometry *g, int dtype, int mode, int angle, const pwbf_tile *tile_in,
               FramePlan *P, std::string *err, int waves) {
  const std::string key = plan_key(g, dtype, mode, angle, tile_in, waves);
  if (!key.empty()) {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    for (int i = 0; i < kPlanCacheSize; ++i)
      if (g_plan_keys[i] == key) {
        *P = g_plans[i];
        return PWBF_OK;
      }
  }
  const int rc = plan_frame_uncached(g, dtype, mode, angle, tile_in, P, err, waves);
  if (rc == PWBF_OK && !key.empty()) {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    g_plan_keys[g_plan_next] = key;
    g_plans[g_plan_next] = *P;
    g_plan_next = (g_plan_next + 1) % kPlanCacheSize;
  }
  return rc;
}

int build_plan(const pwbf_geometry *g, const void *rf, int dtype, int mode, int angle,
               const pwbf_tile *tile, const pwbf_outputs *o, void *ws, size_t ws_bytes,
               FramePlan *P, std::string *err) {
  int rc = plan_frame(g, dtype, mode, angle, tile, P, err);
  if (rc) return rc;
  if (!rf) return fail(err, PWBF_E_INVALID, "rf is NULL");
  if ((uintptr_t)rf % dtype_bytes(dtype))
    return fail(err, PWBF_E_INVALID, "rf not aligned to its element size");
  rc = validate_outputs(g, o, ws, ws_bytes, err, mode);
  if (rc) return rc;
  // one angle's records as the plan reads them: decimated baseband records
  // hold n_samples / D samples each, not the caller's n_samples
  const size_t slab = (size_t)g->n_channels * P->n_samples * dtype_bytes(dtype);
  P->rf = (const char *)rf + (size_t)(angle < 0 ? 0 : angle) * slab;
  P->out = o->rf;
  P->ws_max = o->logimg ? (uint32_t *)ws : nullptr;
  P->out_imag = o->imag;
  P->out_env = nullptr;
  if (is_iq_mode(mode))
    P->out_env = o->env ? o->env : (o->logimg ? (float *)((char *)ws + kMaxSlotBytes) : nullptr);
  return PWBF_OK;
}

int tile_active_channels(const pwbf_geometry *g, const FramePlan &P, int tile) {
  if (g->apod == kNone) return g->n_channels;
  const int tz = tile / P.tiles_x, tx = tile - tz * P.tiles_x;
  const double xlo = g->x0 + (double)tx * P.tile_x * g->dx;
  const double xhi = g->x0 + (double)(std::min((tx + 1) * P.tile_x, g->nx) - 1) * g->dx;
  const double zmax = g->z0 + (double)(std::min((tz + 1) * P.tile_z, g->nz) - 1) * g->dz;
  if (!(zmax > 0)) return 0;
  const double h = zmax / (2.0 * g->f_number);
  int n = 0;
  for (int e = 0; e < g->n_channels; ++e)
    n += (g->elem_x[e] > xlo - h && g->elem_x[e] < xhi + h) ? 1 : 0;
  return n;
}

void tile_channel_hull(const pwbf_geometry *g, const FramePlan &P, int tile, int *lo, int *hi) {
  // The test the kernel makes in float32, here in float64: the channels whose
  // distance to the tile's lateral span is below 1.001 Z_max / (2 F#) (any
  // channel with a nonzero weight at some pixel of the tile passes it either
  // way; the others add exact zeros, so the two hulls give the same sums).
  *lo = 0;
  *hi = g->n_channels;
  if (g->apod == kNone) return;
  const int tz = tile / P.tiles_x, tx = tile - tz * P.tiles_x;
  const double xlo = g->x0 + (double)tx * P.tile_x * g->dx;
  const double xhi = g->x0 + (double)(std::min((tx + 1) * P.tile_x, g->nx) - 1) * g->dx;
  const double zmax = g->z0 + (double)(std::min((tz + 1) * P.tile_z, g->nz) - 1) * g->dz;
  *lo = g->n_channels;
  *hi = 0;
  if (!(zmax > 0)) return;
  for (int e = 0; e < g->n_channels; ++e) {
    const double x = g->elem_x[e];
    const double d = x < xlo ? xlo - x : (x > xhi ? x - xhi : 0.0);
    if (d * 2.0 * g->f_number < zmax * 1.001) {
      *lo = std::min(*lo, e);
      *hi = std::max(*hi, e + 1);
    }
  }
}

double tile_cost(const pwbf_geometry *g, const FramePlan &P, int tile) {
  // Estimated vector lane-operations of the tile, from the kernel's instruction
  // mix: per (pixel, active channel) the receive delay, weight and its
  // per-angle gathers (DAS 5 per angle, DMAS 10, pDAS 9 at p = 2 and 12
  // otherwise; the transcendental operations issue at a quarter of the rate),
  // the window staging (about 5.5 per entry) and the per-tile constants.
  const double px = (double)P.tile_z * P.tile_x;
  const double ch = tile_active_channels(g, P, tile);
  const double A = P.n_angles;
  double per_gather = 5, per_pair = 20;
  if (P.mode == kDmas) {
    per_gather = 10;
    per_pair = 22;
  } else if (P.mode == kPdas) {
    per_gather = P.pdas_p == 2.0f ? 9 : 12;
  }
  const double staging = ch * A * P.win * 5.5;
  const double constants = A * 64 + ch * (wave_ref_mode(P.mode) ? P.wz * P.wx * 64.0 : 64.0);
  return px * ch * (A * per_gather + per_pair) + staging + constants;
}

int build_post_plan(const pwbf_geometry *g, const pwbf_outputs *o, void *ws, PostPlan *Q) {
  std::memset(Q, 0, sizeof *Q);
  Q->src = o->rf;
  Q->filtered = o->filtered;
  Q->ws_max = o->logimg ? (uint32_t *)ws : nullptr;
  Q->env = o->env ? o->env : (o->logimg ? (float *)((char *)ws + kMaxSlotBytes) : nullptr);
  Q->logimg = o->logimg;
  Q->nx = g->nx;
  Q->nz = g->nz;
  int l = 0;
  while ((1 << l) < g->nz) ++l;
  Q->log2nz = l;
  Q->bandpass = g->bandpass;
  Q->floor_db = (float)g->log_floor_db;
  if (g->bandpass) {
    // The same decision, in double, as the definition: bin k' carries the
    // round-trip frequency |k'| c / (2 nz dz); keep it when f0 <= f <= 3 f0.
    int lo = -1, hi = -2;
    for (int k = 0; k <= g->nz / 2; ++k) {
      double f = (double)k * g->c / (2.0 * g->nz * g->dz);
      if (f >= g->f0 && f <= 3.0 * g->f0) {
        if (lo < 0) lo = k;
        hi = k;
      }
    }
    Q->k_lo = lo;
    Q->k_hi = hi;
  }
  return PWBF_OK;
}

bool post_needed(const pwbf_outputs *o) { return post_requested(o); }

}  // namespace pwbf
