// Host side of the f-k migrations (Section II-B): validation, workspace layout
// and the per-angle constants, taken in float64 and split once into float-float
// pairs.
//
// Stolt's: per steering angle th the exploding-reflector velocity is
// v = c / (sqrt2 cos^2 th) and an output pixel (x0, z0) reads the migrated image
// at (x0 + z0 tan th, sqrt2 z0 / cos th): the exploding-reflector hyperbola of
// that velocity then has the apex position, apex time and apex curvature of the
// plane-wave travel time of a scatterer at (x0, z0).
//
// Lu's: the exact plane-wave relation between the data spectrum and the image
// spectrum; the time origin is the moment the transmitted wave crosses the first
// element, the migrated image lies on true coordinates (x1 = x0, z1 = z0 on the
// grid x_first + e p, l c / (2 fs)), and the array is padded to 4 N because the
// remap reads the spatial spectrum at fractional bins.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "../../include/pwbf.h"
#include "fk.h"
#include "frame_max.h"
#include "plan_host.h"

namespace pwbf {
int api_set_error(int code, const std::string &msg);
void api_clear_error();
}  // namespace pwbf

using pwbf::api_set_error;

namespace {

int log2_exact(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return (1 << l) == n ? l : -1;
}

struct FkShape {
  int log2nt, log2nx, nt, nx, kbins;
  double pitch;
};

int fk_shape(const pwbf_geometry *g, int method, FkShape *s, std::string *err) {
  int rc = pwbf::validate_geometry(g, err);
  if (rc) return rc;
  if (method != pwbf::kFkStolt && method != pwbf::kFkLu) {
    *err = "method must be PWBF_FK_STOLT or PWBF_FK_LU";
    return PWBF_E_INVALID;
  }
  const int n = g->n_channels, ns = g->n_samples;
  if (n < 2) {
    *err = "f-k migration needs at least 2 channels";
    return PWBF_E_UNSUPPORTED;
  }
  s->log2nt = log2_exact(ns);
  if (s->log2nt < 1 || ns > pwbf::kFkMaxSamples) {
    *err = "f-k migration needs n_samples a power of two in 2.." +
           std::to_string(pwbf::kFkMaxSamples) + " (n_samples = " + std::to_string(ns) + ")";
    return PWBF_E_UNSUPPORTED;
  }
  s->nt = ns;
  s->nx = 1;
  while (s->nx < (method == pwbf::kFkLu ? 4 : 2) * n) s->nx *= 2;
  s->log2nx = log2_exact(s->nx);
  if (s->nx > pwbf::kFkMaxNx) {
    *err = "f-k migration: padded array length exceeds " + std::to_string(pwbf::kFkMaxNx);
    return PWBF_E_UNSUPPORTED;
  }
  s->kbins = ns / 2 + 1;
  // pixel indices enter the map as exact float32 integers
  if (g->nx > (1 << 24) || g->nz > (1 << 24)) {
    *err = "f-k migration needs nx and nz <= 2^24";
    return PWBF_E_UNSUPPORTED;
  }
  // the spatial transform needs a uniform pitch
  const double p = (g->elem_x[n - 1] - g->elem_x[0]) / (n - 1);
  if (!(p > 0)) {
    *err = "f-k migration needs elem_x increasing with a uniform pitch";
    return PWBF_E_UNSUPPORTED;
  }
  for (int e = 0; e < n; ++e)
    if (std::fabs(g->elem_x[e] - (g->elem_x[0] + e * p)) > 1e-6 * p) {
      *err = "f-k migration needs a uniform pitch (elem_x[" + std::to_string(e) + "] is off)";
      return PWBF_E_UNSUPPORTED;
    }
  s->pitch = p;
  return PWBF_OK;
}

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

// workspace: [max slots | T | P | U | M | envelope scratch], complex float32 for
// the A angles of the call: T [A][Kb][N][R] (Kb R = Nt/2 + 1 rounded up to a
// multiple of R = 4096 / Nx), P [A][Nt/2 + 1][Nx], U [A][Nx][Nt/2 + 1],
// M [A][Nx][Nt] (P is [A][Nx][Nt/2 + 1] for Stolt's method)
struct FkLayout {
  size_t T, P, U, M, env, total;
};

FkLayout fk_layout(const pwbf_geometry *g, const FkShape &s, const pwbf_outputs *o, int n_ang) {
  FkLayout L;
  const size_t npix = (size_t)g->nx * g->nz;
  L.T = pwbf::kMaxSlotBytes;
  L.P = L.T + round256((size_t)n_ang * g->n_channels * pwbf::fk_kbins_padded(s.log2nt, s.log2nx) * 8);
  L.U = L.P + round256((size_t)n_ang * s.kbins * s.nx * 8);
  L.M = L.U + round256((size_t)n_ang * s.nx * s.kbins * 8);
  L.env = L.M + round256((size_t)n_ang * s.nx * s.nt * 8);
  L.total = L.env + ((o && o->logimg && !o->env) ? round256(npix * 4) : 0);
  return L;
}

int check_outputs(const pwbf_geometry *g, const pwbf_outputs *o, std::string *err) {
  if (!o) {
    *err = "outputs is NULL";
    return PWBF_E_INVALID;
  }
  if (!o->rf) {
    *err = "outputs->rf is NULL";
    return PWBF_E_INVALID;
  }
  for (const float *p : {o->rf, o->filtered, o->env, o->logimg, o->imag})
    if (p && (uintptr_t)p % 4) {
      *err = "output plane not 4-byte aligned";
      return PWBF_E_INVALID;
    }
  if (o->filtered || g->bandpass) {
    *err = "band-pass does not apply to the f-k image (its magnitude is the envelope)";
    return PWBF_E_INVALID;
  }
  return PWBF_OK;
}

void split(double v, float *hi, float *lo) { pwbf::split_double(v, hi, lo); }

// The window [lo, lo + n) of indices that bilinear taps at positions
// v0 + i di + k dk (0 <= i < ni, 0 <= k < nk) can reach inside [0, size): the
// floor of the extreme positions, one more for the upper tap, and one more on
// each side for the rounding of the device's float-float positions.
void tap_window(double v0, double di, int ni, double dk, int nk, int size, int32_t *lo,
                int32_t *n) {
  double vmin = v0, vmax = v0;
  for (double v : {v0 + (ni - 1) * di, v0 + (nk - 1) * dk, v0 + (ni - 1) * di + (nk - 1) * dk}) {
    vmin = std::min(vmin, v);
    vmax = std::max(vmax, v);
  }
  const double a = std::max(0.0, std::floor(vmin) - 1.0);
  const double b = std::min((double)(size - 1), std::floor(vmax) + 2.0);
  if (!(a <= b)) {
    *lo = 0;
    *n = 0;
    return;
  }
  *lo = (int32_t)a;
  *n = (int32_t)(b - a) + 1;
}

}  // namespace

extern "C" {

size_t pwbf_fk_workspace_bytes(const pwbf_geometry *g, int32_t method, int32_t angle,
                               const pwbf_outputs *out) {
  pwbf::api_clear_error();
  std::string err;
  FkShape s;
  int rc = fk_shape(g, method, &s, &err);
  if (rc) {
    api_set_error(rc, err);
    return 0;
  }
  if (angle < -1 || angle >= g->n_angles) {
    api_set_error(PWBF_E_INVALID, "angle must be -1 (all) or in 0..n_angles-1");
    return 0;
  }
  return fk_layout(g, s, out, angle < 0 ? g->n_angles : 1).total;
}

int pwbf_fk_migrate(const pwbf_geometry *g, const void *rf, int32_t rf_dtype, int32_t method,
                    int32_t angle, const pwbf_outputs *out, void *workspace,
                    size_t workspace_bytes, void *stream) {
  pwbf::api_clear_error();
  std::string err;
  FkShape s;
  int rc = fk_shape(g, method, &s, &err);
  if (rc) return api_set_error(rc, err);
  if (rf_dtype != pwbf::kI16 && rf_dtype != pwbf::kF16 && rf_dtype != pwbf::kF32)
    return api_set_error(PWBF_E_INVALID, "rf_dtype must be PWBF_I16, PWBF_F16 or PWBF_F32");
  const size_t esz = pwbf::dtype_bytes(rf_dtype);
  if (!rf || (uintptr_t)rf % esz)
    return api_set_error(PWBF_E_INVALID, "rf is NULL or not aligned to its element size");
  if (angle < -1 || angle >= g->n_angles)
    return api_set_error(PWBF_E_INVALID, "angle must be -1 (all) or in 0..n_angles-1");
  rc = check_outputs(g, out, &err);
  if (rc) return api_set_error(rc, err);
  const int a0 = angle < 0 ? 0 : angle, n_ang = angle < 0 ? g->n_angles : 1;
  const FkLayout L = fk_layout(g, s, out, n_ang);
  if (!workspace || (uintptr_t)workspace % 256)
    return api_set_error(PWBF_E_INVALID, "workspace is NULL or not 256-byte aligned");
  if (workspace_bytes < L.total)
    return api_set_error(PWBF_E_INVALID, "workspace " + std::to_string(workspace_bytes) +
                                             " bytes < " + std::to_string(L.total) + " required");

  char *ws = (char *)workspace;
  const int n = g->n_channels;
  const double fs = g->fs, c = g->c, nt = s.nt, p = s.pitch, xf = g->elem_x[0];
  pwbf::FkPlan F = {};
  F.rf = (const char *)rf + (size_t)a0 * n * s.nt * esz;
  F.dtype = rf_dtype;
  F.method = method;
  F.n_ang = n_ang;
  F.n_ch = n;
  F.log2nt = s.log2nt;
  F.log2nx = s.log2nx;
  F.nx_img = g->nx;
  F.nz_img = g->nz;
  F.T = (float2 *)(ws + L.T);
  F.P = (float2 *)(ws + L.P);
  F.U = (float2 *)(ws + L.U);
  F.M = (float2 *)(ws + L.M);
  F.out_rf = out->rf;
  F.out_imag = out->imag;
  F.out_env = out->env ? out->env : (out->logimg ? (float *)(ws + L.env) : nullptr);
  F.ws_max = out->logimg ? (uint32_t *)ws : nullptr;
  for (int k = 0; k < n_ang; ++k) {
    const int a = a0 + k;
    const double th = g->angle_rad[a], sn = std::sin(th), cs = std::cos(th);
    const double t0 = g->t0 ? g->t0[a] : 0.0;
    // firing delay of element e on the uniform array: (xf + e p) sin th - min, over c
    const double fmin = std::min(xf * sn, (xf + (n - 1) * p) * sn);
    pwbf::FkAngleConst &A = F.ang[k];
    if (method == pwbf::kFkLu) {
      // every trace shifted to the moment the wave crosses the first element
      split(((xf * sn - fmin) / c - t0) * fs / nt, &A.c0_hi, &A.c0_lo);
      split(0.0, &A.c1_hi, &A.c1_lo);
      const double beta = c * nt / (2.0 * fs * s.nx * p);  // c / (2 df Nx p)
      split(beta, &A.m0_hi, &A.m0_lo);
      split(sn, &A.m1_hi, &A.m1_lo);
      split(cs, &A.m2_hi, &A.m2_lo);
      split(sn / (2.0 * beta), &A.m3_hi, &A.m3_lo);
      // true coordinates: column (x - x_first) / p, row z / (c / (2 fs))
      const double kz = 2.0 * fs / c;
      split((g->x0 - xf) / p, &A.ux0_hi, &A.ux0_lo);
      split(g->dx / p, &A.uxi_hi, &A.uxi_lo);
      split(0.0, &A.uxk_hi, &A.uxk_lo);
      split(g->z0 * kz, &A.uz0_hi, &A.uz0_lo);
      split(g->dz * kz, &A.uzk_hi, &A.uzk_lo);
      tap_window((g->x0 - xf) / p, g->dx / p, g->nx, 0.0, g->nz, s.nx, &A.col0, &A.ncol);
      tap_window(g->z0 * kz, 0.0, g->nx, g->dz * kz, g->nz, s.nt, &A.row0, &A.nrow);
      continue;
    }
    const double v = c / (std::sqrt(2.0) * cs * cs);
    split(((xf * sn - fmin) / c - t0) * fs / nt, &A.c0_hi, &A.c0_lo);
    split(p * sn / c * fs / nt, &A.c1_hi, &A.c1_lo);
    split(v * nt / (s.nx * p * fs), &A.m0_hi, &A.m0_lo);
    // column: (x + z tan th - x_first) / p; row: sqrt2 z / cos th / (v / fs)
    const double tn = std::tan(th), kz = std::sqrt(2.0) / cs / (v / fs);
    split((g->x0 + g->z0 * tn - xf) / p, &A.ux0_hi, &A.ux0_lo);
    split(g->dx / p, &A.uxi_hi, &A.uxi_lo);
    split(g->dz * tn / p, &A.uxk_hi, &A.uxk_lo);
    split(g->z0 * kz, &A.uz0_hi, &A.uz0_lo);
    split(g->dz * kz, &A.uzk_hi, &A.uzk_lo);
    tap_window((g->x0 + g->z0 * tn - xf) / p, g->dx / p, g->nx, g->dz * tn / p, g->nz, s.nx,
               &A.col0, &A.ncol);
    tap_window(g->z0 * kz, 0.0, g->nx, g->dz * kz, g->nz, s.nt, &A.row0, &A.nrow);
  }
  int ncol_max = 0;
  for (int k = 0; k < n_ang; ++k) {
    pwbf::FkAngleConst &A = F.ang[k];
    if (A.ncol == 0 || A.nrow == 0) A.ncol = A.nrow = 0;  // no pixel reads this angle
    ncol_max = std::max(ncol_max, (int)A.ncol);
  }
  hipError_t e = pwbf::launch_fk(F, ncol_max, (hipStream_t)stream);
  const size_t npix = (size_t)g->nx * g->nz;
  if (e == hipSuccess && out->logimg)
    e = pwbf::launch_logc(F.out_env, out->logimg, F.ws_max, npix, (float)g->log_floor_db,
                          (hipStream_t)stream);
  if (e != hipSuccess)
    return api_set_error(PWBF_E_DEVICE, std::string("f-k launch: ") + hipGetErrorString(e));
  return PWBF_OK;
}

}  // extern "C"
