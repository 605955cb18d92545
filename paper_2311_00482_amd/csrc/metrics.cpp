// Host side of the image metrics: validation, discs in pixel units, launch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "../../include/pwbf.h"
#include "metrics.h"
#include "plan_host.h"

namespace pwbf {
int api_set_error(int code, const std::string &msg);
void api_clear_error();
}  // namespace pwbf

using pwbf::api_set_error;

namespace {

bool finite_disc(const pwbf_disc &d) {
  return std::isfinite(d.x) && std::isfinite(d.z) && std::isfinite(d.r) && d.r > 0;
}

}  // namespace

namespace pwbf {

// The bounding box is one pixel wider than the exact one, then clipped.
DiscPix disc_to_pixels(const pwbf_geometry *g, const pwbf_disc &d) {
  pwbf::DiscPix p;
  const double cx = (d.x - g->x0) / g->dx, cz = (d.z - g->z0) / g->dz;
  p.cx = (float)cx;
  p.cz = (float)cz;
  p.sx = (float)(g->dx / d.r);
  p.sz = (float)(g->dz / d.r);
  const double hx = d.r / g->dx, hz = d.r / g->dz;
  auto clampi = [](double v, int lo, int hi) {
    return (int)std::fmin(std::fmax(v, (double)lo), (double)hi);
  };
  p.ix0 = clampi(std::floor(cx - hx) - 1, 0, g->nx - 1);
  p.ix1 = clampi(std::ceil(cx + hx) + 1, 0, g->nx - 1);
  p.iz0 = clampi(std::floor(cz - hz) - 1, 0, g->nz - 1);
  p.iz1 = clampi(std::ceil(cz + hz) + 1, 0, g->nz - 1);
  if (cx + hx < -1 || cx - hx > g->nx || cz + hz < -1 || cz - hz > g->nz) {
    p.ix0 = 0;  // entirely off the grid: an empty box
    p.ix1 = -1;
  }
  return p;
}

}  // namespace pwbf

namespace {

int check_common(const pwbf_geometry *g, const float *env, int32_t n, const void *regions,
                 const void *out, size_t out_align) {
  std::string err;
  int rc = pwbf::validate_geometry(g, &err);
  if (rc) return api_set_error(rc, err);
  if (!env || (uintptr_t)env % 4) return api_set_error(PWBF_E_INVALID, "env is NULL or misaligned");
  if (!regions) return api_set_error(PWBF_E_INVALID, "regions are NULL");
  if (n < 1 || n > PWBF_MAX_METRIC_REGIONS)
    return api_set_error(PWBF_E_INVALID, "n must be in 1.." +
                                             std::to_string(PWBF_MAX_METRIC_REGIONS));
  if (!out || (uintptr_t)out % out_align)
    return api_set_error(PWBF_E_INVALID, "out is NULL or misaligned");
  return PWBF_OK;
}

}  // namespace

extern "C" {

int pwbf_contrast_metrics(const pwbf_geometry *g, const float *env, const pwbf_cyst *cysts,
                          int32_t n, pwbf_contrast *out, void *stream) {
  pwbf::api_clear_error();
  int rc = check_common(g, env, n, cysts, out, 4);
  if (rc) return rc;
  pwbf::CystSet cs = {};
  for (int k = 0; k < n; ++k) {
    if (!finite_disc(cysts[k].in) || !finite_disc(cysts[k].out))
      return api_set_error(PWBF_E_INVALID, "cyst " + std::to_string(k) + ": bad disc");
    cs.in[k] = pwbf::disc_to_pixels(g, cysts[k].in);
    cs.out[k] = pwbf::disc_to_pixels(g, cysts[k].out);
  }
  hipError_t e = pwbf::launch_contrast(env, g->nz, cs, n, out, (hipStream_t)stream);
  if (e != hipSuccess)
    return api_set_error(PWBF_E_DEVICE, std::string("contrast launch: ") + hipGetErrorString(e));
  return PWBF_OK;
}

int pwbf_resolution_metrics(const pwbf_geometry *g, const float *env, const pwbf_disc *targets,
                            int32_t n, pwbf_resolution *out, void *stream) {
  pwbf::api_clear_error();
  int rc = check_common(g, env, n, targets, out, 4);
  if (rc) return rc;
  pwbf::TargetSet ts = {};
  for (int k = 0; k < n; ++k) {
    if (!finite_disc(targets[k]))
      return api_set_error(PWBF_E_INVALID, "target " + std::to_string(k) + ": bad disc");
    ts.t[k] = pwbf::disc_to_pixels(g, targets[k]);
  }
  hipError_t e = pwbf::launch_resolution(env, g->nx, g->nz, (float)g->dx, (float)g->dz, ts, n,
                                         out, (hipStream_t)stream);
  if (e != hipSuccess)
    return api_set_error(PWBF_E_DEVICE, std::string("resolution launch: ") + hipGetErrorString(e));
  return PWBF_OK;
}

}  // extern "C"
