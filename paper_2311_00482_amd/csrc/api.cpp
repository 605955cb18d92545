// extern "C" entry points of libpwbf: validation, plan, enqueue.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "../../include/pwbf.h"
#include "plan_host.h"

namespace pwbf {
hipError_t launch_beamform(const FramePlan &P, hipStream_t stream);
hipError_t launch_post(const PostPlan &Q, hipStream_t stream);
hipError_t launch_logc(const float *env, float *logimg, const uint32_t *ws_max, size_t n,
                       float floor_db, hipStream_t stream);
hipError_t launch_iq_demod(const void *rf, int dtype, void *iq, int rows, int log2ns, float r_hi,
                           float r_lo, int log2d, int k_lo, int k_hi, hipStream_t stream);
}  // namespace pwbf

namespace {

thread_local std::string g_last_error;

int set_error(int code, const std::string &msg) {
  g_last_error = msg;
  if (code != PWBF_OK) pwbf::debug_log("error %d: %s", code, msg.c_str());
  return code;
}

}  // namespace

namespace pwbf {
int api_set_error(int code, const std::string &msg) { return set_error(code, msg); }
void api_clear_error() { g_last_error.clear(); }
}  // namespace pwbf

namespace pwbf {

// One single-frame call: validate, plan, enqueue (every public single-frame
// entry point, and the allocation-free one, come through here).
int run_frame(const pwbf_geometry *g, const void *rf, int32_t dtype, int32_t mode, int32_t angle,
              const pwbf_tile *tile, const pwbf_outputs *out, void *ws, size_t ws_bytes,
              void *stream) {
  g_last_error.clear();
  pwbf::FramePlan P;
  std::string err;
  int rc = pwbf::build_plan(g, rf, dtype, mode, angle, tile, out, ws, ws_bytes, &P, &err);
  if (rc) return set_error(rc, err);
  hipStream_t s = (hipStream_t)stream;
  if (pwbf::is_iq_mode(mode)) {
    // the image's magnitude comes out of the beamform kernel; only the log remains
    hipError_t e = pwbf::launch_beamform(P, s);
    if (e == hipSuccess && out->logimg)
      e = pwbf::launch_logc(P.out_env, out->logimg, P.ws_max, (size_t)g->nx * g->nz,
                            (float)g->log_floor_db, s);
    if (e != hipSuccess)
      return set_error(PWBF_E_DEVICE, std::string("IQ beamform launch: ") + hipGetErrorString(e));
    return PWBF_OK;
  }
  pwbf::PostPlan Q;
  const bool post = pwbf::post_needed(out);
  if (post) pwbf::build_post_plan(g, out, ws, &Q);
  hipError_t e = pwbf::launch_beamform(P, s);
  if (e != hipSuccess)
    return set_error(PWBF_E_DEVICE, std::string("beamform launch: ") + hipGetErrorString(e));
  if (post) {
    e = pwbf::launch_post(Q, s);
    if (e != hipSuccess)
      return set_error(PWBF_E_DEVICE, std::string("post-processing launch: ") +
                                          hipGetErrorString(e));
  }
  return PWBF_OK;
}

}  // namespace pwbf

namespace {
using pwbf::run_frame;
int run(const pwbf_geometry *g, const void *rf, int32_t dtype, int32_t mode, int32_t angle,
        const pwbf_tile *tile, const pwbf_outputs *out, void *ws, size_t ws_bytes, void *stream) {
  return run_frame(g, rf, dtype, mode, angle, tile, out, ws, ws_bytes, stream);
}
}  // namespace

extern "C" {

uint32_t pwbf_abi_version(void) { return PWBF_ABI_VERSION; }

const char *pwbf_last_error(void) { return g_last_error.c_str(); }

size_t pwbf_workspace_bytes(const pwbf_geometry *g, const pwbf_outputs *out) {
  g_last_error.clear();
  std::string err;
  int rc = pwbf::validate_geometry(g, &err);
  if (rc) {
    set_error(rc, err);
    return 0;
  }
  if (!out) {
    set_error(PWBF_E_INVALID, "outputs is NULL");
    return 0;
  }
  return pwbf::workspace_bytes(g, out);
}

int pwbf_beamform_das(const pwbf_geometry *g, const void *rf, int32_t rf_dtype, int32_t angle,
                      const pwbf_outputs *out, void *workspace, size_t workspace_bytes,
                      void *stream) {
  if (angle < 0) return set_error(PWBF_E_INVALID, "angle must be >= 0");
  return run(g, rf, rf_dtype, pwbf::kDas, angle, nullptr, out, workspace, workspace_bytes,
             stream);
}

int pwbf_beamform_dmas(const pwbf_geometry *g, const void *rf, int32_t rf_dtype, int32_t angle,
                       const pwbf_outputs *out, void *workspace, size_t workspace_bytes,
                       void *stream) {
  if (angle < 0) return set_error(PWBF_E_INVALID, "angle must be >= 0");
  return run(g, rf, rf_dtype, pwbf::kDmas, angle, nullptr, out, workspace, workspace_bytes,
             stream);
}

int pwbf_beamform_pdas(const pwbf_geometry *g, const void *rf, int32_t rf_dtype, int32_t angle,
                       const pwbf_outputs *out, void *workspace, size_t workspace_bytes,
                       void *stream) {
  if (angle < 0) return set_error(PWBF_E_INVALID, "angle must be >= 0");
  return run(g, rf, rf_dtype, pwbf::kPdas, angle, nullptr, out, workspace, workspace_bytes,
             stream);
}

int pwbf_beamform_iqdas(const pwbf_geometry *g, const void *iq, int32_t angle,
                        const pwbf_outputs *out, void *workspace, size_t workspace_bytes,
                        void *stream) {
  if (angle < 0) return set_error(PWBF_E_INVALID, "angle must be >= 0");
  return run(g, iq, pwbf::kC32, pwbf::kIqdas, angle, nullptr, out, workspace, workspace_bytes,
             stream);
}

int pwbf_beamform_bbdmas(const pwbf_geometry *g, const void *iq, int32_t angle,
                         const pwbf_outputs *out, void *workspace, size_t workspace_bytes,
                         void *stream) {
  if (angle < 0) return set_error(PWBF_E_INVALID, "angle must be >= 0");
  return run(g, iq, pwbf::kC32, pwbf::kBbdmas, angle, nullptr, out, workspace, workspace_bytes,
             stream);
}

int pwbf_iq_demodulate(const pwbf_geometry *g, const void *rf, int32_t rf_dtype, void *iq,
                       void *stream) {
  g_last_error.clear();
  std::string err;
  int rc = pwbf::validate_geometry(g, &err);
  if (rc) return set_error(rc, err);
  if (rf_dtype != pwbf::kI16 && rf_dtype != pwbf::kF16 && rf_dtype != pwbf::kF32)
    return set_error(PWBF_E_INVALID, "rf_dtype must be PWBF_I16, PWBF_F16 or PWBF_F32");
  if (!rf || (uintptr_t)rf % pwbf::dtype_bytes(rf_dtype))
    return set_error(PWBF_E_INVALID, "rf is NULL or not aligned to its element size");
  if (!iq || (uintptr_t)iq % 8) return set_error(PWBF_E_INVALID, "iq is NULL or not 8-byte aligned");
  const int ns = g->n_samples;
  if (ns < 2 || ns > 4096 || (ns & (ns - 1)))
    return set_error(PWBF_E_UNSUPPORTED, "IQ demodulation needs n_samples a power of two in 2..4096");
  if (!(g->f0 > 0.0) || !std::isfinite(g->f0))
    return set_error(PWBF_E_INVALID, "IQ demodulation needs f0 > 0");
  int log2ns = 0;
  while ((1 << log2ns) < ns) ++log2ns;
  float r_hi, r_lo;
  pwbf::split_double(g->f0 / g->fs, &r_hi, &r_lo);
  // decimation by D: the positive bins whose frequency lies within fs / (2 D)
  // of the demodulation frequency f0 (a contiguous range, decided in double)
  const int D = pwbf::iq_decimation(g);
  int log2d = 0, k_lo = 1, k_hi = 0;
  while ((1 << log2d) < D) ++log2d;
  if (D > 1) {
    k_lo = ns;
    k_hi = -1;
    for (int k = 0; k <= ns / 2; ++k)
      if (std::fabs((double)k * g->fs / ns - g->f0) < g->fs / (2.0 * D)) {
        k_lo = std::min(k_lo, k);
        k_hi = std::max(k_hi, k);
      }
  }
  hipError_t e = pwbf::launch_iq_demod(rf, rf_dtype, iq, g->n_angles * g->n_channels, log2ns, r_hi,
                                       r_lo, log2d, k_lo, k_hi, (hipStream_t)stream);
  if (e != hipSuccess)
    return set_error(PWBF_E_DEVICE, std::string("IQ demodulation launch: ") + hipGetErrorString(e));
  return PWBF_OK;
}

int pwbf_compound(const pwbf_geometry *g, const void *rf, int32_t rf_dtype, int32_t mode,
                  const pwbf_outputs *out, void *workspace, size_t workspace_bytes,
                  void *stream) {
  return run(g, rf, rf_dtype, mode, -1, nullptr, out, workspace, workspace_bytes, stream);
}

int pwbf_beamform_ex(const pwbf_geometry *g, const void *rf, int32_t rf_dtype, int32_t mode,
                     int32_t angle, const pwbf_tile *tile, const pwbf_outputs *out,
                     void *workspace, size_t workspace_bytes, void *stream) {
  return run(g, rf, rf_dtype, mode, angle, tile, out, workspace, workspace_bytes, stream);
}

int pwbf_validate_call(const pwbf_geometry *g, const void *rf, int32_t rf_dtype, int32_t mode,
                       int32_t angle, const pwbf_tile *tile, const pwbf_outputs *out,
                       const void *workspace, size_t workspace_bytes) {
  g_last_error.clear();
  pwbf::FramePlan P;
  std::string err;
  int rc = pwbf::build_plan(g, rf, rf_dtype, mode, angle, tile, out, (void *)workspace,
                            workspace_bytes, &P, &err);
  if (rc) return set_error(rc, err);
  return PWBF_OK;
}

int pwbf_describe_plan(const pwbf_geometry *g, int32_t mode, int32_t angle,
                       const pwbf_tile *tile, pwbf_plan_info *info) {
  g_last_error.clear();
  if (!info) return set_error(PWBF_E_INVALID, "info is NULL");
  pwbf::FramePlan P;
  std::string err;
  int rc = pwbf::plan_frame(g, pwbf::is_iq_mode(mode) ? pwbf::kC32 : pwbf::kF32, mode, angle,
                            tile, &P, &err);
  if (rc) return set_error(rc, err);
  info->cpw = P.cpw;
  info->lz = P.lz;
  info->tile_z = P.tile_z;
  info->tile_x = P.tile_x;
  info->wz = P.wz;
  info->wx = P.wx;
  info->chunk = P.chunk;
  info->win = P.win;
  info->off_t = P.off_t;
  info->off_r = P.off_r;
  info->tiles_z = P.tiles_z;
  info->tiles_x = P.tiles_x;
  info->threads_per_block = pwbf::kWave * P.wz * P.wx;
  info->blocks = P.n_tiles;
  info->n_angles_used = P.n_angles;
  info->lds_bytes = (int64_t)pwbf::plan_lds_bytes(P);
  info->X0 = P.X0;
  info->DX = P.DX;
  info->Z0 = P.Z0;
  info->DZ = P.DZ;
  info->X0l = P.X0l;
  info->DXl = P.DXl;
  info->Z0l = P.Z0l;
  info->DZl = P.DZl;
  info->ap_k = P.ap_k;
  for (int a = 0; a < PWBF_MAX_ANGLES; ++a) {
    info->sa[a] = P.sa[a];
    info->sal[a] = P.sal[a];
    info->ca[a] = P.ca[a];
    info->cal[a] = P.cal[a];
    info->to[a] = P.to[a];
    info->tol[a] = P.tol[a];
  }
  for (int e = 0; e < PWBF_MAX_CHANNELS; ++e) {
    info->xe[e] = P.xe[e];
    info->xel[e] = P.xel[e];
  }
  return PWBF_OK;
}

}  // extern "C"
