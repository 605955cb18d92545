// The allocation-free form of pwbf_compound: the same kernels, with the
// device scratch they need (the frame maximum's slots for the log image, and
// the envelope plane when the log image is wanted without it) taken from a
// file-scope device array instead of a caller's workspace.
//
// Host code never uses the array's name as an address (on the host it is only
// a stand-in for the symbol): the first call on a device, with that device
// current, looks up the device address of that device's copy once and keeps it
// per device. Every call on a device shares that copy; calls that overlap on
// one device (other streams or threads) race on it.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>
#include <string>

#include "../../include/pwbf.h"
#include "frame_max.h"
#include "plan_host.h"

namespace pwbf {
int api_set_error(int code, const std::string &msg);
void api_clear_error();
int run_frame(const pwbf_geometry *g, const void *rf, int32_t dtype, int32_t mode, int32_t angle,
              const pwbf_tile *tile, const pwbf_outputs *out, void *ws, size_t ws_bytes,
              void *stream);
}  // namespace pwbf

namespace {

// The frame maximum's slots, then an envelope plane of up to
// PWBF_NOALLOC_ENV_PIXELS pixels.
constexpr size_t kScratchBytes =
    pwbf::kMaxSlotBytes + (size_t)PWBF_NOALLOC_ENV_PIXELS * sizeof(float);
static_assert(pwbf::kMaxSlotBytes % 256 == 0, "the envelope plane must stay 256-byte aligned");

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};  // device address of scratch, per device

// The current device's copy of scratch (looked up on its first use).
int scratch_for_current_device(void **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess)
    return pwbf::api_set_error(PWBF_E_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices)
    return pwbf::api_set_error(PWBF_E_UNSUPPORTED, "device ordinal beyond 63");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return pwbf::api_set_error(PWBF_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                                    hipGetErrorString(e));
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return PWBF_OK;
}

}  // namespace

extern "C" {

int pwbf_compound_noalloc(const pwbf_geometry *g, const void *rf, int32_t rf_dtype, int32_t mode,
                          const pwbf_outputs *out, void *stream) {
  pwbf::api_clear_error();
  // the scratch this call needs, against what the array holds (host checks only)
  std::string err;
  int rc = pwbf::validate_geometry(g, &err);
  if (rc) return pwbf::api_set_error(rc, err);
  if (!out) return pwbf::api_set_error(PWBF_E_INVALID, "outputs is NULL");
  const size_t need = pwbf::workspace_bytes(g, out);
  if (need > kScratchBytes) {
    char buf[256];
    snprintf(buf, sizeof buf,
             "the log image of a %d x %d grid without an envelope output needs %zu bytes of "
             "scratch; the allocation-free call holds %zu (envelope planes up to %d pixels): "
             "pass an env plane or use pwbf_compound with a workspace",
             g->nx, g->nz, need, kScratchBytes, PWBF_NOALLOC_ENV_PIXELS);
    return pwbf::api_set_error(PWBF_E_UNSUPPORTED, buf);
  }
  void *ws = nullptr;
  if (need) {
    rc = scratch_for_current_device(&ws);
    if (rc) return rc;
  }
  return pwbf::run_frame(g, rf, rf_dtype, mode, -1, nullptr, out, ws, need ? kScratchBytes : 0,
                         stream);
}

}  // extern "C"
