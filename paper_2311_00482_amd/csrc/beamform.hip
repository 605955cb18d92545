// Single-frame launch of the beamformer: one block per pixel tile. The tile
// body (staging, delays, gather, reductions) lives in beamform_device.h.
//
// Tiles run deepest row first: a tile's cost grows with the receive aperture,
// which widens with depth, so the costliest tiles start first and the cheap
// shallow ones fill the end of the launch. Consecutive block ids go
// round-robin to the 8 XCDs, so every XCD takes every 8th tile of each tile
// row: an equal share of every depth.
#include <hip/hip_runtime.h>

#include "beamform_device.h"

namespace pwbf {

namespace {

using dev::process_tile;

template <int AM, bool PRED, int MODE, bool ONEGRP>
__global__ void __launch_bounds__(kWave * kMaxWavesPerBlock) k_beamform(const FramePlan P) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int b = blockIdx.x;
  // RF modes: clear the frame maximum the post-processing folds into (the IQ
  // modes fold it here, so their launch clears it beforehand)
  if (!is_iq_mode(MODE) && P.ws_max && b == 0) dev::frame_max_clear(P.ws_max, threadIdx.x);
  const int q = b / P.tiles_x;
  const int tz = P.tiles_z - 1 - q, tx = b - q * P.tiles_x;
  process_tile<AM, PRED, MODE, ONEGRP>(P, tz, tx, smem);
}

template <int AM, bool PRED>
hipError_t launch_am(const FramePlan &P, hipStream_t stream) {
  const dim3 block(kWave * P.wz * P.wx);
  const dim3 grid(P.n_tiles);
  const size_t lds = plan_lds_bytes(P);
  const bool one = P.cpw == 1;
  if (P.mode == kDas) {
    if (one)
      hipLaunchKernelGGL((k_beamform<AM, PRED, kDas, true>), grid, block, lds, stream, P);
    else
      hipLaunchKernelGGL((k_beamform<AM, PRED, kDas, false>), grid, block, lds, stream, P);
  } else if (P.mode == kDmas) {
    if (one)
      hipLaunchKernelGGL((k_beamform<AM, PRED, kDmas, true>), grid, block, lds, stream, P);
    else
      hipLaunchKernelGGL((k_beamform<AM, PRED, kDmas, false>), grid, block, lds, stream, P);
  } else {
    if (one)
      hipLaunchKernelGGL((k_beamform<AM, PRED, kPdas, true>), grid, block, lds, stream, P);
    else
      hipLaunchKernelGGL((k_beamform<AM, PRED, kPdas, false>), grid, block, lds, stream, P);
  }
  return hipGetLastError();
}

template <int AM, bool PRED>
hipError_t launch_am_iq(const FramePlan &P, hipStream_t stream) {
  const dim3 block(kWave * P.wz * P.wx);
  const dim3 grid(P.n_tiles);
  const size_t lds = plan_lds_bytes(P);
  const bool one = P.cpw == 1;
  if (P.mode == kIqdas) {
    if (one)
      hipLaunchKernelGGL((k_beamform<AM, PRED, kIqdas, true>), grid, block, lds, stream, P);
    else
      hipLaunchKernelGGL((k_beamform<AM, PRED, kIqdas, false>), grid, block, lds, stream, P);
  } else {
    if (one)
      hipLaunchKernelGGL((k_beamform<AM, PRED, kBbdmas, true>), grid, block, lds, stream, P);
    else
      hipLaunchKernelGGL((k_beamform<AM, PRED, kBbdmas, false>), grid, block, lds, stream, P);
  }
  return hipGetLastError();
}

__global__ void k_clear_max(uint32_t *slots) { dev::frame_max_clear(slots, threadIdx.x); }

// The IQ modes: exact kernels for 1, 5 and 11 angles, predicated ones otherwise.
hipError_t launch_iq(const FramePlan &P, hipStream_t stream) {
  if (P.ws_max) {
    hipLaunchKernelGGL(k_clear_max, dim3(1), dim3(kMaxSlots), 0, stream, P.ws_max);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  switch (P.n_angles) {
    case 1: return launch_am_iq<1, false>(P, stream);
    case 5: return launch_am_iq<5, false>(P, stream);
    case 11: return launch_am_iq<11, false>(P, stream);
    default:
      if (P.n_angles <= 16) return launch_am_iq<16, true>(P, stream);
      if (P.n_angles <= kMaxAngles) return launch_am_iq<kMaxAngles, true>(P, stream);
      return hipErrorInvalidValue;
  }
}

}  // namespace

// Angle counts 1..16 get an exactly unrolled kernel; 17..32 share a predicated one.
hipError_t launch_beamform(const FramePlan &P, hipStream_t stream) {
  if (is_iq_mode(P.mode)) return launch_iq(P, stream);
  switch (P.n_angles) {
#define PWBF_CASE(n) \
  case n: return launch_am<n, false>(P, stream);
    PWBF_CASE(1) PWBF_CASE(2) PWBF_CASE(3) PWBF_CASE(4) PWBF_CASE(5) PWBF_CASE(6) PWBF_CASE(7)
    PWBF_CASE(8) PWBF_CASE(9) PWBF_CASE(10) PWBF_CASE(11) PWBF_CASE(12) PWBF_CASE(13)
    PWBF_CASE(14) PWBF_CASE(15) PWBF_CASE(16)
#undef PWBF_CASE
    default:
      if (P.n_angles >= 1 && P.n_angles <= kMaxAngles) return launch_am<kMaxAngles, true>(P, stream);
      return hipErrorInvalidValue;
  }
}

}  // namespace pwbf
