// Depth-wise post-processing of a beamformed image, one block per image column.
//
// The column (nz samples, a power of two) is transformed with the in-LDS block
// FFT (radix-16 Stockham passes, natural order in and out), multiplied by the
// one-sided weights of the analytic signal (1 at DC and Nyquist, 2 for positive
// bins, 0 for negative ones) and, for the band-pass, by the brick-wall mask
// keeping the round-trip band [f0, 3 f0] (signed bins k_lo..k_hi), then
// transformed back. The
// real part of the result is the band-passed column; its magnitude is the
// envelope. The log image needs the frame maximum of the envelope: each block
// folds its column maximum into the frame's maximum slots, and a second kernel
// maps every pixel to max(20 log10(env / max), floor).
#include <hip/hip_runtime.h>

#include "postz_device.h"

namespace pwbf {

namespace {

using dev::kPostThreads;

__global__ void __launch_bounds__(kPostThreads) k_postz(const PostPlan Q) {
  extern __shared__ __align__(16) float2 sm[];
  dev::postz_column(Q, blockIdx.x, sm);
}

__global__ void k_logc(const float *__restrict__ env, float *__restrict__ out,
                       const uint32_t *__restrict__ ws_max, size_t n, float floor_db) {
  const float m = dev::frame_max_read(ws_max);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    out[i] = dev::log_db(env[i], m, floor_db);
}

}  // namespace

hipError_t launch_logc(const float *env, float *logimg, const uint32_t *ws_max, size_t n,
                       float floor_db, hipStream_t stream) {
  const int threads = 256;
  const int blocks = (int)std::min<size_t>((n + threads - 1) / threads, 4096);
  hipLaunchKernelGGL(k_logc, dim3(blocks), dim3(threads), 0, stream, env, logimg, ws_max, n,
                     floor_db);
  return hipGetLastError();
}

hipError_t launch_post(const PostPlan &Q, hipStream_t stream) {
  const size_t lds = dev::post_lds_bytes(Q.nz);
  hipLaunchKernelGGL(k_postz, dim3(Q.nx), dim3(kPostThreads), lds, stream, Q);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !Q.logimg) return e;
  const size_t n = (size_t)Q.nx * Q.nz;
  const int threads = 256;
  const int blocks = (int)std::min<size_t>((n + threads - 1) / threads, 4096);
  hipLaunchKernelGGL(k_logc, dim3(blocks), dim3(threads), 0, stream, Q.env, Q.logimg, Q.ws_max,
                     n, Q.floor_db);
  return hipGetLastError();
}

}  // namespace pwbf
