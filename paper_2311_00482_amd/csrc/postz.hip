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

#include <algorithm>
#include <cstdint>

#include "postz_device.h"

namespace pwbf {

namespace {

using dev::kPostThreads;

// LZ > 0: columns of 2^LZ samples (the common lengths, compile-time loops);
// LZ = 0: any length
template <int LZ>
__global__ void __launch_bounds__(kPostThreads) k_postz(const PostPlan Q) {
  extern __shared__ __align__(16) float2 sm[];
  dev::postz_column<LZ>(Q, blockIdx.x, sm);
}

__global__ void k_logc(const float *__restrict__ env, float *__restrict__ out,
                       const uint32_t *__restrict__ ws_max, size_t n, float floor_db) {
  const float m = dev::frame_max_read(ws_max);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    out[i] = dev::log_db(env[i], m, floor_db);
}

// four pixels per thread through 16-byte loads and stores (n4 = n / 4)
__global__ void k_logc4(const float4 *__restrict__ env, float4 *__restrict__ out,
                        const uint32_t *__restrict__ ws_max, size_t n4, float floor_db) {
  const float m = dev::frame_max_read(ws_max);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
       i += (size_t)gridDim.x * blockDim.x) {
    const float4 e = env[i];
    out[i] = make_float4(dev::log_db(e.x, m, floor_db), dev::log_db(e.y, m, floor_db),
                         dev::log_db(e.z, m, floor_db), dev::log_db(e.w, m, floor_db));
  }
}

}  // namespace

hipError_t launch_logc(const float *env, float *logimg, const uint32_t *ws_max, size_t n,
                       float floor_db, hipStream_t stream) {
  const int threads = 256;
  if (n % 4 == 0 && (uintptr_t)env % 16 == 0 && (uintptr_t)logimg % 16 == 0) {
    const size_t n4 = n / 4;
    const int blocks = (int)std::min<size_t>((n4 + threads - 1) / threads, 1024);
    hipLaunchKernelGGL(k_logc4, dim3(blocks), dim3(threads), 0, stream, (const float4 *)env,
                       (float4 *)logimg, ws_max, n4, floor_db);
  } else {
    const int blocks = (int)std::min<size_t>((n + threads - 1) / threads, 4096);
    hipLaunchKernelGGL(k_logc, dim3(blocks), dim3(threads), 0, stream, env, logimg, ws_max, n,
                       floor_db);
  }
  return hipGetLastError();
}

hipError_t launch_post(const PostPlan &Q, hipStream_t stream) {
  const size_t lds = dev::post_lds_bytes(Q.nz);
  const dim3 grid(Q.nx), block(kPostThreads);
  switch (Q.log2nz) {
    case 9: hipLaunchKernelGGL(k_postz<9>, grid, block, lds, stream, Q); break;
    case 10: hipLaunchKernelGGL(k_postz<10>, grid, block, lds, stream, Q); break;
    case 11: hipLaunchKernelGGL(k_postz<11>, grid, block, lds, stream, Q); break;
    case 12: hipLaunchKernelGGL(k_postz<12>, grid, block, lds, stream, Q); break;
    default: hipLaunchKernelGGL(k_postz<0>, grid, block, lds, stream, Q); break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !Q.logimg) return e;
  return launch_logc(Q.env, Q.logimg, Q.ws_max, (size_t)Q.nx * Q.nz, Q.floor_db, stream);
}

}  // namespace pwbf
