// Kernels of the serving loop. A serving batch is a list of active ring slots
// passed by value; prefix sums of the slots' tile and column counts map a
// global work index to (slot, tile) or (slot, column), so no per-batch table is
// uploaded. The slots' tiles run in one persistent kernel per class of probe
// (tile_class.h), their columns in one post-processing and one log launch.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <algorithm>

#include "beamform_device.h"
#include "postz_device.h"
#include "serve.h"

namespace pwbf {

namespace {

constexpr int kServeWaves = 8;
constexpr int kServeMaxAngles = 16;

// index k with start[k] <= i < start[k + 1] (start[0] = 0, n entries)
__device__ __forceinline__ int find_slot(const int *start, int n, int i) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= i)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__global__ void k_i16_to_f16(void *buf, size_t n) {
  // element i is read as int16 and written back as binary16 by the same thread;
  // 10-bit samples (|v| <= 2048) convert exactly
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    const int16_t v = ((const int16_t *)buf)[i];
    ((__half *)buf)[i] = __int2half_rn((int)v);
  }
}

__global__ void k_serve_reset(int *counters, const PostPlan *__restrict__ post, ActiveList al) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kTileClasses) counters[i] = 0;
  if (i < al.n) {
    const PostPlan &Q = post[al.plan[i]];
    if (Q.ws_max)
      for (int s = 0; s < kMaxSlots; ++s) dev::frame_max_clear(Q.ws_max, s);
  }
}

template <int MODE, bool ONEGRP, int AB>
__global__ void __launch_bounds__(kWave * kServeWaves)
    k_serve_beamform(const FramePlan *__restrict__ plans, const ActiveList al,
                     int *__restrict__ counter) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_item;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    if (it >= al.tile0[al.n]) break;  // uniform: every wave of the block leaves
    const int k = find_slot(al.tile0, al.n, it);
    const FramePlan &P = plans[al.plan[k]];
    // within a slot, deepest tile row first (the receive aperture, and so the
    // cost, grows with depth)
    const int t = it - al.tile0[k];
    const int q = t / P.tiles_x;
    const int tz = P.tiles_z - 1 - q, tx = t - q * P.tiles_x;
    // the general tile body, as in the batch kernels
    if constexpr (AB == 3)
      dev::process_tile_body<kServeMaxAngles, true, MODE, ONEGRP, true>(P, tz, tx, smem);
    else
      dev::process_tile_body<AB == 0 ? 1 : (AB == 1 ? 5 : 11), false, MODE, ONEGRP, true>(P, tz, tx, smem);
  }
}

#define PWBF_SERVE_CLASSES(X) \
  X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) \
  X(16) X(17) X(18) X(19) X(20) X(21) X(22) X(23)
static_assert(kTileClasses == 24, "one kernel per class");

__global__ void __launch_bounds__(dev::kPostThreads)
    k_serve_postz(const PostPlan *__restrict__ post, const ActiveList al) {
  extern __shared__ __align__(16) float2 sm[];
  const int b = blockIdx.x;
  const int k = find_slot(al.col0, al.n, b);
  dev::postz_column(post[al.plan[k]], b - al.col0[k], sm);
}

__global__ void __launch_bounds__(256) k_serve_logc(const PostPlan *__restrict__ post,
                                                    const ActiveList al) {
  const int b = blockIdx.x;
  const int k = find_slot(al.log0, al.n, b);
  const PostPlan &Q = post[al.plan[k]];
  const float m = dev::frame_max_read(Q.ws_max);
  const size_t base = (size_t)(b - al.log0[k]) * Q.nz;
  for (int i = threadIdx.x; i < Q.nz; i += blockDim.x)
    Q.logimg[base + i] = dev::log_db(Q.env[base + i], m, Q.floor_db);
}

}  // namespace

int serve_waves() { return kServeWaves; }
int serve_max_angles() { return kServeMaxAngles; }

hipError_t serve_occupancy(int cls, size_t lds_bytes, int *blocks_per_cu) {
  switch (cls) {
#define PWBF_OCC(C)                                                                        \
  case C:                                                                                  \
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(                                   \
        blocks_per_cu, k_serve_beamform<C / 8, (C / 4) % 2 == 1, C % 4>, kWave * kServeWaves, \
        lds_bytes);
    PWBF_SERVE_CLASSES(PWBF_OCC)
#undef PWBF_OCC
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_i16_to_f16(void *buf, size_t n, hipStream_t stream) {
  const int threads = 256;
  const int blocks = (int)std::min<size_t>((n + threads - 1) / threads, 2048);
  hipLaunchKernelGGL(k_i16_to_f16, dim3(blocks), dim3(threads), 0, stream, buf, n);
  return hipGetLastError();
}

hipError_t launch_serve(const FramePlan *plans, const PostPlan *post, const ActiveList &al,
                        const int *plan_class, const int *class_blocks, int *counters,
                        size_t lds, int max_nz, hipStream_t stream) {
  hipLaunchKernelGGL(k_serve_reset, dim3((std::max(al.n, kTileClasses) + 255) / 256), dim3(256),
                     0, stream, counters, post, al);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // the slots of each class, with their own tile prefix sums
  for (int c = 0; c < kTileClasses; ++c) {
    ActiveList sub;
    sub.n = 0;
    sub.tile0[0] = 0;
    for (int k = 0; k < al.n; ++k) {
      if (plan_class[al.plan[k]] != c) continue;
      sub.plan[sub.n] = al.plan[k];
      sub.tile0[sub.n + 1] = sub.tile0[sub.n] + (al.tile0[k + 1] - al.tile0[k]);
      ++sub.n;
    }
    if (sub.n == 0) continue;
    const dim3 grid(std::max(1, std::min(class_blocks[c], sub.tile0[sub.n])));
    switch (c) {
#define PWBF_LAUNCH(C)                                                                     \
  case C:                                                                                  \
    hipLaunchKernelGGL((k_serve_beamform<C / 8, (C / 4) % 2 == 1, C % 4>), grid,           \
                       dim3(kWave * kServeWaves), lds, stream, plans, sub, counters + c);  \
    break;
      PWBF_SERVE_CLASSES(PWBF_LAUNCH)
#undef PWBF_LAUNCH
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (al.col0[al.n] > 0) {
    const size_t plds = dev::post_lds_bytes(max_nz);
    hipLaunchKernelGGL(k_serve_postz, dim3(al.col0[al.n]), dim3(dev::kPostThreads), plds, stream,
                       post, al);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (al.log0[al.n] > 0) {
    hipLaunchKernelGGL(k_serve_logc, dim3(al.log0[al.n]), dim3(256), 0, stream, post, al);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace pwbf
