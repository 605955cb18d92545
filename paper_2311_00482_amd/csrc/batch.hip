// Kernels of a batch launch: frames of uneven size, channel count, angle count,
// storage type and mode in one graph-captured launch.
//
// The graph forks into up to four branches of frames balanced by estimated
// cost; each branch runs, in order,
//   k_batch_beamform   one launch per class of its frames (beamformer, lane
//                      grouping, angle count), one block per (frame, tile) item
//                      of its list, the items sorted by estimated tile cost
//                      (active aperture x pixels x angles), largest first, so the
//                      hardware dispatcher starts the longest tiles first
//   k_batch_postz      one block per (frame, depth column) of its frames
//   k_batch_logc       one block per (frame, depth column) with a log image
// and the branches run side by side on the device, so one branch's
// post-processing and tail overlap the others' beamforming. k_batch_reset
// clears every frame's envelope maximum before the fork.
//
// Frame descriptors (FramePlan, PostPlan) live in device tables; a block reads
// its item through a wave-uniform index, so every descriptor field is a scalar
// load.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "batch.h"
#include "beamform_device.h"
#include "postz_device.h"

namespace pwbf {

namespace {

constexpr int kBatchWaves = 8;
constexpr int kBatchMaxAngles = 16;

__global__ void k_batch_reset(const PostPlan *__restrict__ post, int n_frames) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_frames && post[i].ws_max)
    for (int s = 0; s < kMaxSlots; ++s) dev::frame_max_clear(post[i].ws_max, s);
}

// One kernel per class of frames (tile_class.h): one kernel for every class
// (the DMAS and pDAS bodies need up to ~130 VGPRs) would run the compound DAS
// body at two 8-wave blocks per CU instead of three. Angle counts other than 1,
// 5 and 11 run the predicated body of up to kBatchMaxAngles. The tile body is
// chosen per frame as in the single-frame kernels (the select-free Hann body
// for DAS with one lane group).
template <int MODE, bool ONEGRP, int AB>
__global__ void __launch_bounds__(kWave * kBatchWaves)
    k_batch_beamform(const FramePlan *__restrict__ plans, const int4 *__restrict__ items) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int4 w = items[blockIdx.x];
  const FramePlan &P = plans[__builtin_amdgcn_readfirstlane(w.x)];
  const int tile = __builtin_amdgcn_readfirstlane(w.y);
  const int tz = tile / P.tiles_x, tx = tile - tz * P.tiles_x;
  // the tile's channel hull, computed on the host (w.z, w.w)
  if constexpr (AB == 3)
    dev::process_tile<kBatchMaxAngles, true, MODE, ONEGRP>(P, tz, tx, smem, w.z, w.w);
  else
    dev::process_tile<AB == 0 ? 1 : (AB == 1 ? 5 : 11), false, MODE, ONEGRP>(P, tz, tx, smem,
                                                                             w.z, w.w);
}

template <int C>
hipError_t launch_class_kernel(dim3 grid, size_t lds, hipStream_t s, const FramePlan *plans,
                               const int4 *items) {
  hipLaunchKernelGGL((k_batch_beamform<C / 8, (C / 4) % 2 == 1, C % 4>), grid,
                     dim3(kWave * kBatchWaves), lds, s, plans, items);
  return hipGetLastError();
}

template <int C>
hipError_t class_occupancy(size_t lds, int *blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(
      blocks_per_cu, k_batch_beamform<C / 8, (C / 4) % 2 == 1, C % 4>, kWave * kBatchWaves, lds);
}

#define PWBF_BATCH_CLASSES(X) \
  X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) \
  X(16) X(17) X(18) X(19) X(20) X(21) X(22) X(23)

__global__ void __launch_bounds__(dev::kPostThreads)
    k_batch_postz(const PostPlan *__restrict__ post, const int2 *__restrict__ cols) {
  extern __shared__ __align__(16) float2 sm[];
  const int2 c = cols[blockIdx.x];
  dev::postz_column(post[c.x], c.y, sm);
}

__global__ void __launch_bounds__(256)
    k_batch_logc(const PostPlan *__restrict__ post, const int2 *__restrict__ cols) {
  const int2 c = cols[blockIdx.x];
  const PostPlan &Q = post[c.x];
  const float m = dev::frame_max_read(Q.ws_max);
  const size_t base = (size_t)c.y * Q.nz;
  for (int k = threadIdx.x; k < Q.nz; k += blockDim.x)
    Q.logimg[base + k] = dev::log_db(Q.env[base + k], m, Q.floor_db);
}

}  // namespace

int batch_waves() { return kBatchWaves; }
int batch_max_angles() { return kBatchMaxAngles; }

hipError_t batch_occupancy(int cls, size_t lds_bytes, int *blocks_per_cu) {
  switch (cls) {
#define PWBF_OCC(C) \
  case C: return class_occupancy<C>(lds_bytes, blocks_per_cu);
    PWBF_BATCH_CLASSES(PWBF_OCC)
#undef PWBF_OCC
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_batch_reset(const PostPlan *post, int n_frames, hipStream_t stream) {
  hipLaunchKernelGGL(k_batch_reset, dim3((std::max(n_frames, 1) + 255) / 256), dim3(256), 0,
                     stream, post, n_frames);
  return hipGetLastError();
}

// Enqueue one branch on `stream` (captured into the batch graph by the caller).
int batch_branch_steps(int n_classes, int n_post_cols, int n_log_cols) {
  return n_classes + (n_post_cols > 0 ? 1 : 0) + (n_log_cols > 0 ? 1 : 0);
}

hipError_t launch_batch_branch_step(const FramePlan *plans, const PostPlan *post,
                                    const int4 *items, const BatchClass *classes, int n_classes,
                                    const int2 *post_cols, int n_post_cols, const int2 *log_cols,
                                    int n_log_cols, size_t lds, int max_nz, int step,
                                    hipStream_t stream) {
  if (step < n_classes) {
    const BatchClass &k = classes[step];
    switch (k.cls) {
#define PWBF_LAUNCH(C) \
  case C:              \
    return launch_class_kernel<C>(dim3(k.n), lds, stream, plans, items + k.first);
      PWBF_BATCH_CLASSES(PWBF_LAUNCH)
#undef PWBF_LAUNCH
      default: return hipErrorInvalidValue;
    }
  }
  step -= n_classes;
  if (n_post_cols > 0 && step-- == 0) {
    const size_t plds = dev::post_lds_bytes(max_nz);
    hipLaunchKernelGGL(k_batch_postz, dim3(n_post_cols), dim3(dev::kPostThreads), plds, stream,
                       post, post_cols);
    return hipGetLastError();
  }
  if (n_log_cols > 0 && step == 0) {
    hipLaunchKernelGGL(k_batch_logc, dim3(n_log_cols), dim3(256), 0, stream, post, log_cols);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

}  // namespace pwbf
