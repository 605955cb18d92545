// Kernels of a batch launch: frames of uneven size, channel count, angle count,
// storage type and mode in one graph-captured sequence of persistent launches.
//
//   k_batch_reset      clears the classes' work counters and every frame's
//                      envelope maximum (a kernel, not a memset node, so graph
//                      replays stay exact)
//   k_batch_beamform   persistent, one kernel per class of frames (beamformer,
//                      lane grouping, angle count): every block repeatedly claims
//                      the next (frame, tile) item of its class's work list,
//                      sorted by estimated tile cost (active aperture x pixels x
//                      angles), largest first, and runs the tile body for that
//                      frame's plan; all waves leave when the list is exhausted
//   k_batch_postz      one block per (frame, depth column) of frames with
//                      post-processing
//   k_batch_logc       one block per (frame, depth column) of frames with a log image
//
// Frame descriptors (FramePlan, PostPlan) live in device tables; a block reads
// the claimed item through a wave-uniform index, so every descriptor field is a
// scalar load.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "batch.h"
#include "beamform_device.h"
#include "postz_device.h"

namespace pwbf {

namespace {

constexpr int kBatchWaves = 8;
constexpr int kBatchMaxAngles = 16;

__global__ void k_batch_reset(int *counters, int n_classes, const PostPlan *__restrict__ post,
                              int n_frames) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_classes) counters[i] = 0;
  if (i < n_frames && post[i].ws_max)
    for (int s = 0; s < kMaxSlots; ++s) dev::frame_max_clear(post[i].ws_max, s);
}

// One persistent kernel per class of frames (tile_class.h): one kernel for every
// class (the DMAS and pDAS bodies need up to ~130 VGPRs) would run the
// compound DAS body at two 8-wave blocks per CU instead of three. Angle counts
// other than 1, 5 and 11 run the predicated body of up to kBatchMaxAngles.
// Every class runs the general tile body (with the aperture test in the
// weight): a second, select-free body inside the persistent loop raised the
// compound DAS kernel to 84 VGPRs, and even held to 80 it ran 10% slower.
template <int MODE, bool ONEGRP, int AB>
__global__ void __launch_bounds__(kWave * kBatchWaves)
    k_batch_beamform(const FramePlan *__restrict__ plans, const int2 *__restrict__ items,
                     int n_items, int *__restrict__ counter) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_item;
  for (;;) {
    __syncthreads();  // the previous item's LDS and s_item are no longer read
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    if (it >= n_items) break;  // uniform over the block: every wave leaves here
    const int2 w = items[it];
    const FramePlan &P = plans[w.x];
    const int tz = w.y / P.tiles_x, tx = w.y - tz * P.tiles_x;
    if constexpr (AB == 3)
      dev::process_tile_body<kBatchMaxAngles, true, MODE, ONEGRP, true>(P, tz, tx, smem);
    else
      dev::process_tile_body<AB == 0 ? 1 : (AB == 1 ? 5 : 11), false, MODE, ONEGRP, true>(P, tz, tx, smem);
  }
}

template <int C>
hipError_t launch_class_kernel(dim3 grid, size_t lds, hipStream_t s, const FramePlan *plans,
                               const int2 *items, int n_items, int *counter) {
  hipLaunchKernelGGL((k_batch_beamform<C / 8, (C / 4) % 2 == 1, C % 4>), grid,
                     dim3(kWave * kBatchWaves), lds, s, plans, items, n_items, counter);
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

// Enqueue the batch sequence on `stream` (captured into a graph by the caller).
hipError_t launch_batch(const FramePlan *plans, const PostPlan *post, const int2 *items,
                        const BatchClass *classes, int n_classes, const int2 *post_cols,
                        int n_post_cols, const int2 *log_cols, int n_log_cols, int n_frames,
                        int *counters, size_t lds, int max_nz, hipStream_t stream) {
  hipLaunchKernelGGL(k_batch_reset, dim3((std::max(n_frames, n_classes) + 255) / 256), dim3(256),
                     0, stream, counters, n_classes, post, n_frames);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (int c = 0; c < n_classes; ++c) {
    const BatchClass &k = classes[c];
    switch (k.cls) {
#define PWBF_LAUNCH(C)                                                                  \
  case C:                                                                               \
    e = launch_class_kernel<C>(dim3(k.blocks), lds, stream, plans, items + k.first, k.n, \
                               counters + c);                                           \
    break;
      PWBF_BATCH_CLASSES(PWBF_LAUNCH)
#undef PWBF_LAUNCH
      default: e = hipErrorInvalidValue; break;
    }
    if (e != hipSuccess) return e;
  }
  if (n_post_cols > 0) {
    const size_t plds = dev::post_lds_bytes(max_nz);
    hipLaunchKernelGGL(k_batch_postz, dim3(n_post_cols), dim3(dev::kPostThreads), plds, stream,
                       post, post_cols);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (n_log_cols > 0) {
    hipLaunchKernelGGL(k_batch_logc, dim3(n_log_cols), dim3(256), 0, stream, post, log_cols);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace pwbf
