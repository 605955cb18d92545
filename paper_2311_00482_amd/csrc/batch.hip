// Kernels of a batch launch: frames of uneven size, channel count, angle count,
// storage type and mode in one persistent launch.
//
//   k_batch_reset      clears the work counter and every frame's envelope maximum
//                      (a kernel, not a memset node, so graph replays stay exact)
//   k_batch_beamform   persistent: every block repeatedly claims the next
//                      (frame, tile) item of a work list sorted by estimated tile
//                      cost (active aperture x pixels x angles), largest first,
//                      and runs the tile body for that frame's plan; all
//                      waves leave when the list is exhausted
//   k_batch_postz      one block per (frame, depth column) of frames with
//                      post-processing
//   k_batch_logc       one block per (frame, depth column) of frames with a log image
//
// Frame descriptors (FramePlan, PostPlan) live in device tables; a block reads
// the claimed item through a wave-uniform index, so every descriptor field is a
// scalar load.
#include <hip/hip_runtime.h>

#include "beamform_device.h"
#include "postz_device.h"

namespace pwbf {

namespace {

constexpr int kBatchWaves = 8;
constexpr int kBatchMaxAngles = 16;

__global__ void k_batch_reset(int *counter, const PostPlan *__restrict__ post, int n_frames) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *counter = 0;
  if (i < n_frames && post[i].ws_max)
    for (int s = 0; s < kMaxSlots; ++s) dev::frame_max_clear(post[i].ws_max, s);
}

// The tile bodies the persistent kernel can run: exact angle counts 1, 5 and 11
// (the batch workloads), any other count up to kBatchMaxAngles through a
// predicated body (a larger bucket would raise the register budget of the
// whole kernel, and with it lower the occupancy of every frame).
template <int MODE, bool ONEGRP>
__device__ __forceinline__ void run_tile_mode(const FramePlan &P, int tz, int tx,
                                              unsigned char *smem) {
  switch (P.n_angles) {
    case 1: dev::process_tile<1, false, MODE, ONEGRP>(P, tz, tx, smem); break;
    case 5: dev::process_tile<5, false, MODE, ONEGRP>(P, tz, tx, smem); break;
    case 11: dev::process_tile<11, false, MODE, ONEGRP>(P, tz, tx, smem); break;
    default: dev::process_tile<kBatchMaxAngles, true, MODE, ONEGRP>(P, tz, tx, smem); break;
  }
}

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
    if (P.mode == kDas) {
      if (P.cpw == 1)
        run_tile_mode<kDas, true>(P, tz, tx, smem);
      else
        run_tile_mode<kDas, false>(P, tz, tx, smem);
    } else if (P.mode == kDmas) {
      if (P.cpw == 1)
        run_tile_mode<kDmas, true>(P, tz, tx, smem);
      else
        run_tile_mode<kDmas, false>(P, tz, tx, smem);
    } else {
      if (P.cpw == 1)
        run_tile_mode<kPdas, true>(P, tz, tx, smem);
      else
        run_tile_mode<kPdas, false>(P, tz, tx, smem);
    }
  }
}

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

hipError_t batch_occupancy(size_t lds_bytes, int *blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_batch_beamform,
                                                      kWave * kBatchWaves, lds_bytes);
}

// Enqueue the batch sequence on `stream` (captured into a graph by the caller).
hipError_t launch_batch(const FramePlan *plans, const PostPlan *post, const int2 *items,
                        int n_items, const int2 *post_cols, int n_post_cols,
                        const int2 *log_cols, int n_log_cols, int n_frames, int *counter,
                        int blocks, size_t lds, int max_nz, hipStream_t stream) {
  hipLaunchKernelGGL(k_batch_reset, dim3((n_frames + 255) / 256), dim3(256), 0, stream, counter,
                     post, n_frames);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_batch_beamform, dim3(blocks), dim3(kWave * kBatchWaves), lds, stream,
                     plans, items, n_items, counter);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
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
