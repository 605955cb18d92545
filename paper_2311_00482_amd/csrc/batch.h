// Batch launch interface shared by the host code (batch.cpp) and the kernels
// (batch.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "plan.h"
#include "tile_class.h"

namespace pwbf {

// the work of one class within a branch: items [first, first + n) of the
// batch's list, one block each
struct BatchClass {
  int cls, first, n, blocks;
};

int batch_waves();
int batch_max_angles();
hipError_t batch_occupancy(int cls, size_t lds_bytes, int *blocks_per_cu);
// clears every frame's envelope-maximum slots (a kernel, not a memset node)
hipError_t launch_batch_reset(const PostPlan *post, int n_frames, hipStream_t stream);
// One branch of the batch graph is a sequence of launches: its class kernels
// in order, then the depth post-processing and the log image of its frames'
// columns. batch_branch_steps counts them; launch_batch_branch_step enqueues
// launch `step` of that sequence on the stream (the caller keeps the order).
int batch_branch_steps(int n_classes, int n_post_cols, int n_log_cols);
hipError_t launch_batch_branch_step(const FramePlan *plans, const PostPlan *post,
                                    const int4 *items, const BatchClass *classes, int n_classes,
                                    const int2 *post_cols, int n_post_cols, const int2 *log_cols,
                                    int n_log_cols, size_t lds, int max_nz, int step,
                                    hipStream_t stream);

}  // namespace pwbf
