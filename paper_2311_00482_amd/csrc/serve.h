// The active-slot list of one serving batch (passed to the kernels by value).
#pragma once

#include <hip/hip_runtime.h>

#include "plan.h"
#include "tile_class.h"

namespace pwbf {

constexpr int kServeMaxActive = 64;

struct ActiveList {
  int n;                           // active slots in this batch
  int plan[kServeMaxActive];       // plan / post table index of each
  int tile0[kServeMaxActive + 1];  // prefix sums of tiles
  int col0[kServeMaxActive + 1];   // prefix sums of post-processed columns
  int log0[kServeMaxActive + 1];   // prefix sums of log-image columns
};

int serve_waves();
int serve_max_angles();
hipError_t serve_occupancy(int cls, size_t lds_bytes, int *blocks_per_cu);
hipError_t launch_i16_to_f16(void *buf, size_t n, hipStream_t stream);
// plan_class[p]: tile class of plan p; class_blocks[c]: persistent blocks of class c
// (host arrays); counters: kTileClasses device words
hipError_t launch_serve(const FramePlan *plans, const PostPlan *post, const ActiveList &al,
                        const int *plan_class, const int *class_blocks, int *counters,
                        size_t lds, int max_nz, hipStream_t stream);

}  // namespace pwbf
