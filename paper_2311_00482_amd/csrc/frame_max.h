#pragma once
// The frame maximum of the envelope, which the log image divides by, kept as
// kMaxSlots partial maxima on separate 128-byte lines. Each block folds its own
// maximum into slot blockIdx.x % kMaxSlots with an atomic max on the float's
// bit pattern (non-negative floats order like their bits); readers take the
// largest slot. A single word for the whole grid serialises the blocks'
// atomics at the end of a launch: on gfx950, 4096 blocks folding into one word
// took 49 us per launch against 4 us over 64 lines.
#include <hip/hip_runtime.h>

#include "frame_max_layout.h"

namespace pwbf {

namespace dev {

static_assert(kMaxSlots == 64, "frame_max_read reduces the slots within one wavefront");

// one thread of a block folds the block's maximum m >= 0
__device__ __forceinline__ void frame_max_fold(uint32_t *slots, float m) {
  atomicMax(slots + (blockIdx.x % kMaxSlots) * kMaxSlotStride, __float_as_uint(m));
}

// threads t < kMaxSlots of the caller clear one slot each
__device__ __forceinline__ void frame_max_clear(uint32_t *slots, int t) {
  if (t < kMaxSlots) slots[t * kMaxSlotStride] = 0u;
}

// the frame maximum, returned to every thread of a block of >= 64 threads; all
// threads of the block must call it (it ends with a barrier)
__device__ __forceinline__ float frame_max_read(const uint32_t *slots) {
  __shared__ uint32_t s_max;
  if (threadIdx.x < kMaxSlots) {
    uint32_t v = slots[threadIdx.x * kMaxSlotStride];
    for (int off = kMaxSlots / 2; off > 0; off >>= 1) {
      const uint32_t o = (uint32_t)__shfl_xor((int)v, off);
      v = o > v ? o : v;
    }
    if (threadIdx.x == 0) s_max = v;
  }
  __syncthreads();
  return __uint_as_float(s_max);
}

}  // namespace dev
}  // namespace pwbf
