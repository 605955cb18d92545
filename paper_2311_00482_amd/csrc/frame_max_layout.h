#pragma once
// Layout of the frame maximum's slots (frame_max.h), for host and device code:
// kMaxSlots partial maxima, one per 128-byte line.
#include <cstddef>
#include <cstdint>

namespace pwbf {

constexpr int kMaxSlots = 64;
constexpr int kMaxSlotStride = 32;  // uint32 words between slots: one 128-byte line each
constexpr size_t kMaxSlotBytes = (size_t)kMaxSlots * kMaxSlotStride * sizeof(uint32_t);

}  // namespace pwbf
