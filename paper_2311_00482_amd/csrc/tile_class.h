// Classes of frames for the persistent batch and serving kernels: beamformer
// (DAS, DMAS, pDAS) x one lane group per wavefront or several x angle count
// (exactly 1, 5, 11, or any other through a predicated body). Each class has a
// kernel holding only its own tile body, so a kernel's register budget (and
// with it the blocks per CU) is that body's, not the largest of all.
#pragma once

namespace pwbf {

constexpr int kTileClasses = 24;

inline int tile_class(int mode, bool one_group, int n_angles) {
  const int ab = n_angles == 1 ? 0 : (n_angles == 5 ? 1 : (n_angles == 11 ? 2 : 3));
  return (mode * 2 + (one_group ? 1 : 0)) * 4 + ab;
}

}  // namespace pwbf
