// Disc regions of the image metrics, in pixel units, passed to the kernels by value.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/pwbf.h"

namespace pwbf {

struct DiscPix {
  float cx, cz;          // centre in pixel indices
  float sx, sz;          // pixel pitch over the radius, per axis
  int ix0, ix1, iz0, iz1;  // bounding box (inclusive), clipped to the grid
};

struct CystSet {
  DiscPix in[PWBF_MAX_METRIC_REGIONS], out[PWBF_MAX_METRIC_REGIONS];
};

struct TargetSet {
  DiscPix t[PWBF_MAX_METRIC_REGIONS];
};

hipError_t launch_contrast(const float *env, int nz, const CystSet &cs, int n, pwbf_contrast *out,
                           hipStream_t stream);
hipError_t launch_resolution(const float *env, int nx, int nz, float dx, float dz,
                             const TargetSet &ts, int n, pwbf_resolution *out,
                             hipStream_t stream);

}  // namespace pwbf
