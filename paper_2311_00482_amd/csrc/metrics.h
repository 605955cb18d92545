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

// The disc in pixel units (the float32 constants of the membership test) and
// its bounding box, clipped to the grid (empty when the disc misses it).
DiscPix disc_to_pixels(const pwbf_geometry *g, const pwbf_disc &d);

// The per-frame quality check of the serving loop: the frame maximum of a
// slot's envelope (from its frame-maximum slots) and the contrast of one
// region, with ok = maximum > 0 and CR <= max_cr_db.
struct QualityPlan {
  const float *env;
  const uint32_t *ws_max;
  int nz;
  float max_cr_db;
  DiscPix in, out;
};

struct QualityOut {
  float frame_max, cr_db, cnr;
  int ok;
};

constexpr int kQualityMax = 64;

struct QualityList {  // the slots of one batch that want the check
  int n;
  int plan[kQualityMax];  // QualityPlan index of each
};

hipError_t launch_contrast(const float *env, int nz, const CystSet &cs, int n, pwbf_contrast *out,
                           hipStream_t stream);
hipError_t launch_resolution(const float *env, int nx, int nz, float dx, float dz,
                             const TargetSet &ts, int n, pwbf_resolution *out,
                             hipStream_t stream);
// out[k]: the check of ql.plan[k] (device QualityOut[ql.n])
hipError_t launch_quality(const QualityPlan *plans, const QualityList &ql, QualityOut *out,
                          hipStream_t stream);

}  // namespace pwbf
