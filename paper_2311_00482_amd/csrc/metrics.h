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
// region, with ok = maximum > 0 and CR <= max_cr_db. Each disc's bounding box
// is split into column chunks of about kQualityChunkPixels pixels, one block
// per chunk; the blocks leave (count, sum, sum of squares) partials and the
// last block of a slot combines them in chunk order, so results do not depend
// on scheduling.
constexpr int kQualityChunkPixels = 4096;
constexpr int kQualityMaxChunks = 32;  // per disc

struct QualityPlan {
  const float *env;
  const uint32_t *ws_max;
  int nz;
  float max_cr_db;
  DiscPix in, out;
  int chunks_in, chunks_out;  // column chunks of each disc's box (>= 1)
  int cols_in, cols_out;      // columns per chunk
};

// chunking of a disc's bounding box (host side)
inline void quality_chunks(const DiscPix &d, int *chunks, int *cols) {
  const int w = d.ix1 - d.ix0 + 1, h = d.iz1 - d.iz0 + 1;
  if (w <= 0 || h <= 0) {
    *chunks = 1;
    *cols = 1;
    return;
  }
  int c = (kQualityChunkPixels + h - 1) / h;
  if (c < 1) c = 1;
  if ((w + c - 1) / c > kQualityMaxChunks) c = (w + kQualityMaxChunks - 1) / kQualityMaxChunks;
  *cols = c;
  *chunks = (w + c - 1) / c;
}

struct QualityOut {
  float frame_max, cr_db, cnr;
  int ok;
};

constexpr int kQualityMax = 64;

struct QualityList {  // the slots of one batch that want the check
  int n;
  int plan[kQualityMax];        // QualityPlan index of each
  int block0[kQualityMax + 1];  // prefix sums of their blocks (chunks_in + chunks_out)
};

hipError_t launch_contrast(const float *env, int nz, const CystSet &cs, int n, pwbf_contrast *out,
                           hipStream_t stream);
hipError_t launch_resolution(const float *env, int nx, int nz, float dx, float dz,
                             const TargetSet &ts, int n, pwbf_resolution *out,
                             hipStream_t stream);
// out[k]: the check of ql.plan[k] (device QualityOut[ql.n]); partials: device
// float4[ql.block0[ql.n]]; counters: device int[ql.n], zero on entry and left
// zero on exit
hipError_t launch_quality(const QualityPlan *plans, const QualityList &ql, QualityOut *out,
                          float4 *partials, int *counters, hipStream_t stream);

}  // namespace pwbf
