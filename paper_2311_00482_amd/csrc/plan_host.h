// Host-side validation and plan construction (no HIP calls; safe without a GPU).
#pragma once

#include <string>

#include "../../include/pwbf.h"
#include "plan.h"

namespace pwbf {

size_t dtype_bytes(int dtype);
// the decimation factor D of baseband records (1 when the field is 0)
inline int iq_decimation(const pwbf_geometry *g) {
  return g->iq_decimation > 1 ? g->iq_decimation : 1;
}
// v as a float-float pair (hi = v rounded to float, lo = the rest)
void split_double(double v, float *hi, float *lo);
int validate_geometry(const pwbf_geometry *g, std::string *err);
// mode decides which planes apply (IQ modes: no band-pass, imag allowed)
int validate_outputs(const pwbf_geometry *g, const pwbf_outputs *o, void *ws, size_t ws_bytes,
                     std::string *err, int mode = kDas);
size_t workspace_bytes(const pwbf_geometry *g, const pwbf_outputs *o);
pwbf_tile default_tile(const pwbf_geometry *g, int n_angles_used, int mode);
// Geometry and launch shape only (no pointers). angle < 0: all angles
// (compound); angle >= 0: that angle alone.
// waves = 8: the batch kernel's fixed 8-wavefront blocks; 0: any 1..8.
int plan_frame(const pwbf_geometry *g, int dtype, int mode, int angle, const pwbf_tile *tile,
               FramePlan *P, std::string *err, int waves = 0);
// plan_frame plus the pointer, output and workspace checks.
int build_plan(const pwbf_geometry *g, const void *rf, int dtype, int mode, int angle,
               const pwbf_tile *tile, const pwbf_outputs *o, void *ws, size_t ws_bytes,
               FramePlan *P, std::string *err);
// DMAS and pDAS form every delay as a float32 offset from their wavefront's
// centre pixel (whose own delay is split exactly into an integer and a
// fraction), so a gather's delay rounding grows with that offset, and their
// root amplifies it at near-zero delayed samples. For lane groups of lz x lx
// pixels the offset is at most
//   2 hz + hx (max |sin th_a| + sin phi_max)   samples,
// hz, hx the largest depth and lateral distance (samples) from the centre
// pixel (lz / 2 and lx / 2 pixels, rounded down) and sin phi_max the sine of
// the widest receive angle with a nonzero weight (1 / sqrt(1 + 4 F#^2), or 1
// without apodization): transmit and receive each move by at most |dz| in
// depth. The shapes the library picks itself (default, fallback, tuner) keep
// it within kRootOffsetAuto whenever some shape does. On uniform-noise RF of
// 1024 x 256, 64-channel frames, 32-pixel-deep lane groups (10.5 samples)
// were 2.4e-5 off the float64 definition, 16-pixel-deep ones (5.3 - 5.4)
// 4.9e-6 to 9.7e-6 depending on the noise, 8-pixel-deep ones (2.9) 2.0e-6 to
// 3.7e-6: the error grows with the offset, so the bound sits at 4 samples.
// Explicit shapes are taken as given.
constexpr double kRootOffsetAuto = 4.0;
// DMAS and pDAS: whether plan P's lane groups keep every gather within
// kRootOffsetAuto samples of its wavefront's reference pixel (other modes: true)
bool root_compact(const pwbf_geometry *g, const FramePlan &P);
// tuning table (tune.cpp)
std::string shape_key(const pwbf_geometry *g, int dtype, int mode, int angle, int waves);
bool tune_lookup(const std::string &key, pwbf_tile *t);
void tune_store(const std::string &key, const pwbf_tile &t);
int tune_save(const char *path, std::string *err);
int tune_load(const char *path, std::string *err);
void tune_clear();
uint32_t tune_generation();  // changes whenever the table does
const std::string &tune_cache_path();  // PWBF_TUNE_CACHE ("" when unset)
// PWBF_DEBUG: whether it is set (to anything but "0"), and a line to stderr when it is
bool debug_enabled();
void debug_log(const char *fmt, ...) __attribute__((format(printf, 1, 2)));
// Channels whose receive aperture reaches tile `tile` of plan P (all of them
// without apodization), and the tile's relative cost for work ordering.
int tile_active_channels(const pwbf_geometry *g, const FramePlan &P, int tile);
double tile_cost(const pwbf_geometry *g, const FramePlan &P, int tile);
// [lo, hi): the channels whose weight may be nonzero somewhere in the tile
// (a superset of them; lo >= hi when none), decided in float64
void tile_channel_hull(const pwbf_geometry *g, const FramePlan &P, int tile, int *lo, int *hi);
int build_post_plan(const pwbf_geometry *g, const pwbf_outputs *o, void *ws, PostPlan *Q);
bool post_needed(const pwbf_outputs *o);

}  // namespace pwbf
