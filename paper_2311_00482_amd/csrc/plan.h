// Launch plans shared by the host library and the HIP kernels.
//
// A FramePlan holds everything one frame's beamforming kernel needs, in float32
// and in *sample units*: every length is multiplied by fs / c, so a pixel at
// (X, Z) and an element at Xe give the receive delay sqrt((X - Xe)^2 + Z^2)
// directly in samples. The host computes these constants in double precision
// and rounds each one once.
#pragma once

#include <cstddef>
#include <cstdint>

#if defined(__HIPCC__)
#define PWBF_HD __host__ __device__
#else
#define PWBF_HD
#endif

namespace pwbf {

constexpr int kMaxAngles = 32;
constexpr int kMaxChannels = 256;
constexpr int kWave = 64;
constexpr int kMaxWavesPerBlock = 8;
constexpr int kMaxLdsBytes = 64 * 1024;
// Default LDS budget of a block: three blocks fit the 160 KB of a gfx950 CU
// together with their static LDS, at 512-byte allocation granularity.
constexpr int kDefaultLdsBytes = 52 * 1024;
constexpr int kMaxNzPost = 4096;

enum Dtype : int32_t { kI16 = 0, kF16 = 1, kF32 = 2, kC32 = 3 };
enum Mode : int32_t { kDas = 0, kDmas = 1, kPdas = 2, kIqdas = 3, kBbdmas = 4 };

PWBF_HD constexpr bool is_iq_mode(int mode) { return mode == kIqdas || mode == kBbdmas; }

// Longest LDS window per (channel, angle), in entries. DAS, IQ-DAS and BB-DMAS
// hold every per-gather delay as a float32 offset centred on their tile's
// window, so its rounding grows with the window: 64 entries keep the offsets
// below 32 samples (2^-19 of a sample resolution), which holds DAS and IQ-DAS
// within 1e-5 of the float64 definition, and BB-DMAS too: its root acts on a
// sample's complex amplitude, which comes near zero only where both parts do
// (measured on the 11-angle 1024 x 1024 frame, phantom and speckle: at most
// 2.0e-6 at windows of 28, 36 and 48 entries). DMAS and pDAS measure their
// delays from their wavefront's centre pixel instead (the window origin enters
// only through integer shifts), so their rounding follows the lane group's
// extent (the planner bounds it), not the window. Longer windows are refused
// (shallower or narrower tiles keep them short).
constexpr int kMaxWindow = 64;
PWBF_HD constexpr int max_window(int) { return kMaxWindow; }

enum Apod : int32_t { kHann = 0, kBoxcar = 1, kNone = 2 };

struct FramePlan {
  const void *rf;  // RF[n_angles][n_channels][n_samples] of dtype (single angle: its slab)
  float *out;      // [nx][nz] beamformed image (IQ modes: real part)
  uint32_t *ws_max;  // RF modes: cleared by the beamform kernel when the log image is
                     // requested; IQ modes: the frame maximum of |image| (cleared before)
  float *out_imag;   // IQ modes: imaginary part, or null
  float *out_env;    // IQ modes: |image| (the caller's env plane or workspace), or null
  int32_t dtype, mode, apod;
  int32_t n_angles, n_channels, n_samples;
  int32_t nx, nz;
  // Geometry as float-float pairs (value = hi + lo, |lo| <= ulp(hi)/2), so that
  // per-tile reference delays can be formed to ~1e-12 relative without float64.
  float X0, DX, Z0, DZ;      // centre of pixel (0, 0) and pitches, samples (hi)
  float X0l, DXl, Z0l, DZl;  // ... and their lo parts
  float ap_k;            // 2 F#: normalised aperture distance r = |X - Xe| * ap_k / Z
  float pdas_p, pdas_inv_p;  // pDAS root order p and 1 / p (mode kPdas)
  float iq_r, iq_rl;         // IQ modes: f0 / fs, carrier revolutions per sample (hi, lo)
  int32_t entry_bytes;       // LDS bytes per window entry: 8 (RF), 16 (complex IQ)
  // launch shape
  int32_t cpw, lz, lx, wz, wx, chunk;  // lane groups, lanes along z/x per group, waves
  int32_t win;           // LDS entries per (channel, angle) window
  int32_t off_t, off_r;  // centring offsets of the transmit and receive window delays
  int32_t tile_z, tile_x;  // pixels per tile: lz * wz by lx * wx
  int32_t tiles_z, tiles_x, n_tiles, reserved_i32;
  float sa[kMaxAngles], sal[kMaxAngles];  // sin(theta_a), hi and lo
  float ca[kMaxAngles], cal[kMaxAngles];  // cos(theta_a)
  float to[kMaxAngles], tol[kMaxAngles];  // first-firing offset plus t0, samples
  float xe[kMaxChannels], xel[kMaxChannels];  // element x, samples (padded with the last)
};

struct PostPlan {
  const float *src;  // [nx][nz] image to post-process
  float *filtered;   // Re(analytic) of the band-passed column, or null
  float *env;        // |analytic|, or null
  float *logimg;     // log image, or null (needs env and ws_max)
  uint32_t *ws_max;  // the frame maximum's slots (frame_max.h), or null
  int32_t nx, nz, log2nz;
  int32_t bandpass, k_lo, k_hi;  // band [k_lo, k_hi] in |signed bin|
  float floor_db;
};

// The beamformers that take a root of every delayed sample (DMAS, pDAS) form
// each pixel's delays relative to its wavefront's own reference pixel rather
// than the tile's, so the float32 offsets on the gather path stay within the
// wavefront's few samples of delay spread (the root amplifies delay rounding
// near zero crossings); DAS and the IQ modes keep the tile reference.
PWBF_HD constexpr bool wave_ref_mode(int mode) { return mode == kDmas || mode == kPdas; }

// LDS of a block: per angle {tx(q) - LT, LT, transmit phasor} (16 bytes), per
// channel of the chunk {Dq, rq^2, rq, rx(q) - LR} (16) and the receive phasor
// (8, IQ modes only), per (wavefront, channel) of the chunk the wavefront's
// reference terms and integer window offset (16, DMAS and pDAS only), per
// window row (channel, angle) of the chunk its record offset and first sample
// (8), then the windows.
constexpr size_t kLdsAngleBytes = kMaxAngles * 16;
PWBF_HD inline size_t plan_lds_ph_offset(const FramePlan &p) {
  return kLdsAngleBytes + (size_t)p.chunk * 16;
}
PWBF_HD inline size_t plan_lds_wref_offset(const FramePlan &p) {
  return plan_lds_ph_offset(p) + (is_iq_mode(p.mode) ? (size_t)p.chunk * 8 : 0);
}
PWBF_HD inline size_t plan_lds_wref_bytes(const FramePlan &p) {
  return wave_ref_mode(p.mode) ? (size_t)p.wz * p.wx * p.chunk * 16 : 0;
}
PWBF_HD inline size_t plan_lds_row_offset(const FramePlan &p) {
  return plan_lds_wref_offset(p) + plan_lds_wref_bytes(p);
}
PWBF_HD inline size_t plan_lds_win_offset(const FramePlan &p) {
  return (plan_lds_row_offset(p) + (size_t)p.chunk * p.n_angles * 8 + 15) / 16 * 16;
}
PWBF_HD inline size_t plan_lds_bytes(const FramePlan &p) {
  return plan_lds_win_offset(p) + (size_t)p.chunk * p.n_angles * p.win * p.entry_bytes;
}

}  // namespace pwbf
