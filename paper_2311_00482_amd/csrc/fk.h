// f-k migrations (Stolt's and Lu's): launch parameters shared by the host code
// and the kernels (passed by value).
#pragma once

#include <hip/hip_runtime.h>

#include "plan.h"

namespace pwbf {

constexpr int kFkMaxSamples = 4096;  // one LDS FFT along time per block
constexpr int kFkMaxNx = 1024;       // zero-padded array length (2 or 4 x channels)
constexpr int kFkRowPoints = 4096;   // points per block of the kx transforms (rows x Nx)

enum FkMethod { kFkStolt = 0, kFkLu = 1 };

// Per-angle constants, float-float (hi, lo) pairs.
//  c0, c1  shift of the temporal spectrum of channel e: bin k is multiplied by
//          exp(2 pi i k (c0 + e c1)), i.e. (firing delay - t0) fs / Nt
//  m0..m3  remap constants. Stolt: m0 = alpha, the source bin per signed kx
//          index, v Nt / (Nx p fs). Lu: m0 = beta, the kx' step over the kz'
//          step, c / (2 df Nx p); m1, m2 = sin and cos of the angle; m3 =
//          sin / (2 beta), the kx shift per frequency bin in spatial bins
//  ux*     column of the migrated image read by pixel (ix, iz): ux0 + ix uxi + iz uxk
//  uz*     its row: uz0 + iz uzk
//  col0, ncol, row0, nrow  the window of the migrated image that the pixel grid
//          reads (every bilinear tap of every pixel, with a margin); only it is
//          transformed along kz and stored
struct FkAngleConst {
  float c0_hi, c0_lo, c1_hi, c1_lo;
  float m0_hi, m0_lo, m1_hi, m1_lo, m2_hi, m2_lo, m3_hi, m3_lo;
  float ux0_hi, ux0_lo, uxi_hi, uxi_lo, uxk_hi, uxk_lo;
  float uz0_hi, uz0_lo, uzk_hi, uzk_lo;
  int32_t col0, ncol, row0, nrow;
};

struct FkPlan {
  const void *rf;  // records [n_ang][n_ch][Nt] of the first angle handled
  int dtype, method;
  int n_ang, n_ch, log2nt, log2nx;
  int nx_img, nz_img;
  float2 *T;  // [n_ang][Kb][n_ch][R]: shifted temporal spectra, bin k of channel e at
              // block k / R, row k mod R, with R = kFkRowPoints / Nx (the bins of one
              // kx-transform block) and Kb = ceil((Nt/2 + 1) / R)
  float2 *P;  // [n_ang][Nt/2 + 1][Nx] (Lu) or [n_ang][Nx][Nt/2 + 1] (Stolt): 2-D data spectra
  float2 *U;  // [n_ang][Nx][Nt/2 + 1]: remapped spectra after the inverse along kx
  float2 *M;  // [n_ang][Nx][Nt]: migrated complex images on (x1, z1), window only
  float *out_rf, *out_imag, *out_env;  // image planes [nx_img][nz_img]
  uint32_t *ws_max;                    // the frame maximum's slots (frame_max.h), or NULL
  FkAngleConst ang[kMaxAngles];
};

// passed by value to every kernel: keep it inside the 4 KB kernel-argument budget
static_assert(sizeof(FkPlan) <= 4000, "FkPlan too large for a kernel argument");

// bins per block of T (and rows of a kx-transform block) for Nx = 2^log2nx, and
// the bins of T per channel rounded up to whole blocks
__host__ __device__ constexpr int fk_rows(int log2nx) { return kFkRowPoints >> log2nx; }
__host__ __device__ constexpr int fk_kbins_padded(int log2nt, int log2nx) {
  return ((1 << log2nt) / 2 + fk_rows(log2nx)) / fk_rows(log2nx) * fk_rows(log2nx);
}

hipError_t launch_fk(const FkPlan &F, int ncol_max, hipStream_t s);
hipError_t launch_logc(const float *env, float *logimg, const uint32_t *ws_max, size_t n,
                       float floor_db, hipStream_t stream);

}  // namespace pwbf
