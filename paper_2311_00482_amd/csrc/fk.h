// f-k migrations (Stolt's and Lu's): launch parameters shared by the host code
// and the kernels (passed by value).
#pragma once

#include <hip/hip_runtime.h>

#include "plan.h"

namespace pwbf {

constexpr int kFkMaxSamples = 4096;  // one LDS FFT along time per block
constexpr int kFkMaxNx = 1024;       // zero-padded array length (2 or 4 x channels)

enum FkMethod { kFkStolt = 0, kFkLu = 1 };

// Per-angle constants, float-float (hi, lo) pairs.
//  c0, c1  shift of the temporal spectrum of channel e: bin k is multiplied by
//          exp(2 pi i k (c0 + e c1)), i.e. (firing delay - t0) fs / Nt
//  alpha   Stolt: source bin per signed kx index, v Nt / (Nx p fs)
//  beta    Lu: kx' step over kz' step, c / (2 df Nx p)
//  sn, cs  Lu: sin and cos of the angle
//  sb      Lu: sin / (2 beta), the kx shift per frequency bin in spatial bins
//  ux*     column of the migrated image read by pixel (ix, iz): ux0 + ix uxi + iz uxk
//  uz*     its row: uz0 + iz uzk
struct FkAngleConst {
  float c0_hi, c0_lo, c1_hi, c1_lo;
  float alpha_hi, alpha_lo;
  float beta_hi, beta_lo, sn_hi, sn_lo, cs_hi, cs_lo, sb_hi, sb_lo;
  float ux0_hi, ux0_lo, uxi_hi, uxi_lo, uxk_hi, uxk_lo;
  float uz0_hi, uz0_lo, uzk_hi, uzk_lo;
};

struct FkPlan {
  const void *rf;  // records [n_ang][n_ch][Nt] of the first angle handled
  int dtype, method;
  int n_ang, n_ch, log2nt, log2nx;
  int nx_img, nz_img;
  float2 *S;  // [n_ang][Nt/2 + 1][Nx]: shifted temporal spectra, then the remapped spectrum
  float2 *P;  // [n_ang][Nt/2 + 1][Nx]: 2-D data spectra
  float2 *M;  // [n_ang][Nx][Nt]: migrated complex images on (x1, z1)
  float *out_rf, *out_imag, *out_env;  // image planes [nx_img][nz_img]
  uint32_t *ws_max;                    // maximum magnitude (bits of a float), or NULL
  FkAngleConst ang[kMaxAngles];
};

// passed by value to every kernel: keep it inside the 4 KB kernel-argument budget
static_assert(sizeof(FkPlan) <= 4000, "FkPlan too large for a kernel argument");

hipError_t launch_fk(const FkPlan &F, hipStream_t s);
hipError_t launch_logc(const float *env, float *logimg, const uint32_t *ws_max, size_t n,
                       float floor_db, hipStream_t stream);

}  // namespace pwbf
