#pragma once
// Device code of the depth-wise post-processing (band-pass, envelope, column
// maximum), shared by the single-frame and the batched launches.
#include <hip/hip_runtime.h>

#include "fft_lds.h"
#include "frame_max.h"
#include "plan.h"

namespace pwbf {
namespace dev {

constexpr int kPostThreads = 256;
static_assert(kPostThreads == fft::kThreads, "post-processing blocks run the block FFT");

// LDS of one post-processing block: the padded column
__host__ __device__ constexpr size_t post_lds_bytes(int nz) { return fft::lds_bytes(nz, 1); }

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// One-sided weight of the analytic signal at bin k of n: 1 at DC and Nyquist,
// 2 on positive bins, 0 on negative ones.
__device__ __forceinline__ float analytic_weight(int k, int n) {
  const int half_n = n >> 1;
  return (k == 0 || k == half_n) ? 1.f : (k < half_n ? 2.f : 0.f);
}

// Post-process column ix of the frame described by Q, with LDS at sm
// (post_lds_bytes(nz)). LZ > 0: the column length is 2^LZ, known at compile
// time (loop bounds and the transform fixed); LZ = 0: Q.log2nz at run time.
template <int LZ = 0>
__device__ __forceinline__ void postz_column(const PostPlan &Q, int ix, float2 *sm) {
  const int L = LZ ? LZ : Q.log2nz, nz = 1 << L, half_n = nz >> 1;
  float2 *x = sm;  // the column, padded layout
  const int tid = threadIdx.x;
  const float *src = Q.src + (size_t)ix * nz;

  for (int k = tid; k < nz; k += kPostThreads) x[fft::pad(k)] = make_float2(src[k], 0.f);
  __syncthreads();
  if constexpr (LZ > 0)
    fft::transform<LZ, false>(x);
  else
    fft::transform_any<false>(x, L);

  // analytic-signal weights, band mask, and the 1/nz of the inverse
  const float inv_n = 1.0f / (float)nz;
  for (int k = tid; k < nz; k += kPostThreads) {
    float h = analytic_weight(k, nz);
    if (Q.bandpass) {
      const int ak = k <= half_n ? k : nz - k;
      if (ak < Q.k_lo || ak > Q.k_hi) h = 0.f;
    }
    const float2 v = x[fft::pad(k)];
    x[fft::pad(k)] = make_float2(v.x * h * inv_n, v.y * h * inv_n);
  }
  __syncthreads();
  if constexpr (LZ > 0)
    fft::transform<LZ, true>(x);
  else
    fft::transform_any<true>(x, L);

  float m = 0.f;
  for (int k = tid; k < nz; k += kPostThreads) {
    const float2 z = x[fft::pad(k)];
    const size_t o = (size_t)ix * nz + k;
    if (Q.filtered) Q.filtered[o] = z.x;
    const float e = sqrtf(z.x * z.x + z.y * z.y);
    if (Q.env) Q.env[o] = e;
    m = fmaxf(m, e);
  }
  if (Q.ws_max) {
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    __shared__ float wmax[kPostThreads / 64];
    if ((tid & 63) == 0) wmax[tid >> 6] = m;
    __syncthreads();
    if (tid == 0) {
      float bm = wmax[0];
      for (int i = 1; i < kPostThreads / 64; ++i) bm = fmaxf(bm, wmax[i]);
      frame_max_fold(Q.ws_max, bm);
    }
  }
}


// 20 log10(env / max), clipped at the floor (the floor everywhere when max is 0);
// a true division, so the maximum itself maps to exactly 0 dB
__device__ __forceinline__ float log_db(float env, float max, float floor_db) {
  return max > 0.f ? fmaxf(20.0f * log10f(env / max), floor_db) : floor_db;
}

}  // namespace dev
}  // namespace pwbf
