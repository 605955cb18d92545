#pragma once
// Device code of the depth-wise post-processing (band-pass, envelope, column
// maximum), shared by the single-frame and the batched launches.
#include <hip/hip_runtime.h>

#include "plan.h"

namespace pwbf {
namespace dev {

constexpr int kPostThreads = 256;

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ int bitrev(int k, int log2n) {
  return (int)(__brev((unsigned)k) >> (32 - log2n));
}

// Radix-2 FFT of n = 2^L points in LDS, by a block of kPostThreads threads.
// tw holds W^k = exp(-2 pi i k / n) for k < n / 2.
__device__ __forceinline__ void fft_twiddles(float2 *tw, int n) {
  for (int k = threadIdx.x; k < (n >> 1); k += kPostThreads) {
    float s, c;
    sincospif(-2.0f * (float)k / (float)n, &s, &c);
    tw[k] = make_float2(c, s);
  }
}

// Forward transform, decimation in time: x in bit-reversed order -> natural order.
__device__ __forceinline__ void fft_forward(float2 *x, const float2 *tw, int L) {
  const int half_n = 1 << (L - 1);
  for (int s = 0; s < L; ++s) {
    const int half = 1 << s;
    for (int b = threadIdx.x; b < half_n; b += kPostThreads) {
      const int pos = b & (half - 1);
      const int i0 = ((b >> s) << (s + 1)) + pos, i1 = i0 + half;
      const float2 t = cmul(tw[pos << (L - 1 - s)], x[i1]);
      const float2 u = x[i0];
      x[i0] = make_float2(u.x + t.x, u.y + t.y);
      x[i1] = make_float2(u.x - t.x, u.y - t.y);
    }
    __syncthreads();
  }
}

// Inverse transform without the 1/n, decimation in frequency (conjugate
// twiddles): x in natural order -> bit-reversed order.
__device__ __forceinline__ void fft_inverse(float2 *x, const float2 *tw, int L) {
  const int half_n = 1 << (L - 1);
  for (int s = L - 1; s >= 0; --s) {
    const int half = 1 << s;
    for (int b = threadIdx.x; b < half_n; b += kPostThreads) {
      const int pos = b & (half - 1);
      const int i0 = ((b >> s) << (s + 1)) + pos, i1 = i0 + half;
      const float2 w0 = tw[pos << (L - 1 - s)];
      const float2 u = x[i0], v = x[i1];
      x[i0] = make_float2(u.x + v.x, u.y + v.y);
      x[i1] = cmul(make_float2(u.x - v.x, u.y - v.y), make_float2(w0.x, -w0.y));
    }
    __syncthreads();
  }
}

// One-sided weight of the analytic signal at bin k of n: 1 at DC and Nyquist,
// 2 on positive bins, 0 on negative ones.
__device__ __forceinline__ float analytic_weight(int k, int n) {
  const int half_n = n >> 1;
  return (k == 0 || k == half_n) ? 1.f : (k < half_n ? 2.f : 0.f);
}

// Post-process column ix of the frame described by Q, with LDS at sm
// (nz + nz/2 float2).
__device__ __forceinline__ void postz_column(const PostPlan &Q, int ix, float2 *sm) {
  const int nz = Q.nz, L = Q.log2nz, half_n = nz >> 1;
  float2 *x = sm;
  float2 *tw = sm + nz;  // W^k = exp(-2 pi i k / nz), k < nz / 2
  const int tid = threadIdx.x;
  const float *src = Q.src + (size_t)ix * nz;

  fft_twiddles(tw, nz);
  for (int k = tid; k < nz; k += kPostThreads) x[bitrev(k, L)] = make_float2(src[k], 0.f);
  __syncthreads();
  fft_forward(x, tw, L);

  // analytic-signal weights, band mask, and the 1/nz of the inverse
  const float inv_n = 1.0f / (float)nz;
  for (int k = tid; k < nz; k += kPostThreads) {
    float h = analytic_weight(k, nz);
    if (Q.bandpass) {
      const int ak = k <= half_n ? k : nz - k;
      if (ak < Q.k_lo || ak > Q.k_hi) h = 0.f;
    }
    const float2 v = x[k];
    x[k] = make_float2(v.x * h * inv_n, v.y * h * inv_n);
  }
  __syncthreads();
  fft_inverse(x, tw, L);

  float m = 0.f;
  for (int k = tid; k < nz; k += kPostThreads) {
    const float2 z = x[bitrev(k, L)];
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
      atomicMax(Q.ws_max, __float_as_uint(bm));
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
