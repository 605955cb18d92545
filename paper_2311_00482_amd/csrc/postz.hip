// Depth-wise post-processing of a beamformed image, one block per image column.
//
// The column (nz samples, a power of two) is transformed with an in-LDS radix-2
// FFT (decimation in time from bit-reversed order), multiplied by the one-sided
// weights of the analytic signal (1 at DC and Nyquist, 2 for positive bins, 0
// for negative ones) and, for the band-pass, by the brick-wall mask keeping the
// round-trip band [f0, 3 f0] (signed bins k_lo..k_hi), then transformed back
// with a decimation-in-frequency inverse that leaves bit-reversed order. The
// real part of the result is the band-passed column; its magnitude is the
// envelope. The log image needs the frame maximum of the envelope: each block
// folds its column maximum into one word with an atomic max on the float bit
// pattern (non-negative floats order like their bits), and a second kernel maps
// every pixel to max(20 log10(env / max), floor).
#include <hip/hip_runtime.h>

#include "plan.h"

namespace pwbf {

namespace {

constexpr int kPostThreads = 256;

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ int bitrev(int k, int log2n) {
  return (int)(__brev((unsigned)k) >> (32 - log2n));
}

__global__ void __launch_bounds__(kPostThreads) k_postz(const PostPlan Q) {
  extern __shared__ __align__(16) float2 sm[];
  const int nz = Q.nz, L = Q.log2nz, half_n = nz >> 1;
  float2 *x = sm;
  float2 *tw = sm + nz;  // W^k = exp(-2 pi i k / nz), k < nz / 2
  const int ix = blockIdx.x;
  const int tid = threadIdx.x;
  const float *src = Q.src + (size_t)ix * nz;

  for (int k = tid; k < half_n; k += kPostThreads) {
    float s, c;
    sincospif(-2.0f * (float)k / (float)nz, &s, &c);
    tw[k] = make_float2(c, s);
  }
  for (int k = tid; k < nz; k += kPostThreads) x[bitrev(k, L)] = make_float2(src[k], 0.f);
  __syncthreads();

  // forward transform, decimation in time
  for (int s = 0; s < L; ++s) {
    const int half = 1 << s;
    for (int b = tid; b < half_n; b += kPostThreads) {
      const int pos = b & (half - 1);
      const int i0 = ((b >> s) << (s + 1)) + pos, i1 = i0 + half;
      const float2 t = cmul(tw[pos << (L - 1 - s)], x[i1]);
      const float2 u = x[i0];
      x[i0] = make_float2(u.x + t.x, u.y + t.y);
      x[i1] = make_float2(u.x - t.x, u.y - t.y);
    }
    __syncthreads();
  }

  // analytic-signal weights, band mask, and the 1/nz of the inverse
  const float inv_n = 1.0f / (float)nz;
  for (int k = tid; k < nz; k += kPostThreads) {
    float h = (k == 0 || k == half_n) ? 1.f : (k < half_n ? 2.f : 0.f);
    if (Q.bandpass) {
      const int ak = k <= half_n ? k : nz - k;
      if (ak < Q.k_lo || ak > Q.k_hi) h = 0.f;
    }
    const float2 v = x[k];
    x[k] = make_float2(v.x * h * inv_n, v.y * h * inv_n);
  }
  __syncthreads();

  // inverse transform, decimation in frequency (conjugate twiddles)
  for (int s = L - 1; s >= 0; --s) {
    const int half = 1 << s;
    for (int b = tid; b < half_n; b += kPostThreads) {
      const int pos = b & (half - 1);
      const int i0 = ((b >> s) << (s + 1)) + pos, i1 = i0 + half;
      const float2 w0 = tw[pos << (L - 1 - s)];
      const float2 u = x[i0], v = x[i1];
      x[i0] = make_float2(u.x + v.x, u.y + v.y);
      x[i1] = cmul(make_float2(u.x - v.x, u.y - v.y), make_float2(w0.x, -w0.y));
    }
    __syncthreads();
  }

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

__global__ void k_logc(const float *__restrict__ env, float *__restrict__ out,
                       const uint32_t *__restrict__ ws_max, size_t n, float floor_db) {
  const float m = __uint_as_float(*ws_max);
  const float inv = m > 0.f ? 1.0f / m : 0.f;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    float v = floor_db;
    if (m > 0.f) v = fmaxf(20.0f * log10f(env[i] * inv), floor_db);
    out[i] = v;
  }
}

}  // namespace

hipError_t launch_post(const PostPlan &Q, hipStream_t stream) {
  const size_t lds = (size_t)Q.nz * sizeof(float2) + (size_t)(Q.nz / 2) * sizeof(float2);
  hipLaunchKernelGGL(k_postz, dim3(Q.nx), dim3(kPostThreads), lds, stream, Q);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !Q.logimg) return e;
  const size_t n = (size_t)Q.nx * Q.nz;
  const int threads = 256;
  const int blocks = (int)std::min<size_t>((n + threads - 1) / threads, 4096);
  hipLaunchKernelGGL(k_logc, dim3(blocks), dim3(threads), 0, stream, Q.env, Q.logimg, Q.ws_max,
                     n, Q.floor_db);
  return hipGetLastError();
}

}  // namespace pwbf
