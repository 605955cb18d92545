// Baseband (IQ) demodulation of channel records, two records per block, and
// the decimating form, one record per block.
//
// The analytic signal of a record x of n = 2^L samples is the inverse DFT of
// its spectrum times the one-sided weights w(k) (1 at DC and Nyquist, 2 on
// positive bins, 0 on negative ones); since w(k) + w(n - k) = 2, its real part
// is x itself and its imaginary part is the discrete Hilbert transform H(x).
// Two records x1, x2 go through one transform pair: the inverse DFT of w(k)
// times the DFT of x1 + i x2 is (x1 + i H(x1)) + i (x2 + i H(x2)), so
// H(x1) = Im - x2 and H(x2) = x1 - Re, with x1 and x2 the samples kept in
// registers. Each analytic record is then multiplied by exp(-2 pi i r k) with
// r = f0 / fs, k the sample index. The carrier phase is formed in revolutions
// from r as a float-float pair: k * r_hi splits exactly into a rounded product
// and its error (one FMA), so frac(k r) is accurate to ~1e-7 revolutions for
// every k, where a plain float product would drift by ~k ulp.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "postz_device.h"

namespace pwbf {

namespace {

using dev::kPostThreads;

template <int DT>
__device__ __forceinline__ float rf_sample(const void *rf, size_t i) {
  if constexpr (DT == kI16) return (float)((const int16_t *)rf)[i];
  if constexpr (DT == kF16) return __half2float(((const __half *)rf)[i]);
  return ((const float *)rf)[i];
}

constexpr int kIqMaxPerThread = 4096 / kPostThreads;  // samples of a record per thread

// exp(-2 pi i r k): the carrier phase at sample k in revolutions, from r as a
// float-float pair (the FMA gives the exact error of the rounded product); the
// hardware sine and cosine take their argument in revolutions, as the IQ
// beamformer's phase rotation does
__device__ __forceinline__ float2 carrier(int k, float r_hi, float r_lo) {
  const float fk = (float)k;
  const float p = fk * r_hi;
  const float e = fmaf(fk, r_hi, -p);  // exact error of the product
  const float rho = (p - floorf(p)) + fmaf(fk, r_lo, e);
  return make_float2(__builtin_amdgcn_cosf(rho), -__builtin_amdgcn_sinf(rho));
}

template <int DT>
__global__ void __launch_bounds__(kPostThreads)
    k_iq_demod(const void *__restrict__ rf, float2 *__restrict__ iq, int rows, int log2ns,
               float r_hi, float r_lo) {
  extern __shared__ __align__(16) float2 sm[];
  const int ns = 1 << log2ns;
  float2 *x = sm;
  const int r0 = 2 * blockIdx.x;
  const bool two = r0 + 1 < rows;  // a missing second record is zero
  const size_t base0 = (size_t)r0 * ns, base1 = two ? base0 + ns : base0;
  float2 keep[kIqMaxPerThread];  // (x1, x2) at the thread's samples
#pragma unroll
  for (int i = 0; i < kIqMaxPerThread; ++i) {
    const int k = threadIdx.x + i * kPostThreads;
    if (k < ns) {
      const float v1 = rf_sample<DT>(rf, base1 + k);
      keep[i] = make_float2(rf_sample<DT>(rf, base0 + k), two ? v1 : 0.f);
      x[fft::pad(k)] = keep[i];
    }
  }
  __syncthreads();
  fft::transform_any<false>(x, log2ns);
  const float inv_n = 1.0f / (float)ns;
  for (int k = threadIdx.x; k < ns; k += kPostThreads) {
    const float h = dev::analytic_weight(k, ns) * inv_n;
    const float2 v = x[fft::pad(k)];
    x[fft::pad(k)] = make_float2(v.x * h, v.y * h);
  }
  __syncthreads();
  fft::transform_any<true>(x, log2ns);
#pragma unroll
  for (int i = 0; i < kIqMaxPerThread; ++i) {
    const int k = threadIdx.x + i * kPostThreads;
    if (k < ns) {
      const float2 w = x[fft::pad(k)];
      const float2 ph = carrier(k, r_hi, r_lo);
      iq[base0 + k] = dev::cmul(make_float2(keep[i].x, w.y - keep[i].y), ph);
      if (two) iq[base1 + k] = dev::cmul(make_float2(keep[i].y, keep[i].x - w.x), ph);
    }
  }
}

// Decimation by D = 2^log2d, one record per block: the analytic signal is
// band-limited to the bins k_lo..k_hi (those within fs / (2 D) of f0, decided
// on the host) before the inverse transform, then mixed down, and every D-th
// sample is kept. The band limit takes the real part off the record itself, so
// the two-records-per-transform form above does not apply here.
template <int DT>
__global__ void __launch_bounds__(kPostThreads)
    k_iq_demod_decim(const void *__restrict__ rf, float2 *__restrict__ iq, int log2ns,
                     int log2d, int k_lo, int k_hi, float r_hi, float r_lo) {
  extern __shared__ __align__(16) float2 sm[];
  const int ns = 1 << log2ns;
  float2 *x = sm;
  const size_t base = (size_t)blockIdx.x * ns;
  for (int k = threadIdx.x; k < ns; k += kPostThreads)
    x[fft::pad(k)] = make_float2(rf_sample<DT>(rf, base + k), 0.f);
  __syncthreads();
  fft::transform_any<false>(x, log2ns);
  const float inv_n = 1.0f / (float)ns;
  for (int k = threadIdx.x; k < ns; k += kPostThreads) {
    const float h = (k >= k_lo && k <= k_hi) ? dev::analytic_weight(k, ns) * inv_n : 0.f;
    const float2 v = x[fft::pad(k)];
    x[fft::pad(k)] = make_float2(v.x * h, v.y * h);
  }
  __syncthreads();
  fft::transform_any<true>(x, log2ns);
  const int nd = ns >> log2d;
  const size_t out = (size_t)blockIdx.x * nd;
  for (int m = threadIdx.x; m < nd; m += kPostThreads) {
    const int k = m << log2d;
    iq[out + m] = dev::cmul(x[fft::pad(k)], carrier(k, r_hi, r_lo));
  }
}

}  // namespace

size_t iq_demod_lds_bytes(int ns) { return fft::lds_bytes(ns, 1); }

hipError_t launch_iq_demod(const void *rf, int dtype, void *iq, int rows, int log2ns, float r_hi,
                           float r_lo, int log2d, int k_lo, int k_hi, hipStream_t stream) {
  const size_t lds = iq_demod_lds_bytes(1 << log2ns);
  float2 *out = (float2 *)iq;
  if (log2d > 0) {
    if (dtype == kI16)
      hipLaunchKernelGGL(k_iq_demod_decim<kI16>, dim3(rows), dim3(kPostThreads), lds, stream, rf,
                         out, log2ns, log2d, k_lo, k_hi, r_hi, r_lo);
    else if (dtype == kF16)
      hipLaunchKernelGGL(k_iq_demod_decim<kF16>, dim3(rows), dim3(kPostThreads), lds, stream, rf,
                         out, log2ns, log2d, k_lo, k_hi, r_hi, r_lo);
    else
      hipLaunchKernelGGL(k_iq_demod_decim<kF32>, dim3(rows), dim3(kPostThreads), lds, stream, rf,
                         out, log2ns, log2d, k_lo, k_hi, r_hi, r_lo);
    return hipGetLastError();
  }
  const dim3 pairs((rows + 1) / 2);  // two records per block
  if (dtype == kI16)
    hipLaunchKernelGGL(k_iq_demod<kI16>, pairs, dim3(kPostThreads), lds, stream, rf, out, rows,
                       log2ns, r_hi, r_lo);
  else if (dtype == kF16)
    hipLaunchKernelGGL(k_iq_demod<kF16>, pairs, dim3(kPostThreads), lds, stream, rf, out, rows,
                       log2ns, r_hi, r_lo);
  else
    hipLaunchKernelGGL(k_iq_demod<kF32>, pairs, dim3(kPostThreads), lds, stream, rf, out, rows,
                       log2ns, r_hi, r_lo);
  return hipGetLastError();
}

}  // namespace pwbf
