// Baseband (IQ) demodulation of channel records, one block per record.
//
// A record of n = 2^L samples is transformed with the in-LDS block FFT,
// multiplied by the one-sided weights of the analytic signal (and the 1/n of
// the inverse), transformed back, and multiplied by exp(-2 pi i r k) with
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

template <int DT>
__global__ void __launch_bounds__(kPostThreads)
    k_iq_demod(const void *__restrict__ rf, float2 *__restrict__ iq, int log2ns, float r_hi,
               float r_lo) {
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
    const float h = dev::analytic_weight(k, ns) * inv_n;
    const float2 v = x[fft::pad(k)];
    x[fft::pad(k)] = make_float2(v.x * h, v.y * h);
  }
  __syncthreads();
  fft::transform_any<true>(x, log2ns);
  for (int k = threadIdx.x; k < ns; k += kPostThreads) {
    const float2 z = x[fft::pad(k)];
    const float fk = (float)k;
    const float p = fk * r_hi;
    const float e = fmaf(fk, r_hi, -p);  // exact error of the product
    const float rho = (p - floorf(p)) + fmaf(fk, r_lo, e);
    float s, c;
    sincospif(-2.0f * rho, &s, &c);
    iq[base + k] = dev::cmul(z, make_float2(c, s));
  }
}

}  // namespace

size_t iq_demod_lds_bytes(int ns) { return fft::lds_bytes(ns, 1); }

hipError_t launch_iq_demod(const void *rf, int dtype, void *iq, int rows, int log2ns, float r_hi,
                           float r_lo, hipStream_t stream) {
  const size_t lds = iq_demod_lds_bytes(1 << log2ns);
  float2 *out = (float2 *)iq;
  if (dtype == kI16)
    hipLaunchKernelGGL(k_iq_demod<kI16>, dim3(rows), dim3(kPostThreads), lds, stream, rf, out,
                       log2ns, r_hi, r_lo);
  else if (dtype == kF16)
    hipLaunchKernelGGL(k_iq_demod<kF16>, dim3(rows), dim3(kPostThreads), lds, stream, rf, out,
                       log2ns, r_hi, r_lo);
  else
    hipLaunchKernelGGL(k_iq_demod<kF32>, dim3(rows), dim3(kPostThreads), lds, stream, rf, out,
                       log2ns, r_hi, r_lo);
  return hipGetLastError();
}

}  // namespace pwbf
