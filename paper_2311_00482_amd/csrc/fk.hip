// f-k migrations (Stolt's and Lu's) for steered plane waves. Every stage runs
// over all angles of the call in one launch (blockIdx.y or the flat index
// selects the angle), so even a single frame gives the chip thousands of blocks.
// The two methods share every stage but the remap:
//
//  k_fk_time      block per (channel, angle): FFT of the trace (Nt samples); the
//                 positive bins times exp(2 pi i k c_e) (the trace advanced by its
//                 element's firing delay and shifted to t = 0) go to S[k][e]
//  k_fk_space     block per (bin k, angle): FFT along the array, zero-padded to Nx
//  k_fk_stolt     thread per (kz_j, kx_m, angle): the spectrum at the bin
//                 u = sqrt((alpha m')^2 + j^2) (m' the signed index), linearly
//                 interpolated (zeros past the last bin), times the Jacobian j / u
//  k_fk_lu        (Lu's remap instead) thread per (kz'_j, kx'_m, angle): the data
//                 spectrum at frequency bin u = (beta^2 m'^2 + j^2) /
//                 (beta m' sin + j cos) and spatial bin m' - u sin / (2 beta),
//                 bilinearly (periodic in the spatial bin), times the Jacobian
//                 (j - u cos / 2) / (beta m' sin + j cos); zero where the
//                 receive wavenumber j - u cos / 2 is negative
//  k_fk_ispace    block per (kz_j, angle): inverse FFT along kx
//  k_fk_itime     block per (x1 column, angle): inverse FFT along kz with the
//                 one-sided spectrum zero-filled to Nt, scaled by 1/(Nx Nt)
//  k_fk_image     thread per pixel: for every angle the migrated image at
//                 (x1, z1), affine in the pixel indices, by bilinear interpolation;
//                 the complex sum over angles gives the real, imaginary and
//                 magnitude planes and the frame maximum
//
// Interpolation positions are float-float: neighbouring spectral bins of an echo
// differ by up to a half turn of phase, so a weight off by 1e-4 (a float32
// position near bin 2000) would show in the image; products of a float-float
// constant and an integer index are exact up to the final rounding.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "beamform_device.h"
#include "fk.h"
#include "postz_device.h"

namespace pwbf {

namespace {

using dev::ff;
using dev::kPostThreads;

template <int DT>
__device__ __forceinline__ float trace_sample(const void *rf, size_t i) {
  if constexpr (DT == kI16) return (float)((const int16_t *)rf)[i];
  if constexpr (DT == kF16) return __half2float(((const __half *)rf)[i]);
  return ((const float *)rf)[i];
}

__device__ __forceinline__ ff ffi(int i) { return {(float)i, 0.f}; }

// frac(k c) in revolutions for an integer k and c = hi + lo
__device__ __forceinline__ float frac_revs(int k, ff c) {
#pragma clang fp contract(off)
  const float fk = (float)k;
  const float p = fk * c.hi;
  return (p - floorf(p)) + fmaf(fk, c.lo, fmaf(fk, c.hi, -p));
}

// integer part and fraction of a float-float value (fraction in [0, 1))
__device__ __forceinline__ int split_index(ff u, float *frac) {
  int i = (int)floorf(u.hi);
  float f = (u.hi - (float)i) + u.lo;
  if (f < 0.f) {
    f += 1.f;
    --i;
  } else if (f >= 1.f) {
    f -= 1.f;
    ++i;
  }
  *frac = f;
  return i;
}

// a / b in float-float (one correction step)
__device__ __forceinline__ ff ff_div(ff a, ff b) {
#pragma clang fp contract(off)
  const float q1 = a.hi / b.hi;
  const ff r = dev::ff_add(a, dev::ff_neg(dev::ff_mul({q1, 0.f}, b)));
  return dev::two_sum(q1, r.hi / b.hi);
}

__device__ __forceinline__ size_t spec_elems(const FkPlan &F) {
  return (size_t)((1 << F.log2nt) / 2 + 1) << F.log2nx;
}

template <int DT>
__global__ void __launch_bounds__(kPostThreads) k_fk_time(FkPlan F) {
  extern __shared__ __align__(16) float2 sm[];
  const int nt = 1 << F.log2nt, nx = 1 << F.log2nx, e = blockIdx.x, a = blockIdx.y;
  float2 *x = sm, *tw = sm + nt;
  dev::fft_twiddles(tw, nt);
  const size_t base = ((size_t)a * F.n_ch + e) * nt;
  for (int k = threadIdx.x; k < nt; k += kPostThreads)
    x[dev::bitrev(k, F.log2nt)] = make_float2(trace_sample<DT>(F.rf, base + k), 0.f);
  __syncthreads();
  dev::fft_forward(x, tw, F.log2nt);
  const FkAngleConst &A = F.ang[a];
  const ff c = dev::ff_add({A.c0_hi, A.c0_lo}, dev::ff_mul(ffi(e), {A.c1_hi, A.c1_lo}));
  float2 *S = F.S + (size_t)a * spec_elems(F);
  for (int k = threadIdx.x; k <= nt / 2; k += kPostThreads) {
    float sn, cs;
    sincospif(2.0f * frac_revs(k, c), &sn, &cs);
    S[(size_t)k * nx + e] = dev::cmul(x[k], make_float2(cs, sn));
  }
}

__global__ void __launch_bounds__(kPostThreads) k_fk_space(FkPlan F) {
  extern __shared__ __align__(16) float2 sm[];
  const int nx = 1 << F.log2nx;
  float2 *x = sm, *tw = sm + nx;
  dev::fft_twiddles(tw, nx);
  const size_t row = (size_t)blockIdx.y * spec_elems(F) + (size_t)blockIdx.x * nx;
  for (int e = threadIdx.x; e < nx; e += kPostThreads)
    x[dev::bitrev(e, F.log2nx)] = e < F.n_ch ? F.S[row + e] : make_float2(0.f, 0.f);
  __syncthreads();
  dev::fft_forward(x, tw, F.log2nx);
  for (int m = threadIdx.x; m < nx; m += kPostThreads) F.P[row + m] = x[m];
}

__global__ void __launch_bounds__(256) k_fk_stolt(FkPlan F) {
  const int nx = 1 << F.log2nx, kbins = (1 << F.log2nt) / 2 + 1;
  const size_t per = spec_elems(F), n = per * F.n_ang;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (size_t)gridDim.x * blockDim.x) {
    const int a = (int)(t / per);
    const size_t r = t - (size_t)a * per;
    const int j = (int)(r >> F.log2nx), m = (int)(r & (nx - 1));
    const int ms = m < nx / 2 ? m : m - nx;  // signed kx index
    // u^2 = (alpha ms)^2 + j^2 in float-float, then its square root
    const ff am = dev::ff_mul(ffi(ms), {F.ang[a].alpha_hi, F.ang[a].alpha_lo});
    const ff u2 = dev::ff_add(dev::ff_mul(am, am), dev::ff_mul(ffi(j), ffi(j)));
    float2 val = make_float2(0.f, 0.f);
    if (u2.hi > 0.f && u2.hi < (float)(kbins + 1) * (float)(kbins + 1)) {
      const ff u = dev::ff_sqrt(u2);
      float w;
      const int i0 = split_index(u, &w);
      // the one-sided spectrum extended by zeros past its last bin
      if (i0 >= 0 && i0 <= kbins - 1) {
        const float2 *P = F.P + (size_t)a * per + m;
        const float2 lo = P[(size_t)i0 * nx];
        const float2 hi = i0 + 1 <= kbins - 1 ? P[(size_t)(i0 + 1) * nx] : make_float2(0.f, 0.f);
        const float jac = (float)j / dev::ff_f(u);
        val = make_float2(((1.f - w) * lo.x + w * hi.x) * jac, ((1.f - w) * lo.y + w * hi.y) * jac);
      }
    }
    F.S[t] = val;
  }
}

__global__ void __launch_bounds__(256) k_fk_lu(FkPlan F) {
  const int nx = 1 << F.log2nx, kbins = (1 << F.log2nt) / 2 + 1;
  const size_t per = spec_elems(F), n = per * F.n_ang;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (size_t)gridDim.x * blockDim.x) {
    const int a = (int)(t / per);
    const size_t r = t - (size_t)a * per;
    const int j = (int)(r >> F.log2nx), m = (int)(r & (nx - 1));
    const int ms = m < nx / 2 ? m : m - nx;  // signed kx' index
    const FkAngleConst &A = F.ang[a];
    const ff bm = dev::ff_mul(ffi(ms), {A.beta_hi, A.beta_lo});
    const ff den = dev::ff_add(dev::ff_mul(bm, {A.sn_hi, A.sn_lo}),
                               dev::ff_mul(ffi(j), {A.cs_hi, A.cs_lo}));
    float2 val = make_float2(0.f, 0.f);
    if (den.hi > 0.f) {
      const ff num = dev::ff_add(dev::ff_mul(bm, bm), dev::ff_mul(ffi(j), ffi(j)));
      const ff u = ff_div(num, den);  // source frequency bin
      // receive wavenumber in kz' steps: j - u cos / 2 (>= 0 on the wave's branch)
      const ff kzr = dev::ff_add(ffi(j), dev::ff_neg(dev::ff_mul(u, {0.5f * A.cs_hi, 0.5f * A.cs_lo})));
      if (kzr.hi >= 0.f && u.hi < (float)kbins) {
        const ff mf = dev::ff_add(ffi(ms), dev::ff_neg(dev::ff_mul(u, {A.sb_hi, A.sb_lo})));
        float wu, wm;
        const int i0 = split_index(u, &wu);
        const int m0 = split_index(mf, &wm);
        if (i0 >= 0 && i0 <= kbins - 1) {
          const float2 *P = F.P + (size_t)a * per;
          const int ma = m0 & (nx - 1), mb = (m0 + 1) & (nx - 1);  // periodic in kx
          const float2 p00 = P[(size_t)i0 * nx + ma], p01 = P[(size_t)i0 * nx + mb];
          float2 p10 = make_float2(0.f, 0.f), p11 = p10;  // zeros past the last bin
          if (i0 + 1 <= kbins - 1) {
            p10 = P[(size_t)(i0 + 1) * nx + ma];
            p11 = P[(size_t)(i0 + 1) * nx + mb];
          }
          const float w00 = (1.f - wm) * (1.f - wu), w01 = wm * (1.f - wu);
          const float w10 = (1.f - wm) * wu, w11 = wm * wu;
          const float jac = dev::ff_f(kzr) / dev::ff_f(den);
          val = make_float2((w00 * p00.x + w01 * p01.x + w10 * p10.x + w11 * p11.x) * jac,
                            (w00 * p00.y + w01 * p01.y + w10 * p10.y + w11 * p11.y) * jac);
        }
      }
    }
    F.S[t] = val;
  }
}

__global__ void __launch_bounds__(kPostThreads) k_fk_ispace(FkPlan F) {
  extern __shared__ __align__(16) float2 sm[];
  const int nx = 1 << F.log2nx;
  float2 *x = sm, *tw = sm + nx;
  dev::fft_twiddles(tw, nx);
  float2 *row = F.S + (size_t)blockIdx.y * spec_elems(F) + (size_t)blockIdx.x * nx;
  for (int m = threadIdx.x; m < nx; m += kPostThreads) x[m] = row[m];
  __syncthreads();
  dev::fft_inverse(x, tw, F.log2nx);
  for (int e = threadIdx.x; e < nx; e += kPostThreads) row[e] = x[dev::bitrev(e, F.log2nx)];
}

__global__ void __launch_bounds__(kPostThreads) k_fk_itime(FkPlan F) {
  extern __shared__ __align__(16) float2 sm[];
  const int nt = 1 << F.log2nt, nx = 1 << F.log2nx, kbins = nt / 2 + 1;
  const int col = blockIdx.x, a = blockIdx.y;
  float2 *x = sm, *tw = sm + nt;
  dev::fft_twiddles(tw, nt);
  const float2 *I = F.S + (size_t)a * spec_elems(F) + col;
  for (int j = threadIdx.x; j < nt; j += kPostThreads)
    x[j] = j < kbins ? I[(size_t)j * nx] : make_float2(0.f, 0.f);
  __syncthreads();
  dev::fft_inverse(x, tw, F.log2nt);
  const float scale = 1.0f / ((float)nx * (float)nt);
  float2 *out = F.M + ((size_t)a * nx + col) * nt;
  for (int l = threadIdx.x; l < nt; l += kPostThreads) {
    const float2 v = x[dev::bitrev(l, F.log2nt)];
    out[l] = make_float2(v.x * scale, v.y * scale);
  }
}

__global__ void __launch_bounds__(256) k_fk_image(FkPlan F) {
  const int nt = 1 << F.log2nt, nx1 = 1 << F.log2nx;
  const size_t n = (size_t)F.nx_img * F.nz_img;
  float m = 0.f;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (size_t)gridDim.x * blockDim.x) {
    const int ix = (int)(t / F.nz_img), iz = (int)(t - (size_t)ix * F.nz_img);
    float re = 0.f, im = 0.f;
    for (int a = 0; a < F.n_ang; ++a) {
      const FkAngleConst &A = F.ang[a];
      const ff ux = dev::ff_add(
          dev::ff_add({A.ux0_hi, A.ux0_lo}, dev::ff_mul(ffi(ix), {A.uxi_hi, A.uxi_lo})),
          dev::ff_mul(ffi(iz), {A.uxk_hi, A.uxk_lo}));
      const ff uz = dev::ff_add({A.uz0_hi, A.uz0_lo}, dev::ff_mul(ffi(iz), {A.uzk_hi, A.uzk_lo}));
      // far outside the migrated image (also keeps the integer parts in range)
      if (!(ux.hi > -2.f && ux.hi < (float)(nx1 + 1) && uz.hi > -2.f && uz.hi < (float)(nt + 1)))
        continue;
      float fx, fz;
      const int i0 = split_index(ux, &fx), j0 = split_index(uz, &fz);
      const float2 *M = F.M + (size_t)a * nx1 * nt;
#pragma unroll
      for (int di = 0; di < 2; ++di) {
#pragma unroll
        for (int dj = 0; dj < 2; ++dj) {
          const int i = i0 + di, j = j0 + dj;
          if (i >= 0 && i < nx1 && j >= 0 && j < nt) {
            const float w = (di ? fx : 1.f - fx) * (dj ? fz : 1.f - fz);
            const float2 v = M[(size_t)i * nt + j];
            re = fmaf(w, v.x, re);
            im = fmaf(w, v.y, im);
          }
        }
      }
    }
    const float e = sqrtf(re * re + im * im);
    F.out_rf[t] = re;
    if (F.out_imag) F.out_imag[t] = im;
    if (F.out_env) F.out_env[t] = e;
    m = fmaxf(m, e);
  }
  if (F.ws_max) {
    __shared__ float wm[4];
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0)
      atomicMax(F.ws_max, __float_as_uint(fmaxf(fmaxf(wm[0], wm[1]), fmaxf(wm[2], wm[3]))));
  }
}

__global__ void k_fk_clear(uint32_t *w) { *w = 0u; }

int grid_for(size_t n) { return (int)std::min<size_t>((n + 255) / 256, 16384); }

}  // namespace

hipError_t launch_fk(const FkPlan &F, hipStream_t s) {
  const int nt = 1 << F.log2nt, nx = 1 << F.log2nx, kbins = nt / 2 + 1;
  const size_t lds_t = (size_t)nt * sizeof(float2) * 3 / 2;
  const size_t lds_x = (size_t)nx * sizeof(float2) * 3 / 2;
  const dim3 blk(kPostThreads);
  hipError_t e;
  if (F.ws_max) {
    hipLaunchKernelGGL(k_fk_clear, dim3(1), dim3(1), 0, s, F.ws_max);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (F.dtype == kI16)
    hipLaunchKernelGGL(k_fk_time<kI16>, dim3(F.n_ch, F.n_ang), blk, lds_t, s, F);
  else if (F.dtype == kF16)
    hipLaunchKernelGGL(k_fk_time<kF16>, dim3(F.n_ch, F.n_ang), blk, lds_t, s, F);
  else
    hipLaunchKernelGGL(k_fk_time<kF32>, dim3(F.n_ch, F.n_ang), blk, lds_t, s, F);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_fk_space, dim3(kbins, F.n_ang), blk, lds_x, s, F);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (F.method == kFkLu)
    hipLaunchKernelGGL(k_fk_lu, dim3(grid_for((size_t)kbins * nx * F.n_ang)), dim3(256), 0, s, F);
  else
    hipLaunchKernelGGL(k_fk_stolt, dim3(grid_for((size_t)kbins * nx * F.n_ang)), dim3(256), 0, s,
                       F);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_fk_ispace, dim3(kbins, F.n_ang), blk, lds_x, s, F);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_fk_itime, dim3(nx, F.n_ang), blk, lds_t, s, F);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_fk_image, dim3(grid_for((size_t)F.nx_img * F.nz_img)), dim3(256), 0, s,
                     F);
  return hipGetLastError();
}

}  // namespace pwbf
