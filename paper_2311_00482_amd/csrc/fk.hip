// f-k migrations (Stolt's and Lu's) for steered plane waves. Every stage runs
// over all angles of the call in one launch (blockIdx.y selects the angle), so
// even a single frame gives the chip thousands of blocks. The two methods share
// every stage but the remap. Transforms run in LDS (fft_lds.h); the two
// transposes between channel-major and bin-major data happen in LDS, inside
// blocks that hold several rows, so every global access is a contiguous run:
//
//  k_fk_time      block per (channel pair, angle): one complex FFT of two traces
//                 (Nt samples each, as real and imaginary parts), split into the
//                 two spectra; the positive bins times exp(2 pi i k c_e) (the trace
//                 advanced by its element's firing delay and shifted to t = 0) go
//                 to T, blocked by the ROWS bins of one kx-transform block
//  k_fk_space     block per (ROWS bins, angle): reads the bins k0..k0+ROWS of every
//                 channel (one contiguous block of T), FFTs along the array
//                 zero-padded to Nx, writes P[k][m]
//                 (Lu) or P[m][k] (Stolt, whose remap reads along frequency)
//  k_fk_remap     block per (ROWS image rows kz_j, angle): each cell (j, m) takes
//                 the data spectrum from P -
//                   Stolt: at bin u = sqrt((alpha m')^2 + j^2) (m' the signed
//                   index), linearly (zeros past the last bin), times j / u;
//                   Lu: at frequency bin u = (beta^2 m'^2 + j^2) /
//                   (beta m' sin + j cos) and spatial bin m' - u sin / (2 beta),
//                   bilinearly (periodic in the spatial bin), times
//                   (j - u cos / 2) / (beta m' sin + j cos), zero where the
//                   receive wavenumber j - u cos / 2 is negative -
//                 then inverse FFTs along kx, and writes the window's columns
//                 transposed, U[e][j0..j0+ROWS)
//  k_fk_itime     block per window column x1 (and angle): inverse FFT along kz of
//                 U[e][.], zero-filled to Nt, scaled by 1/(Nx Nt); stores the
//                 window's rows of M
//  k_fk_image     thread per two pixels (adjacent columns, one depth): for every
//                 angle the migrated image at (x1, z1), affine in the pixel
//                 indices, by bilinear interpolation; the complex sum over angles
//                 gives the real, imaginary and magnitude planes and the frame
//                 maximum
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

// integer part and fraction of a float-float value (fraction in [0, 1)),
// |u| < 2^24
__device__ __forceinline__ int split_index(ff u, float *frac) {
  const float fl = floorf(u.hi);
  const float f = (u.hi - fl) + u.lo;
  const float c = floorf(f);  // -1, 0 or 1: the low part crossed an integer
  *frac = f - c;
  return (int)fl + (int)c;
}

__device__ __forceinline__ int kbins_of(const FkPlan &F) { return (1 << F.log2nt) / 2 + 1; }

// Two traces per block: channels e0 = 2 blockIdx.x and e0 + 1 go in as the
// real and imaginary parts of one complex sequence z (a missing second trace
// is zero). With Z its DFT and Z(Nt) = Z(0), the traces' spectra are
// X0(k) = (Z(k) + conj Z(Nt - k)) / 2 and X1(k) = (Z(k) - conj Z(Nt - k)) / (2i).
template <int DT>
__global__ void __launch_bounds__(kPostThreads) k_fk_time(FkPlan F) {
  extern __shared__ __align__(16) float2 sm[];
  const int nt = 1 << F.log2nt, kbins = kbins_of(F), e0 = 2 * blockIdx.x, a = blockIdx.y;
  const bool two = e0 + 1 < F.n_ch;
  // the frame maximum that the image kernel, last of the call, folds into
  if (F.ws_max && blockIdx.x == 0 && blockIdx.y == 0) dev::frame_max_clear(F.ws_max, threadIdx.x);
  float2 *x = sm;
  const size_t base = ((size_t)a * F.n_ch + e0) * nt;
  const size_t base1 = two ? base + nt : base;  // every read inside the record array
  for (int k = threadIdx.x; k < nt; k += kPostThreads) {
    const float v1 = trace_sample<DT>(F.rf, base1 + k);
    x[fft::pad(k)] = make_float2(trace_sample<DT>(F.rf, base + k), two ? v1 : 0.f);
  }
  __syncthreads();
  fft::transform_any<false>(x, F.log2nt);
  const FkAngleConst &A = F.ang[a];
  const ff c0 = dev::ff_add({A.c0_hi, A.c0_lo}, dev::ff_mul(ffi(e0), {A.c1_hi, A.c1_lo}));
  const ff c1 = dev::ff_add({A.c0_hi, A.c0_lo}, dev::ff_mul(ffi(e0 + 1), {A.c1_hi, A.c1_lo}));
  // T[a][k / R][e][k mod R]: the pair's rows of a block are adjacent, 2 R bins
  const int LR = 12 - F.log2nx, R = 1 << LR;
  float2 *T0 = F.T + (size_t)a * F.n_ch * fk_kbins_padded(F.log2nt, F.log2nx) + e0 * R;
  // exp(2 pi i k c) at the thread's first bin, then by the step of kPostThreads
  // bins: a thread's bins are at most 9 products from an accurate phase
  float sn, cs;
  sincospif(2.0f * frac_revs(threadIdx.x, c0), &sn, &cs);
  float2 ph0 = make_float2(cs, sn);
  sincospif(2.0f * frac_revs(kPostThreads, c0), &sn, &cs);
  const float2 step0 = make_float2(cs, sn);
  sincospif(2.0f * frac_revs(threadIdx.x, c1), &sn, &cs);
  float2 ph1 = make_float2(cs, sn);
  sincospif(2.0f * frac_revs(kPostThreads, c1), &sn, &cs);
  const float2 step1 = make_float2(cs, sn);
  for (int k = threadIdx.x; k < kbins; k += kPostThreads) {
    const float2 z = x[fft::pad(k)], w = x[fft::pad((nt - k) & (nt - 1))];  // Z(k), Z(Nt - k)
    const float2 x0 = make_float2(0.5f * (z.x + w.x), 0.5f * (z.y - w.y));
    const float2 x1 = make_float2(0.5f * (z.y + w.y), 0.5f * (w.x - z.x));
    float2 *t = T0 + (size_t)(k >> LR) * F.n_ch * R + (k & (R - 1));
    t[0] = dev::cmul(x0, ph0);
    if (two) t[R] = dev::cmul(x1, ph1);
    ph0 = dev::cmul(ph0, step0);
    ph1 = dev::cmul(ph1, step1);
  }
}

template <int L, int METHOD>
__global__ void __launch_bounds__(kPostThreads) k_fk_space(FkPlan F) {
  constexpr int nx = 1 << L, ROWS = kFkRowPoints >> L, stride = fft::row_stride(nx, ROWS);
  extern __shared__ __align__(16) float2 sm[];
  float2 *x = sm;
  const int kbins = kbins_of(F), k0 = blockIdx.x * ROWS, a = blockIdx.y;
  // the block's bins of every channel are one contiguous run of T (bins past
  // the last are never written and read as zero)
  const float2 *T = F.T + ((size_t)a * fk_kbins_padded(F.log2nt, L) + k0) * F.n_ch;
  for (int t = threadIdx.x; t < nx * ROWS; t += kPostThreads) {
    const int e = t / ROWS, r = t - e * ROWS, k = k0 + r;
    x[r * stride + fft::pad(e)] = (e < F.n_ch && k < kbins) ? T[t] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  fft::transform<L, false, ROWS>(x);
  float2 *P = F.P + (size_t)a * kbins * nx;
  if (METHOD == kFkStolt) {
    // Stolt's remap reads along frequency at fixed kx: store P[m][k], consecutive
    // threads on consecutive bins
    for (int t = threadIdx.x; t < nx * ROWS; t += kPostThreads) {
      const int m = t / ROWS, r = t - m * ROWS, k = k0 + r;
      if (k < kbins) P[(size_t)m * kbins + k] = x[r * stride + fft::pad(m)];
    }
  } else {
    for (int t = threadIdx.x; t < nx * ROWS; t += kPostThreads) {
      const int r = t >> L, m = t & (nx - 1), k = k0 + r;
      if (k < kbins) P[(size_t)k * nx + m] = x[r * stride + fft::pad(m)];
    }
  }
}

// Float-float helpers with hardware reciprocal and square root in the leading
// term: the error-free residual of the correction step absorbs their ulp-level
// error, so the results match the correctly rounded versions to ~1e-14.
__device__ __forceinline__ ff quick_two_sum(float a, float b) {  // |a| >= |b|
#pragma clang fp contract(off)
  const float s = a + b;
  return {s, b - (s - a)};
}

__device__ __forceinline__ ff ff_sqrt_hw(ff a) {  // a.hi > 0
#pragma clang fp contract(off)
  const float s = __builtin_amdgcn_sqrtf(a.hi);
  const float r = fmaf(-s, s, a.hi) + a.lo;
  return quick_two_sum(s, r * (0.5f * __builtin_amdgcn_rcpf(s)));
}

__device__ __forceinline__ ff ff_div_hw(ff a, ff b) {  // b.hi != 0
#pragma clang fp contract(off)
  const float rb = __builtin_amdgcn_rcpf(b.hi);
  const float q1 = a.hi * rb;
  const float p = q1 * b.hi, e = fmaf(q1, b.hi, -p);
  const float r = ((a.hi - p) - e) + (a.lo - q1 * b.lo);
  return quick_two_sum(q1, r * rb);
}

// v - u c for float-float v, u, c (c's product split exactly)
__device__ __forceinline__ ff ff_sub_mul(ff v, ff u, float c_hi, float c_lo) {
#pragma clang fp contract(off)
  const float p = u.hi * c_hi, e = fmaf(u.hi, c_hi, -p) + (u.hi * c_lo + u.lo * c_hi);
  const ff d = dev::two_sum(v.hi, -p);
  return dev::two_sum(d.hi, d.lo + (v.lo - e));
}

// The remap bodies below leave floating-point contraction on (their weights
// and sums may fuse into FMAs); every error-free step sits in a helper that
// turns it off.

// The cells of a remap block: per thread a fixed set of kx columns m (one when
// Nx <= 256) and, for each, every row of the block that falls to the thread.
template <int L>
struct RemapCells {
  static constexpr int nx = 1 << L, ROWS = kFkRowPoints >> L;
  static constexpr int MPT = nx >= kPostThreads ? nx / kPostThreads : 1;  // columns per thread
  static constexpr int RSTEP = nx >= kPostThreads ? 1 : kPostThreads / nx;  // rows apart
  __device__ static int m(int mi) {
    return nx >= kPostThreads ? (int)threadIdx.x + kPostThreads * mi : (int)threadIdx.x & (nx - 1);
  }
  __device__ static int r0() { return nx >= kPostThreads ? 0 : (int)threadIdx.x >> L; }
};

// Stolt's remap of the block's rows: the cell (j, m) takes the data spectrum at
// bin u = sqrt((alpha m')^2 + j^2), linearly (zeros past the last bin), times
// j / u. P is stored [m][k]; consecutive threads take consecutive rows j of one
// column, so their bins u are close and the gathers contiguous.
template <int L>
__device__ __forceinline__ void stolt_rows(const FkAngleConst &A, const float2 *__restrict__ P,
                                           int j0, int kbins, float2 *x) {
  constexpr int nx = 1 << L, ROWS = kFkRowPoints >> L, LR = 12 - L;
  constexpr int stride = fft::row_stride(nx, ROWS);
  static_assert((1 << LR) == ROWS, "rows of a block");
#pragma unroll 4
  for (int t = threadIdx.x; t < kFkRowPoints; t += kPostThreads) {
    const int r = t & (ROWS - 1), m = t >> LR, ms = m < nx / 2 ? m : m - nx;
    const int j = min(j0 + r, kbins - 1);  // rows past the last bin store zero below
    const float fj = (float)j;
    const ff am = dev::ff_mul(ffi(ms), {A.m0_hi, A.m0_lo});
    const ff am2 = dev::ff_mul(am, am);  // (alpha m')^2
    const ff u2 = dev::two_sum(am2.hi, fj * fj);  // j^2 < 2^24 is exact
    const ff u2n = dev::two_sum(u2.hi, u2.lo + am2.lo);
    const bool in_band = u2n.hi > 0.f && u2n.hi < (float)(kbins + 1) * (float)(kbins + 1);
    const ff u = ff_sqrt_hw(in_band ? u2n : ff{1.f, 0.f});
    float w;
    const int i0 = split_index(u, &w);
    // clamped loads, always issued; taps outside the spectrum weigh zero
    const bool ok = in_band && i0 >= 0 && i0 <= kbins - 1 && j0 + r < kbins;
    const int ia = ok ? i0 : 0, ib = min(ia + 1, kbins - 1);
    const unsigned cb = (unsigned)(m * kbins);  // < 2^21 cells per angle
    const float2 lo = P[cb + ia], hi = P[cb + ib];
    const float jac = ok ? fj * __builtin_amdgcn_rcpf(u.hi) : 0.f;
    const float wl = (1.f - w) * jac, wh = (ok && i0 + 1 <= kbins - 1) ? w * jac : 0.f;
    x[r * stride + fft::pad(m)] = make_float2(wl * lo.x + wh * hi.x, wl * lo.y + wh * hi.y);
  }
}

// Lu's remap of the block's rows: the cell (j, m) takes the data spectrum at
// frequency bin u = (beta^2 m'^2 + j^2) / (beta m' sin + j cos) and spatial bin
// m' - u sin / (2 beta), bilinearly (periodic in the spatial bin, zeros past the
// last frequency bin), times (j - u cos / 2) / (beta m' sin + j cos); zero where
// the receive wavenumber j - u cos / 2 is negative or the denominator is not
// positive.
template <int L>
__device__ __forceinline__ void lu_rows(const FkAngleConst &A, const float2 *__restrict__ P,
                                        int j0, int kbins, float2 *x) {
  using C = RemapCells<L>;
  constexpr int stride = fft::row_stride(C::nx, C::ROWS);
  const float ch = 0.5f * A.m2_hi, cl = 0.5f * A.m2_lo;  // cos / 2
  for (int mi = 0; mi < C::MPT; ++mi) {
    const int m = C::m(mi), ms = m < C::nx / 2 ? m : m - C::nx;
    const ff bm = dev::ff_mul(ffi(ms), {A.m0_hi, A.m0_lo});
    const ff bm2 = dev::ff_mul(bm, bm);                     // beta^2 m'^2
    const ff bms = dev::ff_mul(bm, {A.m1_hi, A.m1_lo});     // beta m' sin
#pragma unroll 2
    for (int r = C::r0(); r < C::ROWS; r += C::RSTEP) {
      const int j = min(j0 + r, kbins - 1);
      const float fj = (float)j;
      // den = beta m' sin + j cos
      const float pc = fj * A.m2_hi, ec = fmaf(fj, A.m2_hi, -pc) + fj * A.m2_lo;
      const ff d0 = dev::two_sum(bms.hi, pc);
      const ff den = dev::two_sum(d0.hi, d0.lo + (bms.lo + ec));
      const bool pos = den.hi > 0.f;
      // num = beta^2 m'^2 + j^2
      const ff n0 = dev::two_sum(bm2.hi, fj * fj);
      const ff num = dev::two_sum(n0.hi, n0.lo + bm2.lo);
      const ff u = ff_div_hw(num, pos ? den : ff{1.f, 0.f});  // source frequency bin
      // the receive wavenumber j - u cos / 2 only weighs the cell: float suffices
      const float kzr = fmaf(-u.lo, ch, fmaf(-u.hi, ch, fj)) - u.hi * cl;
      const bool branch = pos && kzr >= 0.f && u.hi < (float)kbins && j0 + r < kbins;
      const ff mf = ff_sub_mul(ffi(ms), u, A.m3_hi, A.m3_lo);  // spatial bin
      float wu, wm;
      const int i0 = split_index(branch ? u : ff{0.f, 0.f}, &wu);
      const int m0 = split_index(branch ? mf : ff{0.f, 0.f}, &wm);
      const bool ok = branch && i0 >= 0 && i0 <= kbins - 1;
      const int ia = ok ? i0 : 0, ib = min(ia + 1, kbins - 1);
      const int ma = m0 & (C::nx - 1), mb = (m0 + 1) & (C::nx - 1);  // periodic in kx
      const unsigned ra = (unsigned)(ia * C::nx), rb = (unsigned)(ib * C::nx);  // < 2^21
      const float2 p00 = P[ra + ma], p01 = P[ra + mb], p10 = P[rb + ma], p11 = P[rb + mb];
      const float jac = ok ? kzr * __builtin_amdgcn_rcpf(den.hi) : 0.f;
      const float hw = (ok && i0 + 1 <= kbins - 1) ? wu : 0.f;  // zeros past the last bin
      const float w00 = (1.f - wm) * (1.f - wu) * jac, w01 = wm * (1.f - wu) * jac;
      const float w10 = (1.f - wm) * hw * jac, w11 = wm * hw * jac;
      x[r * stride + fft::pad(m)] =
          make_float2(w00 * p00.x + w01 * p01.x + w10 * p10.x + w11 * p11.x,
                      w00 * p00.y + w01 * p01.y + w10 * p10.y + w11 * p11.y);
    }
  }
}

template <int L, int METHOD>
__global__ void __launch_bounds__(kPostThreads) k_fk_remap(FkPlan F) {
  constexpr int nx = 1 << L, ROWS = kFkRowPoints >> L, stride = fft::row_stride(nx, ROWS);
  extern __shared__ __align__(16) float2 sm[];
  float2 *x = sm;
  const int kbins = kbins_of(F), j0 = blockIdx.x * ROWS, a = blockIdx.y;
  const FkAngleConst &A = F.ang[a];
  const float2 *P = F.P + (size_t)a * kbins * nx;
  if (METHOD == kFkLu)
    lu_rows<L>(A, P, j0, kbins, x);
  else
    stolt_rows<L>(A, P, j0, kbins, x);
  __syncthreads();
  fft::transform<L, true, ROWS>(x);
  // the window's columns, transposed: consecutive threads take consecutive rows
  float2 *U = F.U + (size_t)a * nx * kbins;
  for (int t = threadIdx.x; t < A.ncol * ROWS; t += kPostThreads) {
    const int c = t / ROWS, r = t - c * ROWS, j = j0 + r, e = A.col0 + c;
    if (j < kbins) U[(size_t)e * kbins + j] = x[r * stride + fft::pad(e)];
  }
}

__global__ void __launch_bounds__(kPostThreads) k_fk_itime(FkPlan F) {
  extern __shared__ __align__(16) float2 sm[];
  const int a = blockIdx.y;
  const FkAngleConst &A = F.ang[a];
  if ((int)blockIdx.x >= A.ncol) return;  // the whole block: outside this angle's window
  const int nt = 1 << F.log2nt, nx = 1 << F.log2nx, kbins = kbins_of(F);
  const int col = A.col0 + blockIdx.x;
  float2 *x = sm;
  const float2 *I = F.U + ((size_t)a * nx + col) * kbins;
  for (int j = threadIdx.x; j < nt; j += kPostThreads)
    x[fft::pad(j)] = j < kbins ? I[j] : make_float2(0.f, 0.f);
  __syncthreads();
  fft::transform_any<true>(x, F.log2nt);
  const float scale = 1.0f / ((float)nx * (float)nt);
  float2 *out = F.M + ((size_t)a * nx + col) * nt;
  for (int l = A.row0 + threadIdx.x; l < A.row0 + A.nrow; l += kPostThreads) {
    const float2 v = x[fft::pad(l)];
    out[l] = make_float2(v.x * scale, v.y * scale);
  }
}

// Integer part and fraction of v0 + k c for float-float v0, c and an integer
// 0 <= k < 2^24: the product split exactly (one FMA), the large terms summed
// with an error-free addition, the small ones added once; the fraction is
// accurate to ~1e-7 of an index step. Returns false when the value is outside
// (lo, hi), before any conversion to an integer.
__device__ __forceinline__ bool map_index(float v0h, float v0l, float k, float ch, float cl,
                                          float lo, float hi, int *idx, float *frac) {
#pragma clang fp contract(off)
  const float p = k * ch, e = fmaf(k, ch, -p);
  const ff t = dev::two_sum(v0h, p);
  if (!(t.hi > lo && t.hi < hi)) return false;
  const float small = (t.lo + (v0l + e)) + k * cl;
  const float fl = floorf(t.hi);
  const float f = (t.hi - fl) + small;
  const float c = floorf(f);  // -1, 0 or 1: the small terms crossed an integer
  *idx = (int)fl + (int)c;
  *frac = f - c;
  return true;
}

// Adds the bilinear value of one angle's migrated image M at column i0 + fx,
// row j0 + fz to (re, im); taps outside the angle's window are outside
// [0, Nx) x [0, Nt) too (the window holds every tap inside, with a margin), so
// they read as zero.
__device__ __forceinline__ void add_taps(const float2 *M, int nt, const FkAngleConst &A, int i0,
                                         float fx, int j0, float fz, float &re, float &im) {
  const int c1 = A.col0 + A.ncol, r1 = A.row0 + A.nrow;
  if (i0 >= A.col0 && i0 + 1 < c1 && j0 >= A.row0 && j0 + 1 < r1) {
    const float2 *q = M + (unsigned)(i0 * nt + j0);
    const float2 v00 = q[0], v01 = q[1], v10 = q[nt], v11 = q[nt + 1];
    const float w00 = (1.f - fx) * (1.f - fz), w01 = (1.f - fx) * fz;
    const float w10 = fx * (1.f - fz), w11 = fx * fz;
    re += w00 * v00.x + w01 * v01.x + w10 * v10.x + w11 * v11.x;
    im += w00 * v00.y + w01 * v01.y + w10 * v10.y + w11 * v11.y;
  } else {
#pragma unroll
    for (int di = 0; di < 2; ++di) {
#pragma unroll
      for (int dj = 0; dj < 2; ++dj) {
        const int i = i0 + di, j = j0 + dj;
        if (i >= A.col0 && i < c1 && j >= A.row0 && j < r1) {
          const float w = (di ? fx : 1.f - fx) * (dj ? fz : 1.f - fz);
          const float2 v = M[(unsigned)(i * nt + j)];
          re = fmaf(w, v.x, re);
          im = fmaf(w, v.y, im);
        }
      }
    }
  }
}

// Pixel (ix, iz) reads column ux0 + ix uxi + iz uxk and row uz0 + iz uzk of the
// migrated image of each angle. A block is a depth run of two image columns:
// each column's lateral base ux0 + ix uxi (float-float) is formed once per
// angle and shared through LDS, and a thread's two pixels share the row map.
__global__ void __launch_bounds__(256) k_fk_image(FkPlan F, int zchunks) {
  const int nt = 1 << F.log2nt, nx1 = 1 << F.log2nx;
  const int px = blockIdx.x / zchunks, iz = (blockIdx.x - px * zchunks) * 256 + threadIdx.x;
  const int ix0 = 2 * px;
  const bool two = ix0 + 1 < F.nx_img, mine = iz < F.nz_img;
  const float fiz = (float)iz;
  __shared__ float2 s_xb[2][kMaxAngles];
  {
    const int c = threadIdx.x >> 5, a = threadIdx.x & 31;  // column c of the pair, angle a
    if (c < 2 && a < F.n_ang) {
#pragma clang fp contract(off)
      const FkAngleConst &A = F.ang[a];
      const float fix = (float)(ix0 + c);
      const float p = fix * A.uxi_hi, e = fmaf(fix, A.uxi_hi, -p);
      const ff t = dev::two_sum(A.ux0_hi, p);
      const ff b = dev::two_sum(t.hi, (t.lo + (A.ux0_lo + e)) + fix * A.uxi_lo);
      s_xb[c][a] = make_float2(b.hi, b.lo);
    }
  }
  __syncthreads();
  float re0 = 0.f, im0 = 0.f, re1 = 0.f, im1 = 0.f;
  for (int a = 0; a < F.n_ang; ++a) {
    const FkAngleConst &A = F.ang[a];
    if (A.ncol == 0) continue;
    // far outside the migrated image: nothing to read (and no integer overflow)
    int j0;
    float fz;
    if (!map_index(A.uz0_hi, A.uz0_lo, fiz, A.uzk_hi, A.uzk_lo, -2.f, (float)(nt + 1), &j0, &fz))
      continue;
    const float2 *M = F.M + (size_t)a * nx1 * nt;
    int i0;
    float fx;
    const float2 xb0 = s_xb[0][a], xb1 = s_xb[1][a];
    if (map_index(xb0.x, xb0.y, fiz, A.uxk_hi, A.uxk_lo, -2.f, (float)(nx1 + 1), &i0, &fx))
      add_taps(M, nt, A, i0, fx, j0, fz, re0, im0);
    if (two && map_index(xb1.x, xb1.y, fiz, A.uxk_hi, A.uxk_lo, -2.f, (float)(nx1 + 1), &i0, &fx))
      add_taps(M, nt, A, i0, fx, j0, fz, re1, im1);
  }
  const float e0 = sqrtf(re0 * re0 + im0 * im0), e1 = sqrtf(re1 * re1 + im1 * im1);
  if (mine) {
    const size_t t = (size_t)ix0 * F.nz_img + iz;
    F.out_rf[t] = re0;
    if (F.out_imag) F.out_imag[t] = im0;
    if (F.out_env) F.out_env[t] = e0;
    if (two) {
      const size_t t1 = t + F.nz_img;
      F.out_rf[t1] = re1;
      if (F.out_imag) F.out_imag[t1] = im1;
      if (F.out_env) F.out_env[t1] = e1;
    }
  }
  if (F.ws_max) {
    __shared__ float wm[4];
    float m = mine ? fmaxf(e0, two ? e1 : 0.f) : 0.f;
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0)
      dev::frame_max_fold(F.ws_max, fmaxf(fmaxf(wm[0], wm[1]), fmaxf(wm[2], wm[3])));
  }
}

template <int L>
hipError_t launch_rows(const FkPlan &F, hipStream_t s) {
  constexpr int ROWS = kFkRowPoints >> L;
  const int kbins = (1 << F.log2nt) / 2 + 1;
  const dim3 grid((kbins + ROWS - 1) / ROWS, F.n_ang), blk(kPostThreads);
  const size_t lds = fft::lds_bytes(1 << L, ROWS);
  if (F.method == kFkLu) {
    hipLaunchKernelGGL((k_fk_space<L, kFkLu>), grid, blk, lds, s, F);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_fk_remap<L, kFkLu>), grid, blk, lds, s, F);
  } else {
    hipLaunchKernelGGL((k_fk_space<L, kFkStolt>), grid, blk, lds, s, F);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_fk_remap<L, kFkStolt>), grid, blk, lds, s, F);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_fk(const FkPlan &F, int ncol_max, hipStream_t s) {
  const int nt = 1 << F.log2nt;
  const size_t lds_t = fft::lds_bytes(nt, 1);
  const dim3 blk(kPostThreads);
  hipError_t e;
  const dim3 pairs((F.n_ch + 1) / 2, F.n_ang);  // two traces per block
  if (F.dtype == kI16)
    hipLaunchKernelGGL(k_fk_time<kI16>, pairs, blk, lds_t, s, F);
  else if (F.dtype == kF16)
    hipLaunchKernelGGL(k_fk_time<kF16>, pairs, blk, lds_t, s, F);
  else
    hipLaunchKernelGGL(k_fk_time<kF32>, pairs, blk, lds_t, s, F);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  switch (F.log2nx) {
    case 2: e = launch_rows<2>(F, s); break;
    case 3: e = launch_rows<3>(F, s); break;
    case 4: e = launch_rows<4>(F, s); break;
    case 5: e = launch_rows<5>(F, s); break;
    case 6: e = launch_rows<6>(F, s); break;
    case 7: e = launch_rows<7>(F, s); break;
    case 8: e = launch_rows<8>(F, s); break;
    case 9: e = launch_rows<9>(F, s); break;
    case 10: e = launch_rows<10>(F, s); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  if (ncol_max > 0) {
    hipLaunchKernelGGL(k_fk_itime, dim3(ncol_max, F.n_ang), blk, lds_t, s, F);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const int zchunks = (F.nz_img + 255) / 256;
  hipLaunchKernelGGL(k_fk_image, dim3((F.nx_img + 1) / 2 * zchunks), dim3(256), 0, s, F,
                     zchunks);
  return hipGetLastError();
}

}  // namespace pwbf
