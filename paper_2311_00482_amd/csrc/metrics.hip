// Image metrics of the evaluation (Section II-D) on an envelope image
// [nx][nz]: contrast of cysts, Eq. (5) CR and Eq. (6) CNR, and the lateral and
// axial full width at half maximum of point targets.
//
// Regions are discs in pixel units. A pixel is inside when
// ((ix - cx) sx)^2 + ((iz - cz) sz)^2 <= 1, evaluated with separately rounded
// float32 operations (no fused multiply-add), so that the decision is
// reproducible bit for bit on the host. One block per cyst or target; sums are
// taken per thread in a fixed stride order and combined by a fixed-shape tree,
// so results do not depend on scheduling.
#include <hip/hip_runtime.h>

#include "frame_max.h"
#include "metrics.h"

namespace pwbf {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ bool inside(const DiscPix &d, int ix, int iz) {
  // every operation rounded on its own: a fused u*u + v*v would decide pixels on
  // the circle differently from the host
#pragma clang fp contract(off)
  const float u = ((float)ix - d.cx) * d.sx;
  const float v = ((float)iz - d.cz) * d.sz;
  return u * u + v * v <= 1.0f;
}

// Sum over the block in a fixed order: LDS tree over the 256 partials.
__device__ float block_sum(float v, float *sh) {
  __syncthreads();
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  return sh[0];
}

// count, mean and population standard deviation of env over the disc (two passes)
__device__ void disc_stats(const float *env, int nz, const DiscPix &d, float *sh, int *n_out,
                           float *mu_out, float *sd_out) {
  const int w = d.ix1 - d.ix0 + 1, h = d.iz1 - d.iz0 + 1;
  const int total = w > 0 && h > 0 ? w * h : 0;
  float s = 0.f, c = 0.f;
  for (int k = threadIdx.x; k < total; k += kThreads) {
    const int ix = d.ix0 + k / h, iz = d.iz0 + k % h;
    if (inside(d, ix, iz)) {
      s += env[(size_t)ix * nz + iz];
      c += 1.f;
    }
  }
  const float n = block_sum(c, sh);
  const float mu = block_sum(s, sh) / n;
  float q = 0.f;
  for (int k = threadIdx.x; k < total; k += kThreads) {
    const int ix = d.ix0 + k / h, iz = d.iz0 + k % h;
    if (inside(d, ix, iz)) {
      const float e = env[(size_t)ix * nz + iz] - mu;
      q = fmaf(e, e, q);
    }
  }
  const float var = block_sum(q, sh) / n;
  *n_out = (int)n;
  *mu_out = n > 0.f ? mu : __builtin_nanf("");
  *sd_out = n > 0.f ? sqrtf(var) : __builtin_nanf("");
}

// CR (Eq. (5)) and CNR (Eq. (6)) of env between two discs; the result is
// complete in thread 0
__device__ pwbf_contrast disc_contrast(const float *env, int nz, const DiscPix &in,
                                       const DiscPix &bg, float *sh) {
  int n_in, n_bg;
  float mu_in, sd_in, mu_bg, sd_bg;
  disc_stats(env, nz, in, sh, &n_in, &mu_in, &sd_in);
  disc_stats(env, nz, bg, sh, &n_bg, &mu_bg, &sd_bg);
  pwbf_contrast r;
  r.mu_in = mu_in;
  r.mu_out = mu_bg;
  r.sigma_in = sd_in;
  r.sigma_out = sd_bg;
  r.cr_db = (mu_in > 0.f && mu_bg > 0.f) ? 20.0f * log10f(mu_in / mu_bg) : __builtin_nanf("");
  const float den = sqrtf(0.5f * (sd_in * sd_in + sd_bg * sd_bg));
  r.cnr = den > 0.f ? (mu_in - mu_bg) / den : __builtin_nanf("");
  r.n_in = n_in;
  r.n_out = n_bg;
  return r;
}

__global__ void __launch_bounds__(kThreads)
    k_contrast(const float *__restrict__ env, int nz, CystSet cs, pwbf_contrast *__restrict__ out) {
  __shared__ float sh[kThreads];
  const int k = blockIdx.x;
  const pwbf_contrast r = disc_contrast(env, nz, cs.in[k], cs.out[k], sh);
  if (threadIdx.x == 0) out[k] = r;
}

// the block's item: the k with block0[k] <= b < block0[k + 1]
__device__ __forceinline__ int quality_item(const QualityList &ql, int b) {
  int lo = 0, hi = ql.n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ql.block0[mid] <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// (count, sum, sum of squares) of env over the disc's pixels in columns
// [c0, c1] of its box
__device__ float4 disc_partial(const float *env, int nz, const DiscPix &d, int c0, int c1,
                               float *sh) {
  const int h = d.iz1 - d.iz0 + 1, w = c1 - c0 + 1;
  const int total = w > 0 && h > 0 ? w * h : 0;
  float c = 0.f, s = 0.f, q = 0.f;
  for (int k = threadIdx.x; k < total; k += kThreads) {
    const int ix = c0 + k / h, iz = d.iz0 + k % h;
    if (inside(d, ix, iz)) {
      const float e = env[(size_t)ix * nz + iz];
      c += 1.f;
      s += e;
      q = fmaf(e, e, q);
    }
  }
  const float n = block_sum(c, sh), sum = block_sum(s, sh), sq = block_sum(q, sh);
  return make_float4(n, sum, sq, 0.f);
}

// mean and population deviation from combined partials
__device__ __forceinline__ void stats_of(float n, float s, float q, float *mu, float *sd) {
  if (!(n > 0.f)) {
    *mu = __builtin_nanf("");
    *sd = __builtin_nanf("");
    return;
  }
  const float m = s / n;
  *mu = m;
  *sd = sqrtf(fmaxf(q / n - m * m, 0.f));
}

// one block per column chunk of a disc of a checked slot
__global__ void __launch_bounds__(kThreads)
    k_quality(const QualityPlan *__restrict__ plans, QualityList ql, QualityOut *__restrict__ out,
              float4 *__restrict__ partials, int *__restrict__ counters) {
  __shared__ float sh[kThreads];
  __shared__ bool s_last;
  const int k = quality_item(ql, blockIdx.x);
  const QualityPlan &Q = plans[ql.plan[k]];
  const int b = blockIdx.x - ql.block0[k];
  const bool in = b < Q.chunks_in;
  const DiscPix &d = in ? Q.in : Q.out;
  const int chunk = in ? b : b - Q.chunks_in, cols = in ? Q.cols_in : Q.cols_out;
  const int c0 = d.ix0 + chunk * cols, c1 = min(d.ix1, c0 + cols - 1);
  const float4 p = disc_partial(Q.env, Q.nz, d, c0, c1, sh);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = p;
    __threadfence();  // the partial is visible before the count says so
    const int nb = ql.block0[k + 1] - ql.block0[k];
    s_last = atomicAdd(&counters[k], 1) == nb - 1;
  }
  __syncthreads();
  if (!s_last) return;  // uniform over the block
  __threadfence();
  const float m = dev::frame_max_read(Q.ws_max);
  if (threadIdx.x == 0) {
    // the slot's partials in chunk order: inside disc, then background
    float ni = 0.f, si = 0.f, qi = 0.f, no = 0.f, so = 0.f, qo = 0.f;
    const int first = ql.block0[k];
    for (int j = 0; j < Q.chunks_in; ++j) {
      const float4 v = partials[first + j];
      ni += v.x;
      si += v.y;
      qi += v.z;
    }
    for (int j = 0; j < Q.chunks_out; ++j) {
      const float4 v = partials[first + Q.chunks_in + j];
      no += v.x;
      so += v.y;
      qo += v.z;
    }
    float mu_in, sd_in, mu_bg, sd_bg;
    stats_of(ni, si, qi, &mu_in, &sd_in);
    stats_of(no, so, qo, &mu_bg, &sd_bg);
    QualityOut r;
    r.frame_max = m;
    r.cr_db = (mu_in > 0.f && mu_bg > 0.f) ? 20.0f * log10f(mu_in / mu_bg) : __builtin_nanf("");
    const float den = sqrtf(0.5f * (sd_in * sd_in + sd_bg * sd_bg));
    r.cnr = den > 0.f ? (mu_in - mu_bg) / den : __builtin_nanf("");
    r.ok = (m > 0.f && r.cr_db <= Q.max_cr_db) ? 1 : 0;  // a NaN CR fails
    out[k] = r;
    counters[k] = 0;  // ready for the next batch that uses this buffer
  }
}

// where the line through (0, a) and (1, b) crosses the half level, as a
// fraction of the pixel step from a
__device__ __forceinline__ float cross(float a, float b, float half) {
  return (half - a) / (b - a);
}

__global__ void __launch_bounds__(kThreads)
    k_resolution(const float *__restrict__ env, int nx, int nz, float dx, float dz, TargetSet ts,
                 pwbf_resolution *__restrict__ out) {
  __shared__ float sv[kThreads];
  __shared__ int si[kThreads];
  const DiscPix d = ts.t[blockIdx.x];
  const int w = d.ix1 - d.ix0 + 1, h = d.iz1 - d.iz0 + 1;
  const int total = w > 0 && h > 0 ? w * h : 0;
  // argmax; among equal values the smallest flat index ix * nz + iz
  float best = -__builtin_inff();
  int bi = -1;
  for (int k = threadIdx.x; k < total; k += kThreads) {
    const int ix = d.ix0 + k / h, iz = d.iz0 + k % h;
    if (!inside(d, ix, iz)) continue;
    const int flat = ix * nz + iz;
    const float v = env[flat];
    if (v > best || (v == best && (bi < 0 || flat < bi))) {
      best = v;
      bi = flat;
    }
  }
  sv[threadIdx.x] = best;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      const float v = sv[threadIdx.x + s];
      const int i = si[threadIdx.x + s];
      if (i >= 0 && (si[threadIdx.x] < 0 || v > sv[threadIdx.x] ||
                     (v == sv[threadIdx.x] && i < si[threadIdx.x]))) {
        sv[threadIdx.x] = v;
        si[threadIdx.x] = i;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  pwbf_resolution r;
  const float nanv = __builtin_nanf("");
  r.peak = nanv;
  r.fwhm_x = nanv;
  r.fwhm_z = nanv;
  r.ix = -1;
  r.iz = -1;
  const int flat = si[0];
  if (flat >= 0) {
    const int ix = flat / nz, iz = flat - (flat / nz) * nz;
    const float peak = sv[0], half = peak * 0.5f;
    r.peak = peak;
    r.ix = ix;
    r.iz = iz;
    // lateral profile: row iz, stride nz
    int i = ix;
    while (i >= 0 && env[(size_t)i * nz + iz] >= half) --i;
    int j = ix;
    while (j < nx && env[(size_t)j * nz + iz] >= half) ++j;
    if (i >= 0 && j < nx) {
      const float left =
          (float)i + cross(env[(size_t)i * nz + iz], env[(size_t)(i + 1) * nz + iz], half);
      const float right =
          (float)(j - 1) + cross(env[(size_t)(j - 1) * nz + iz], env[(size_t)j * nz + iz], half);
      r.fwhm_x = (right - left) * dx;
    }
    // axial profile: column ix, contiguous
    const float *col = env + (size_t)ix * nz;
    i = iz;
    while (i >= 0 && col[i] >= half) --i;
    j = iz;
    while (j < nz && col[j] >= half) ++j;
    if (i >= 0 && j < nz) {
      const float left = (float)i + cross(col[i], col[i + 1], half);
      const float right = (float)(j - 1) + cross(col[j - 1], col[j], half);
      r.fwhm_z = (right - left) * dz;
    }
  }
  out[blockIdx.x] = r;
}

}  // namespace

hipError_t launch_quality(const QualityPlan *plans, const QualityList &ql, QualityOut *out,
                          float4 *partials, int *counters, hipStream_t stream) {
  if (ql.n < 1) return hipSuccess;
  hipLaunchKernelGGL(k_quality, dim3(ql.block0[ql.n]), dim3(kThreads), 0, stream, plans, ql, out,
                     partials, counters);
  return hipGetLastError();
}

hipError_t launch_contrast(const float *env, int nz, const CystSet &cs, int n, pwbf_contrast *out,
                           hipStream_t stream) {
  hipLaunchKernelGGL(k_contrast, dim3(n), dim3(kThreads), 0, stream, env, nz, cs, out);
  return hipGetLastError();
}

hipError_t launch_resolution(const float *env, int nx, int nz, float dx, float dz,
                             const TargetSet &ts, int n, pwbf_resolution *out,
                             hipStream_t stream) {
  hipLaunchKernelGGL(k_resolution, dim3(n), dim3(kThreads), 0, stream, env, nx, nz, dx, dz, ts,
                     out);
  return hipGetLastError();
}

}  // namespace pwbf
