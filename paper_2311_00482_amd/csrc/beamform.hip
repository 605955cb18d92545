// Pixel-tiled plane-wave receive beamformer for gfx950.
//
// One block owns a tile of TZ x TX pixels (TZ = 64/cpw * wz along depth, TX = wx
// along x). Each wavefront covers one pixel column segment: lane -> depth, so
// the LDS gathers of a wave hit nearly consecutive addresses and the image
// writes are contiguous. With cpw > 1 a wavefront is split into cpw lane groups
// that share the same pixels and divide the channels; their partial sums are
// reduced across lanes at the end.
//
// For every chunk of channels the block stages, per (channel, angle), a window
// of RF samples that covers every delay of every pixel of the tile, as pairs
// (u[n], u[n+1] - u[n]) so one 8-byte LDS read and one FMA interpolate. Windows
// start at floor(min transmit delay) - 1 + floor(min receive delay) - 1 over the
// tile rectangle; outside [0, n_samples) the record is zero (the zero-extended
// signal of the definition).
//
// Per pixel the transmit delays of all angles are kept in registers; per
// (pixel, channel) the receive delay (one square root) and the apodization
// weight are computed once and reused for every angle. Per (pixel, channel,
// angle) the gather costs an add, a floor, a fraction, an address, one LDS read
// and two accumulate operations. DMAS adds a square root and the signed-root
// accumulation per gather.
//
// Tiles are mapped to blocks XCD-aware: consecutive block ids go round-robin
// to the 8 XCDs, so block b takes tile (b % 8) * ceil(T/8) + b / 8 and each XCD
// walks a contiguous range of depth bands, keeping its L2 working set local.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "plan.h"

namespace pwbf {

namespace {

template <int DT>
struct RfT;
template <>
struct RfT<kI16> {
  using T = int16_t;
  static __device__ __forceinline__ float f(T v) { return (float)v; }
};
template <>
struct RfT<kF16> {
  using T = __half;
  static __device__ __forceinline__ float f(T v) { return __half2float(v); }
};
template <>
struct RfT<kF32> {
  using T = float;
  static __device__ __forceinline__ float f(T v) { return v; }
};

// Stage the windows of `rows` = chunk * A (channel, angle) pairs, one row per wavefront.
template <int DT>
__device__ __forceinline__ void stage_windows(const FramePlan &P, int e0, const int *s_lt,
                                              const float2 *s_xr, float2 *s_pairs) {
  using R = RfT<DT>;
  const typename R::T *rf = (const typename R::T *)P.rf;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int nwaves = blockDim.x / kWave;
  const int A = P.n_angles, N = P.n_channels, Ns = P.n_samples, win = P.win;
  const int rows = P.chunk * A;
  for (int r = wave; r < rows; r += nwaves) {
    const int c = r / A, a = r - c * A;
    const int e = e0 + c;
    float2 *dst = s_pairs + (size_t)r * win;
    if (e < N) {
      const int base = s_lt[a] + (int)s_xr[c].y;
      const typename R::T *src = rf + ((size_t)a * N + e) * Ns;
      for (int j = lane; j < win; j += kWave) {
        const int n = base + j;
        const float u0 = (n >= 0 && n < Ns) ? R::f(src[n]) : 0.f;
        const float u1 = (n + 1 >= 0 && n + 1 < Ns) ? R::f(src[n + 1]) : 0.f;
        dst[j] = make_float2(u0, u1 - u0);
      }
    } else {
      for (int j = lane; j < win; j += kWave) dst[j] = make_float2(0.f, 0.f);
    }
  }
}

// floor(s) as an int in one instruction (v_cvt_flr_i32_f32; pure ALU)
__device__ __forceinline__ int floor_i32(float s) {
  int n;
  asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(n) : "v"(s));
  return n;
}

// Apodization weight for r = |x - x_e| / half-aperture: hk cos(pi r) + hb inside
// the aperture (Hann: hk = hb = 1/2; boxcar: hk = 0, hb = 1), 0 outside. r is NaN
// or inf when z <= 0, which falls outside. "none" passes r = 0, so w = 1. The
// hardware cosine takes its argument in revolutions; clamping keeps it in range
// and makes the evaluation unconditional.
__device__ __forceinline__ float apod_weight(float r, float hk, float hb) {
  const float c = __builtin_amdgcn_cosf(0.5f * fminf(r, 1.f));
  return r < 1.f ? fmaf(hk, c, hb) : 0.f;
}

// AM: angles handled per pixel; PRED: AM is an upper bound and angles >= A are
// skipped (generic bucket), else exactly AM == A angles, fully unrolled.
// ONEGRP: one lane group per wavefront (cpw == 1), so the LDS window of a
// channel is the same for the whole wavefront and its address stays scalar.
template <int AM, bool PRED, int MODE, bool ONEGRP>
__device__ __forceinline__ void process_tile(const FramePlan &P, int tz, int tx, int *s_lt,
                                             float2 *s_xr, float2 *s_pairs) {
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1), wave = tid / kWave;
  const int cpw = ONEGRP ? 1 : P.cpw;
  const int ppw = kWave / cpw;
  const int pl = lane & (ppw - 1), grp = ONEGRP ? 0 : lane / ppw;
  const int wzi = wave % P.wz, wxi = wave / P.wz;
  const int TZ = ppw * P.wz, TX = P.wx;
  const int iz0 = tz * TZ, ix0 = tx * TX;
  const int iz = iz0 + wzi * ppw + pl, ix = ix0 + wxi;
  const int A = PRED ? P.n_angles : AM;
  const int N = P.n_channels, win = P.win, chunk = P.chunk;
  const float hk = P.apod == kHann ? 0.5f : 0.f, hb = 1.f - hk;

  // Lanes past the grid edge evaluate the edge pixel again and write nothing, so
  // the tile rectangle (and every window) only spans pixels of the grid.
  const int ixe = min(ix0 + TX - 1, P.nx - 1), ize = min(iz0 + TZ - 1, P.nz - 1);
  const float X = fmaf((float)min(ix, ixe), P.DX, P.X0);
  const float Z = fmaf((float)min(iz, ize), P.DZ, P.Z0);
  const float Z2 = Z * Z;
  const float Xlo = fmaf((float)ix0, P.DX, P.X0), Xhi = fmaf((float)ixe, P.DX, P.X0);
  const float Zlo = fmaf((float)iz0, P.DZ, P.Z0), Zhi = fmaf((float)ize, P.DZ, P.Z0);
  const float invA = P.apod == kNone ? 0.f : (Z > 0.f ? P.ap_k / Z : __builtin_inff());

  // Transmit delay per angle, relative to the tile's window origin. The same
  // float expression evaluated at the tile corner that minimises it gives the
  // exact float32 minimum over the tile (it is monotone in X and in Z).
  float txl[AM];
#pragma unroll
  for (int a = 0; a < AM; ++a) {
    if (!PRED || a < A) {
      const float sa = P.sa[a], ca = P.ca[a], to = P.to[a];
      const float t = fmaf(X, sa, fmaf(Z, ca, -to));
      const float xc = sa >= 0.f ? Xlo : Xhi, zc = ca >= 0.f ? Zlo : Zhi;
      const float lt = floorf(fmaf(xc, sa, fmaf(zc, ca, -to))) - 1.f;
      txl[a] = t - lt;
      if (tid == 0) s_lt[a] = (int)lt;
    }
  }

  float total = 0.f;
  float S[MODE == kDmas ? AM : 1];
  float Q = 0.f;
#pragma unroll
  for (int a = 0; a < (MODE == kDmas ? AM : 1); ++a) S[a] = 0.f;

  for (int e0 = 0; e0 < N; e0 += chunk) {
    __syncthreads();  // the previous chunk's reads are done (and s_lt is visible)
    // receive-delay origin of each channel of the chunk: the tile point nearest
    // to the element, minus one sample
    for (int c = tid; c < chunk; c += blockDim.x) {
      const float xe = P.xe[min(e0 + c, N - 1)];
      const float dxm = fmaxf(fmaxf(Xlo - xe, xe - Xhi), 0.f);
      const float dzm = Zlo > 0.f ? Zlo : (Zhi < 0.f ? -Zhi : 0.f);
      const float rmin = __builtin_amdgcn_sqrtf(fmaf(dxm, dxm, dzm * dzm));
      s_xr[c] = make_float2(xe, floorf(rmin) - 1.f);
    }
    __syncthreads();
    if (P.dtype == kI16)
      stage_windows<kI16>(P, e0, s_lt, s_xr, s_pairs);
    else if (P.dtype == kF16)
      stage_windows<kF16>(P, e0, s_lt, s_xr, s_pairs);
    else
      stage_windows<kF32>(P, e0, s_lt, s_xr, s_pairs);
    __syncthreads();

    const int wstride = win * (int)sizeof(float2);  // bytes between angle windows
    for (int k = 0; k < chunk; k += cpw) {
      const int c = ONEGRP ? k : k + grp;
      const float2 xr = s_xr[c];
      const float dxe = X - xr.x;
      const float rx = __builtin_amdgcn_sqrtf(fmaf(dxe, dxe, Z2));
      const float rxl = rx - xr.y;
      const float w = apod_weight(fabsf(dxe) * invA, hk, hb);
      const char *wb = (const char *)(s_pairs + (size_t)c * A * win);
      if constexpr (MODE == kDas) {
        float acc = 0.f;
#pragma unroll
        for (int a = 0; a < AM; ++a) {
          if (!PRED || a < A) {
            const float s = txl[a] + rxl;
            const int n = floor_i32(s);
            const float f = __builtin_amdgcn_fractf(s);
            const float2 p = *(const float2 *)(wb + a * wstride + (n << 3));
            acc += p.x;
            acc = fmaf(f, p.y, acc);
          }
        }
        total = fmaf(w, acc, total);
      } else {
        float q = 0.f;
#pragma unroll
        for (int a = 0; a < AM; ++a) {
          if (!PRED || a < A) {
            const float s = txl[a] + rxl;
            const int n = floor_i32(s);
            const float f = __builtin_amdgcn_fractf(s);
            const float2 p = *(const float2 *)(wb + a * wstride + (n << 3));
            const float v = fmaf(f, p.y, p.x);
            const float r = __builtin_amdgcn_sqrtf(fabsf(v));
            S[a] = fmaf(w, copysignf(r, v), S[a]);
            q += fabsf(v);
          }
        }
        Q = fmaf(w * w, q, Q);
      }
    }
  }

  float y;
  if constexpr (MODE == kDas) {
    for (int off = ppw; off < kWave; off <<= 1) total += __shfl_xor(total, off);
    y = total;
  } else {
    for (int off = ppw; off < kWave; off <<= 1) Q += __shfl_xor(Q, off);
    float sq = 0.f;
#pragma unroll
    for (int a = 0; a < AM; ++a) {
      if (!PRED || a < A) {
        float s = S[a];
        for (int off = ppw; off < kWave; off <<= 1) s += __shfl_xor(s, off);
        sq = fmaf(s, s, sq);
      }
    }
    y = 0.5f * (sq - Q);
  }
  if (grp == 0 && ix < P.nx && iz < P.nz) P.out[(size_t)ix * P.nz + iz] = y;
}

template <int AM, bool PRED, int MODE, bool ONEGRP>
__global__ void __launch_bounds__(kWave * kMaxWavesPerBlock) k_beamform(const FramePlan P) {
  extern __shared__ __align__(16) unsigned char smem[];
  int *s_lt = (int *)smem;
  float2 *s_xr = (float2 *)(smem + kMaxAngles * sizeof(int));
  float2 *s_pairs = s_xr + P.chunk;
  const int b = blockIdx.x;
  const int L = (b & 7) * P.tiles_per_xcd + (b >> 3);
  if (L >= P.n_tiles) return;
  if (P.ws_max && b == 0 && threadIdx.x == 0) *P.ws_max = 0u;
  const int tz = L / P.tiles_x, tx = L - tz * P.tiles_x;
  process_tile<AM, PRED, MODE, ONEGRP>(P, tz, tx, s_lt, s_xr, s_pairs);
}

template <int AM, bool PRED>
hipError_t launch_am(const FramePlan &P, hipStream_t stream) {
  const dim3 block(kWave * P.wz * P.wx);
  const dim3 grid(8 * P.tiles_per_xcd);
  const size_t lds = plan_lds_bytes(P);
  const bool one = P.cpw == 1;
  if (P.mode == kDas) {
    if (one)
      hipLaunchKernelGGL((k_beamform<AM, PRED, kDas, true>), grid, block, lds, stream, P);
    else
      hipLaunchKernelGGL((k_beamform<AM, PRED, kDas, false>), grid, block, lds, stream, P);
  } else {
    if (one)
      hipLaunchKernelGGL((k_beamform<AM, PRED, kDmas, true>), grid, block, lds, stream, P);
    else
      hipLaunchKernelGGL((k_beamform<AM, PRED, kDmas, false>), grid, block, lds, stream, P);
  }
  return hipGetLastError();
}

}  // namespace

// Angle counts 1..16 get an exactly unrolled kernel; 17..32 share a predicated one.
hipError_t launch_beamform(const FramePlan &P, hipStream_t stream) {
  switch (P.n_angles) {
#define PWBF_CASE(n) \
  case n: return launch_am<n, false>(P, stream);
    PWBF_CASE(1) PWBF_CASE(2) PWBF_CASE(3) PWBF_CASE(4) PWBF_CASE(5) PWBF_CASE(6) PWBF_CASE(7)
    PWBF_CASE(8) PWBF_CASE(9) PWBF_CASE(10) PWBF_CASE(11) PWBF_CASE(12) PWBF_CASE(13)
    PWBF_CASE(14) PWBF_CASE(15) PWBF_CASE(16)
#undef PWBF_CASE
    default:
      if (P.n_angles >= 1 && P.n_angles <= kMaxAngles) return launch_am<kMaxAngles, true>(P, stream);
      return hipErrorInvalidValue;
  }
}

}  // namespace pwbf
