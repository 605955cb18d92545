#pragma once
// Device code of the pixel-tiled plane-wave receive beamformer (gfx950),
// shared by the single-frame kernels and the persistent batch kernel.
//
// One block owns a tile of TZ x TX pixels. A wavefront's lanes run along depth
// first (lz lanes) and then along x, so the LDS gathers of a wave hit nearly
// consecutive addresses and the image writes are contiguous runs. With cpw > 1
// a wavefront is split into cpw lane groups that share the same pixels and
// divide the channels; their partial sums are reduced across lanes at the end.
//
// For every chunk of channels the block stages, per (channel, angle), a window
// of RF samples that covers every delay of every pixel of the tile, as pairs
// (DAS: the line through u[n] and u[n+1] in the delay coordinate; DMAS: u[n]
// and u[n+1] - u[n]) so one 8-byte LDS read and one FMA interpolate. Windows
// start at floor(min transmit delay) - 1 + floor(min receive delay) - 1 over the
// tile rectangle; outside [0, n_samples) the record is zero (the zero-extended
// signal of the definition).
//
// Per pixel the transmit delays of all angles are kept in registers; per
// (pixel, channel) the receive delay (one square root) and the apodization
// weight are computed once and reused for every angle. Per (pixel, channel,
// angle) the DAS gather costs an add, a floor, an address, one LDS read and two
// accumulate operations. DMAS adds the fraction, a square root and the
// signed-root accumulation per gather; pDAS takes the p-th root through the
// hardware base-2 logarithm and exponential (the square root at p = 2).

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "frame_max.h"
#include "plan.h"

namespace pwbf {
namespace dev {

// RF storage types: element size and a load through a raw buffer resource
// (32-bit byte offset, scalar base), widened to float.
template <int DT>
struct RfT;
template <>
struct RfT<kI16> {
  static constexpr int kBytes = 2;
  static __device__ __forceinline__ float load(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return (float)(short)__builtin_amdgcn_raw_buffer_load_b16(r, (int)off, 0, 0);
  }
};
template <>
struct RfT<kF16> {
  static constexpr int kBytes = 2;
  static __device__ __forceinline__ float load(__amdgpu_buffer_rsrc_t r, unsigned off) {
    const unsigned short h = (unsigned short)__builtin_amdgcn_raw_buffer_load_b16(r, (int)off, 0, 0);
    return __half2float(__ushort_as_half(h));
  }
};
template <>
struct RfT<kF32> {
  static constexpr int kBytes = 4;
  static __device__ __forceinline__ float load(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __int_as_float((int)__builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
  }
};

// Buffer resource word 3 for raw (unformatted, unswizzled) loads on gfx9.
constexpr int kRawBufferWord3 = 0x00020000;

// Stage the windows of a chunk: rows r = c A + a (channel e0 + c, angle a) of
// win entries each (win a multiple of 4), described by the row table s_row:
// {offset of the record of (angle, channel) in elements, first sample n0 of the
// window}. Entry j of a row covers samples n = n0 + j and n + 1, i.e. kernel
// delays s in [m, m + 1) with m = j - off, and holds, with du = u[n+1] - u[n],
//   DAS:  the line through both samples in s:  (u[n] - m du, du),
//         so the interpolated value is b + s du (no fraction needed);
//   DMAS: (u[n], du), interpolated as u[n] + frac(s) du, which keeps the
//         rounding of v small where the signed square root is steep.
// Samples outside [0, n_samples) read as zero (the table gives rows that must
// be all zero a first sample far below 0).
//
// Each thread fills 4 consecutive entries of a row from 5 consecutive samples,
// read through one 32-bit buffer offset with immediate increments; where the 5
// samples straddle an end of the record the reads are clamped into it and the
// outside samples replaced by zero. Every read stays inside the RF buffer.
//
// Threads keep a fixed column of quads: with W4 = win / 4 quads per row and
// R = blockDim / W4 >= 1, thread t stages quad t mod W4 of rows t / W4, + R,
// + 2R, ..., so its entry offsets are set up once (the fewer than W4 threads
// past R W4 stay idle). A window holds at most kMaxWindow = 64 entries (the
// host refuses longer ones), so W4 <= 16 is never more than a wavefront.
struct QuadWalk {
  int row0, drow, j0;
  bool active;
};
__device__ __forceinline__ QuadWalk quad_walk(int W4) {
  const int bs = blockDim.x, t = threadIdx.x;
  QuadWalk w;
  // t / W4 through a float reciprocal: (t + 0.5) / W4 lies at least 0.5 / W4
  // from an integer and t < 2^10, so truncation yields the exact quotient
  const float rw = __builtin_amdgcn_rcpf((float)W4);
  w.row0 = (int)fmaf((float)t, rw, 0.5f * rw);
  w.j0 = (t - w.row0 * W4) << 2;
  w.drow = bs / W4;
  w.active = w.row0 < w.drow;
  return w;
}

template <int DT, int MODE>
__device__ __forceinline__ void stage_windows(const FramePlan &P, int rows, int off,
                                              const int2 *s_row, float2 *s_pairs) {
  using R = RfT<DT>;
  constexpr int B = R::kBytes;
  const int Ns = P.n_samples, win = P.win;
  const unsigned lim = (unsigned)max(Ns - 4, 0);  // n in [0, lim): all 5 samples inside
  // the plan's angles only: A * N * Ns * B < 2^31 bytes (checked on the host)
  const __amdgpu_buffer_rsrc_t res = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<void *>(P.rf), (short)0, P.n_angles * P.n_channels * Ns * B, kRawBufferWord3);
  const QuadWalk w = quad_walk(win >> 2);
  if (!w.active) return;
  {
    const int j0 = w.j0;
    const float m0 = (float)(off - j0);  // delay coordinate of entry j0
    for (int row = w.row0; row < rows; row += w.drow) {
      const int2 rb = s_row[row];
      const int n = rb.y + j0;
      float u[5];
      if ((unsigned)n < lim) {
        const unsigned vo = (unsigned)(rb.x + n) * B;
#pragma unroll
        for (int k = 0; k < 5; ++k) u[k] = R::load(res, vo + k * B);
      } else {
#pragma unroll
        for (int k = 0; k < 5; ++k) {
          const int i = n + k;
          const float v = R::load(res, (unsigned)(rb.x + min(max(i, 0), Ns - 1)) * B);
          u[k] = (unsigned)i < (unsigned)Ns ? v : 0.f;
        }
      }
      float v8[8];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float du = u[k + 1] - u[k];
        v8[2 * k] = MODE == kDas ? fmaf(m0 - (float)k, du, u[k]) : u[k];
        v8[2 * k + 1] = du;
      }
      float4 *dst = (float4 *)(s_pairs + __mul24(row, win) + j0);
      dst[0] = make_float4(v8[0], v8[1], v8[2], v8[3]);
      dst[1] = make_float4(v8[4], v8[5], v8[6], v8[7]);
    }
  }
}

// Stage the complex windows of the IQ modes: as stage_windows for DAS, with
// each entry the lines of the real and imaginary parts, (b_re, d_re, b_im, d_im)
// (16 bytes), from complex float32 samples.
__device__ __forceinline__ void stage_windows_iq(const FramePlan &P, int rows, int off,
                                                 const int2 *s_row, float4 *s_ent) {
  const int Ns = P.n_samples, win = P.win;
  const unsigned lim = (unsigned)max(Ns - 4, 0);
  const __amdgpu_buffer_rsrc_t res = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<void *>(P.rf), (short)0, P.n_angles * P.n_channels * Ns * 8, kRawBufferWord3);
  const QuadWalk w = quad_walk(win >> 2);
  if (!w.active) return;
  {
    const int j0 = w.j0;
    const float m0 = (float)(off - j0);
    for (int row = w.row0; row < rows; row += w.drow) {
      const int2 rb = s_row[row];
      const int n = rb.y + j0;
      float ur[5], ui[5];
      if ((unsigned)n < lim) {
        const unsigned vo = (unsigned)(rb.x + n) * 8u;
#pragma unroll
        for (int k = 0; k < 5; ++k) {
          ur[k] = __int_as_float((int)__builtin_amdgcn_raw_buffer_load_b32(res, (int)(vo + 8 * k), 0, 0));
          ui[k] = __int_as_float(
              (int)__builtin_amdgcn_raw_buffer_load_b32(res, (int)(vo + 8 * k + 4), 0, 0));
        }
      } else {
#pragma unroll
        for (int k = 0; k < 5; ++k) {
          const int i = n + k;
          const unsigned vo = (unsigned)(rb.x + min(max(i, 0), Ns - 1)) * 8u;
          const float re =
              __int_as_float((int)__builtin_amdgcn_raw_buffer_load_b32(res, (int)vo, 0, 0));
          const float im =
              __int_as_float((int)__builtin_amdgcn_raw_buffer_load_b32(res, (int)(vo + 4u), 0, 0));
          const bool in = (unsigned)i < (unsigned)Ns;
          ur[k] = in ? re : 0.f;
          ui[k] = in ? im : 0.f;
        }
      }
      float4 *dst = s_ent + __mul24(row, win) + j0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float m = m0 - (float)k;
        const float dr = ur[k + 1] - ur[k], di = ui[k + 1] - ui[k];
        dst[k] = make_float4(fmaf(m, dr, ur[k]), dr, fmaf(m, di, ui[k]), di);
      }
    }
  }
}

// exp(2 pi i r K) for an integer K and r = rh + rl given as a float-float pair:
// the revolutions K r are reduced modulo 1 exactly enough (~1e-7) for any K the
// windows use.
__device__ __forceinline__ float2 carrier_phasor(int K, float rh, float rl) {
  const float fk = (float)K;
  const float p = fk * rh;
  const float rho = (p - floorf(p)) + fmaf(fk, rl, fmaf(fk, rh, -p));
  float sn, cs;
  sincospif(2.0f * rho, &sn, &cs);
  return make_float2(cs, sn);
}

// floor(s) as an int in one instruction (v_cvt_flr_i32_f32; pure ALU)
__device__ __forceinline__ int floor_i32(float s) {
  int n;
  asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(n) : "v"(s));
  return n;
}

// Apodization weight for h = |x - x_e| / (2 half-apertures), i.e. half the
// normalised aperture distance r: hk cos(pi r) + hb inside the aperture (Hann:
// hk = hb = 1/2; boxcar: hk = 0, hb = 1), 0 outside. h is NaN or inf when
// z <= 0, which falls outside. "none" passes h = 0, so w = 1. The hardware
// cosine takes its argument in revolutions (cos(pi r) = cos(2 pi h)); clamping
// keeps it in range and makes the evaluation unconditional. The pixel's scale
// carries the factor 1/2 (exact), so h < 1/2 holds exactly where r < 1 does.
template <bool SEL>
__device__ __forceinline__ float apod_weight(float h, float hk, float hb) {
  const float c = __builtin_amdgcn_cosf(fminf(h, 0.5f));
  // Hann and "none" need no aperture test: at h >= 1/2 the clamped cosine is
  // that of half a revolution, which the hardware returns as exactly -1, so the
  // Hann weight 1/2 + c/2 is exactly 0 (and "none" has h = 0). Boxcar does.
  if constexpr (SEL) return h < 0.5f ? fmaf(hk, c, hb) : 0.f;
  return fmaf(hk, c, hb);
}

// Window origin LR = floor(min over the tile of rx) - 1 for an element at
// lateral offset dq = Xq - Xe from the tile's reference column: the tile point
// nearest the element, over lateral offsets [dq + dxlo, dq + dxhi] and depths
// [zlo, zhi]. The margin of one sample absorbs the float rounding, including
// the hardware square root's (under 1 ulp).
__device__ __forceinline__ float window_lr(float dq, float dxlo, float dxhi, float zlo,
                                           float zhi) {
  const float ddx = fmaxf(fmaxf(dq + dxlo, -(dq + dxhi)), 0.f);
  const float ddz = zlo > 0.f ? zlo : (zhi < 0.f ? -zhi : 0.f);
  return floorf(__builtin_amdgcn_sqrtf(fmaf(ddx, ddx, ddz * ddz))) - 1.f;
}

// Float-float arithmetic (value = hi + lo) from error-free transformations; used
// only for per-tile reference delays, so that no absolute delay (hundreds to
// thousands of samples) is ever rounded to float32 on the per-gather path.
// Floating-point contraction is off inside these helpers: fusing the product
// of ff_mul into the following sum (allowed by the device default
// -ffp-contract=fast) would silently drop the error terms.
struct ff {
  float hi, lo;
};
__device__ __forceinline__ ff two_sum(float a, float b) {
#pragma clang fp contract(off)
  const float s = a + b, bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}
__device__ __forceinline__ ff ff_add(ff a, ff b) {
#pragma clang fp contract(off)
  ff s = two_sum(a.hi, b.hi);
  return two_sum(s.hi, s.lo + a.lo + b.lo);
}
__device__ __forceinline__ ff ff_mul(ff a, ff b) {
#pragma clang fp contract(off)
  const float p = a.hi * b.hi;
  const float e = fmaf(a.hi, b.hi, -p) + (a.hi * b.lo + a.lo * b.hi);
  return two_sum(p, e);
}
__device__ __forceinline__ ff ff_neg(ff a) { return {-a.hi, -a.lo}; }
// sqrt(a) from the hardware square root s of a.hi (within an ulp) and one
// correction step: the residual a - s^2 is exact through the FMA, and its
// quotient by 2 s needs only float32 relative accuracy (it is ~2^-24 of s)
__device__ __forceinline__ ff ff_sqrt(ff a) {
#pragma clang fp contract(off)
  if (!(a.hi > 0.f)) return {0.f, 0.f};
  const float s = __builtin_amdgcn_sqrtf(a.hi);
  const float r = fmaf(-s, s, a.hi) + a.lo;
  return two_sum(s, r * (0.5f * __builtin_amdgcn_rcpf(s)));
}
__device__ __forceinline__ float ff_f(ff a) { return a.hi + a.lo; }

// a compile-time flag handed to the generic lambdas of the channel loop
template <bool B> struct Flag { static constexpr bool value = B; };

// AM: angles handled per pixel; PRED: AM is an upper bound and angles >= A are
// skipped (generic bucket), else exactly AM == A angles, fully unrolled.
// ONEGRP: one lane group per wavefront (cpw == 1), so the LDS window of a
// channel is the same for the whole wavefront and its address stays scalar.
// SEL: the apodization weight carries the aperture test (needed for boxcar).
//
// Delays of pixel p are formed relative to the tile's reference pixel q:
//   transmit  tx(p) - LT - off_t = [tx(q) - LT - off_t] + dx sin + dz cos,
//   receive   rx(p) - LR - off_r = [rx(q) - LR - off_r]
//                                  + (2 Dq dx + 2 Zq dz + dx^2 + dz^2) / (rx(p) + rx(q)),
// with (dx, dz) = p - q, Dq = Xq - Xe, and the bracketed tile constants taken
// from float-float reference delays; the integer offsets off_t, off_r centre
// both terms on zero and are added back in the LDS address. Every float32
// quantity on the per-gather path is then a small offset inside the tile's
// window, accurate to ~1e-6 samples, instead of an absolute delay rounded at
// ~1e-4 samples.
//
// DMAS and pDAS take a root of every delayed sample, which is steep where the
// sample crosses zero, so they take q as the wavefront's own centre pixel
// instead: the bracketed terms are then split, in float-float, into an integer
// (kT per angle, kR per channel, wave-uniform, folded into the LDS address)
// and a float32 fraction of at most half a sample, and the float32 offsets
// span only the wavefront's pixels (a few samples), which keeps the delay
// rounding near 5e-7 of a sample. Their window entries are (u[n], du), read at
// the fraction of the delay, so the per-wavefront integer shift needs no
// change to the windows.
// hull_lo >= 0: the tile's channel hull [hull_lo, hull_hi) comes from the
// caller (the batch computes it on the host); else the block finds it.
template <int AM, bool PRED, int MODE, bool ONEGRP, bool SEL>
__device__ __forceinline__ void process_tile_body(const FramePlan &P, int tz, int tx,
                                                  unsigned char *smem, int hull_lo = -1,
                                                  int hull_hi = -1) {
  constexpr bool IQ = is_iq_mode(MODE);
  float *s_txq = (float *)smem;                        // [kMaxAngles] tx(q) - LT
  int *s_lt = (int *)(smem + kMaxAngles * 4);          // [kMaxAngles] LT
  float2 *s_tph = (float2 *)(smem + kMaxAngles * 8);   // [kMaxAngles] IQ: exp(2 pi i r (LT + off_t))
  float4 *s_ch = (float4 *)(smem + kLdsAngleBytes);    // [chunk] {Dq, rq^2, rq, rx(q) - LR}
  float2 *s_ph = (float2 *)(smem + plan_lds_ph_offset(P));  // [chunk] IQ: exp(2 pi i r (LR + off_r))
  int2 *s_row = (int2 *)(smem + plan_lds_row_offset(P));  // [chunk * A] window rows
  float2 *s_pairs = (float2 *)(smem + plan_lds_win_offset(P));
  // DMAS, pDAS: per (wavefront, channel) {Dw, kR (int bits), rw, rx(w) - LR - off_r - kR}
  constexpr bool WREF = wave_ref_mode(MODE);
  float4 *s_chw = (float4 *)(smem + plan_lds_wref_offset(P));

  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);  // uniform
  const int cpw = ONEGRP ? 1 : P.cpw;
  const int ppw = kWave / cpw;  // lanes per group
  const int pl = lane & (ppw - 1), grp = ONEGRP ? 0 : lane / ppw;
  const int lz = P.lz, lx = P.lx;  // a group's pixels: lz along depth by lx along x
  // wave / wz for wave < 8 and wz <= 8 through a float reciprocal ((wave + 0.5) /
  // wz lies at least 1 / 16 from an integer); lz is a power of two
  const int wxi = (int)((wave + 0.5f) * __builtin_amdgcn_rcpf((float)P.wz));
  const int wzi = wave - wxi * P.wz;
  const int lzs = __builtin_ctz(lz);
  const int TZ = P.tile_z, TX = P.tile_x;
  const int iz0 = tz * TZ, ix0 = tx * TX;
  const int iz = iz0 + wzi * lz + (pl & (lz - 1)), ix = ix0 + wxi * lx + (pl >> lzs);
  const int A = PRED ? P.n_angles : AM;
  const int N = P.n_channels, win = P.win, chunk = P.chunk;
  // hk in a scalar register, hb in a vector one: the weight's FMA may read only
  // one scalar operand, and an opaque hb is not re-derived in every iteration
  const float hk = __int_as_float(
      __builtin_amdgcn_readfirstlane(__float_as_int(P.apod == kHann ? 0.5f : 0.f)));
  float hb = P.apod == kHann ? 0.5f : 1.f;
  asm("" : "+v"(hb));

  // Tile extent, clipped to the grid: lanes past the edge evaluate the edge
  // pixel again and write nothing, so every window only spans grid pixels.
  const int ixe = min(ix0 + TX - 1, P.nx - 1), ize = min(iz0 + TZ - 1, P.nz - 1);
  const int ixq = (ix0 + ixe) >> 1, izq = (iz0 + ize) >> 1;  // reference pixel q of the tile
  // the tile's offset range from q (window origins)
  const float dxlo = (float)(ix0 - ixq) * P.DX, dxhi = (float)(ixe - ixq) * P.DX;
  const float dzlo = (float)(iz0 - izq) * P.DZ, dzhi = (float)(ize - izq) * P.DZ;
  // tile reference position in float-float
  const ff Xq = ff_add(ff_mul({(float)ixq, 0.f}, {P.DX, P.DXl}), {P.X0, P.X0l});
  const ff Zq = ff_add(ff_mul({(float)izq, 0.f}, {P.DZ, P.DZl}), {P.Z0, P.Z0l});
  const float Zqf = ff_f(Zq);
  // reference of the per-gather offsets: q, or the centre of the wavefront's
  // pixels (clipped to the tile's grid pixels) for DMAS and pDAS
  int ixr = ixq, izr = izq;
  if constexpr (WREF) {
    const int bx0 = min(ix0 + wxi * lx, ixe), bz0 = min(iz0 + wzi * lz, ize);
    ixr = (bx0 + min(bx0 + lx - 1, ixe)) >> 1;
    izr = (bz0 + min(bz0 + lz - 1, ize)) >> 1;
  }
  const ff Xr = WREF ? ff_add(ff_mul({(float)ixr, 0.f}, {P.DX, P.DXl}), {P.X0, P.X0l}) : Xq;
  const ff Zr = WREF ? ff_add(ff_mul({(float)izr, 0.f}, {P.DZ, P.DZl}), {P.Z0, P.Z0l}) : Zq;
  const float Zrf = ff_f(Zr);
  // the pixel's offsets from the reference
  const float dx = (float)(min(ix, ixe) - ixr) * P.DX;
  const float dz = (float)(min(iz, ize) - izr) * P.DZ;
  const float Zp = Zrf + dz;
  // half the aperture scale: |x - x_e| * hA is half the normalised distance r
  const float hA = P.apod == kNone ? 0.f : (Zp > 0.f ? 0.5f * (P.ap_k / Zp) : __builtin_inff());
  const float cp = fmaf(2.f * Zrf, dz, fmaf(dx, dx, dz * dz));
  float dx2 = 2.f * dx;
  asm("" : "+v"(dx2));  // computed once, not again in every channel iteration

  // Active aperture of the tile. A channel whose apodization weight is zero at
  // every pixel of the tile adds exactly nothing to any sum (w * acc with w = 0
  // and finite acc), so the channel loop runs over the hull [e_lo, e_hi) of the
  // channels that may reach the tile: distance from x_e to the tile's lateral
  // span below Z_max / (2 F#). The test carries a 1e-3 relative margin, so
  // float rounding can only add a channel, never drop one; outputs are those
  // of the loop over all channels.
  __shared__ int s_erange[2 * kMaxWavesPerBlock];
  const bool given_hull = hull_lo >= 0;
  if (P.apod != kNone && !given_hull) {
    const float zmax = Zqf + dzhi;
    int lo = N, hi = 0;
    for (int e = tid; e < N; e += blockDim.x) {
      const float dq = ff_f(ff_add(Xq, ff_neg({P.xe[e], P.xel[e]})));
      const float ddx = fmaxf(fmaxf(dq + dxlo, -(dq + dxhi)), 0.f);
      if (zmax > 0.f && ddx * P.ap_k < zmax * 1.001f) {
        lo = min(lo, e);
        hi = max(hi, e + 1);
      }
    }
    // only wavefronts whose threads hold a channel (wave * 64 < N) reduce
    if (wave * kWave < N) {
      for (int off = 1; off < kWave; off <<= 1) {
        lo = min(lo, __shfl_xor(lo, off));
        hi = max(hi, __shfl_xor(hi, off));
      }
      if (lane == 0) {
        s_erange[2 * wave] = lo;
        s_erange[2 * wave + 1] = hi;
      }
    }
  }

  // Per-angle tile constants: window origin LT = floor(min_tile tx) - 1 and
  // tx(q) - LT. tx is linear, so its tile minimum is at a corner. Angle a is
  // taken by thread blockDim - 1 - a: another wavefront than the aperture hull
  // above, which starts at thread 0, so the two run side by side.
  for (int a = (int)blockDim.x - 1 - tid; a < A; a += blockDim.x) {
    const ff sa = {P.sa[a], P.sal[a]}, ca = {P.ca[a], P.cal[a]}, to = {P.to[a], P.tol[a]};
    const ff txq = ff_add(ff_add(ff_mul(Xq, sa), ff_mul(Zq, ca)), ff_neg(to));
    const float dmin = fminf(dxlo * sa.hi, dxhi * sa.hi) + fminf(dzlo * ca.hi, dzhi * ca.hi);
    const float fl = floorf(txq.hi);
    const float lt = fl + floorf((txq.hi - fl) + txq.lo + dmin) - 1.f;
    s_txq[a] = ff_f(ff_add(txq, {-(lt + (float)P.off_t), 0.f}));
    s_lt[a] = (int)lt;
    if constexpr (IQ) s_tph[a] = carrier_phasor((int)lt + P.off_t, P.iq_r, P.iq_rl);
  }
  __syncthreads();
  int e_lo = 0, e_hi = N;
  if (given_hull) {
    e_lo = __builtin_amdgcn_readfirstlane(hull_lo);
    e_hi = __builtin_amdgcn_readfirstlane(hull_hi);
  } else if (P.apod != kNone) {
    e_hi = 0;
    e_lo = N;
    const int nwr = min((int)(blockDim.x / kWave), (N + kWave - 1) / kWave);
    for (int w = 0; w < nwr; ++w) {
      e_lo = min(e_lo, s_erange[2 * w]);
      e_hi = max(e_hi, s_erange[2 * w + 1]);
    }
    e_lo = __builtin_amdgcn_readfirstlane(e_lo);
    e_hi = __builtin_amdgcn_readfirstlane(e_hi);
  }
  float txl[AM];
  int kt8[WREF ? AM : 1];  // DMAS, pDAS: window byte offset of angle a's integer shift kT
  if constexpr (WREF) {
    // lane a of every wavefront: its reference's transmit delay in the window
    // of angle a, split into kT (integer) and a fraction of at most 1/2
    float ftl = 0.f;
    int ktl = 0;
    if (lane < A) {
      const ff sa = {P.sa[lane], P.sal[lane]}, ca = {P.ca[lane], P.cal[lane]};
      const ff to = {P.to[lane], P.tol[lane]};
      const ff t = ff_add(ff_add(ff_add(ff_mul(Xr, sa), ff_mul(Zr, ca)), ff_neg(to)),
                          {-(float)(s_lt[lane] + P.off_t), 0.f});
      const float k = rintf(t.hi);
      ftl = (t.hi - k) + t.lo;  // t.hi - k is exact (|t.hi - k| <= 1/2 and k integral)
      ktl = (int)k;
    }
#pragma unroll
    for (int a = 0; a < AM; ++a)
      if (!PRED || a < A) {
        txl[a] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ftl), a)) +
                 fmaf(dx, P.sa[a], dz * P.ca[a]);
        kt8[a] = __builtin_amdgcn_readlane(ktl, a) * 8 + a * win * 8;
      }
  } else {
#pragma unroll
    for (int a = 0; a < AM; ++a)
      if (!PRED || a < A) txl[a] = s_txq[a] + fmaf(dx, P.sa[a], dz * P.ca[a]);
  }

  float total = 0.f;
  float S[MODE == kDas ? 1 : AM];  // per-angle sums: compressed samples (DMAS, pDAS), Re (IQ)
  float SI[IQ ? AM : 1];           // per-angle sums, Im (IQ)
  float Q = 0.f;
#pragma unroll
  for (int a = 0; a < (MODE == kDas ? 1 : AM); ++a) S[a] = 0.f;
#pragma unroll
  for (int a = 0; a < (IQ ? AM : 1); ++a) SI[a] = 0.f;

  for (int e0 = e_lo; e0 < e_hi; e0 += chunk) {
    if (e0 > e_lo) __syncthreads();  // the previous chunk's windows have been read
    const int cnt = min(chunk, e_hi - e0);                   // channels of this chunk
    const int cnt_pad = ONEGRP ? cnt : (cnt + cpw - 1) / cpw * cpw;  // rows read
    // Per-channel tile constants: the window origin LR, the reference delay
    // rx(q) in float-float, and the terms of the receive-delay difference;
    // channel c is taken by thread blockDim - 1 - c, so that these run in other
    // wavefronts than the row table below, which starts at thread 0.
    for (int c = (int)blockDim.x - 1 - tid; !WREF && c < cnt_pad; c += blockDim.x) {
      const int e = min(e0 + c, N - 1);
      const ff xe = {P.xe[e], P.xel[e]};
      const ff dq = ff_add(Xq, ff_neg(xe));
      const ff rq2 = ff_add(ff_mul(dq, dq), ff_mul(Zq, Zq));
      const ff rq = ff_sqrt(rq2);
      const float dqf = ff_f(dq);
      const float lr = window_lr(dqf, dxlo, dxhi, Zqf + dzlo, Zqf + dzhi);
      s_ch[c] = make_float4(dqf, ff_f(rq2), ff_f(rq) + 1e-20f,
                            ff_f(ff_add(rq, {-(lr + (float)P.off_r), 0.f})));
      if constexpr (IQ) s_ph[c] = carrier_phasor((int)lr + P.off_r, P.iq_r, P.iq_rl);
    }
    // Window rows r = c A + a: the record of (angle a, channel e0 + c) and the
    // first sample LT_a + LR (LR from the same expression as above); rows of
    // padding channels (past e_hi) read all zero. The record offset is a full
    // 32-bit product (n_samples may exceed the 24-bit multiplier's range; the
    // host bounds the product below 2^31).
    const int rows = cnt_pad * A, off = P.off_t + P.off_r;
    for (int r = tid; r < rows; r += blockDim.x) {
      const int c = r / A, a = r - c * A;
      const int e = min(e0 + c, N - 1);
      const float dqf = ff_f(ff_add(Xq, ff_neg({P.xe[e], P.xel[e]})));
      const float lr = window_lr(dqf, dxlo, dxhi, Zqf + dzlo, Zqf + dzhi);
      s_row[r] = make_int2((__mul24(a, N) + e) * P.n_samples,
                           e0 + c < e_hi ? s_lt[a] + (int)lr : -(1 << 30));
    }
    if constexpr (WREF) {
      // every wavefront, for its own reference pixel and each channel of the
      // chunk: Dw = Xw - Xe, rw^2, rw, and rw - LR - off_r split into the
      // integer kR and a fraction of at most 1/2 (LR from the same expression
      // as the window rows)
      for (int c = lane; c < cnt_pad; c += kWave) {
        const int e = min(e0 + c, N - 1);
        const ff xe = {P.xe[e], P.xel[e]};
        const float dqf = ff_f(ff_add(Xq, ff_neg(xe)));
        const float lr = window_lr(dqf, dxlo, dxhi, Zqf + dzlo, Zqf + dzhi);
        const ff dw = ff_add(Xr, ff_neg(xe));
        const ff rw2 = ff_add(ff_mul(dw, dw), ff_mul(Zr, Zr));
        const ff rw = ff_sqrt(rw2);
        const ff rrel = ff_add(rw, {-(lr + (float)P.off_r), 0.f});
        const float k = rintf(rrel.hi);
        const int slot = wave * chunk + c;
        s_chw[slot] = make_float4(ff_f(dw), __int_as_float((int)k), ff_f(rw) + 1e-20f,
                                  (rrel.hi - k) + rrel.lo);
      }
    }
    __syncthreads();
    if constexpr (IQ)
      stage_windows_iq(P, rows, off, s_row, (float4 *)s_pairs);
    else if (P.dtype == kI16)
      stage_windows<kI16, MODE>(P, rows, off, s_row, s_pairs);
    else if (P.dtype == kF16)
      stage_windows<kF16, MODE>(P, rows, off, s_row, s_pairs);
    else
      stage_windows<kF32, MODE>(P, rows, off, s_row, s_pairs);
    __syncthreads();

    const int wstride = win * P.entry_bytes;  // bytes between angle windows
    // SQ: pDAS with p = 2 (square root in place of exp2/log2). The test is
    // uniform over the kernel; taking it once per chunk rather than per
    // channel keeps the angle sums in the same registers through the channel
    // loop (a per-channel branch made the compiler copy all of them at its
    // join, two moves per angle and channel)
    auto channel = [&](int k, auto sq) __attribute__((always_inline)) {
      const int c = ONEGRP ? k : k + grp;
      const int slot = wave * chunk + c;
      const float4 ch = WREF ? s_chw[slot] : s_ch[c];
      // DMAS, pDAS: the wavefront's integer shift of this channel's window
      int kr = 0;
      if constexpr (WREF)
        kr = ONEGRP ? __builtin_amdgcn_readfirstlane(__float_as_int(ch.y)) : __float_as_int(ch.y);
      // receive delay relative to the window origin, as a difference from rx(q)
      const float num = fmaf(dx2, ch.x, cp);
      // rx(p) + rx(ref): rx(ref)^2 + num in one rounding (the sum only needs
      // float32 relative accuracy); DMAS and pDAS keep kR where DAS keeps rx(q)^2
      const float den = __builtin_amdgcn_sqrtf(WREF ? fmaf(ch.z, ch.z, num) : ch.y + num) + ch.z;
      const float rxl = fmaf(num, __builtin_amdgcn_rcpf(den), ch.w);
      const float w = apod_weight<SEL>(fabsf(ch.x + dx) * hA, hk, hb);
      // delays are centred: entry n of the window is read as n + off_t + off_r
      const char *wb = (const char *)s_pairs +
                       ((size_t)c * A * win + P.off_t + P.off_r + kr) * (IQ ? 16 : 8);
      // the window of angle a: wb + a * wstride, with the wavefront's transmit
      // shift kT for DMAS and pDAS (kt8 holds both, in bytes)
      if constexpr (MODE == kDas) {
        float acc = -0.f;  // x + (-0) == x for every x: the first add folds away
#pragma unroll
        for (int a = 0; a < AM; ++a) {
          if (!PRED || a < A) {
            const float s = txl[a] + rxl;
            const int n = floor_i32(s);
            const float2 p = *(const float2 *)(wb + a * wstride + (n << 3));
            acc += p.x;  // the entry's line at s: b + s du
            acc = fmaf(s, p.y, acc);
          }
        }
        total = fmaf(w, acc, total);
      } else if constexpr (IQ) {
        // receive phasor of this (pixel, channel), weight folded in:
        // w exp(2 pi i r (LR + off_r + rx(p) - LR - off_r))
        const float2 pk = s_ph[c];
        const float rho = P.iq_r * rxl;
        const float cr = __builtin_amdgcn_cosf(rho), sr = __builtin_amdgcn_sinf(rho);
        const float Rx = w * (pk.x * cr - pk.y * sr), Ry = w * (pk.x * sr + pk.y * cr);
#pragma unroll
        for (int a = 0; a < AM; ++a) {
          if (!PRED || a < A) {
            const float s = txl[a] + rxl;
            const int n = floor_i32(s);
            const float4 q = *(const float4 *)(wb + a * wstride + (n << 4));
            const float I = fmaf(s, q.y, q.x), Qv = fmaf(s, q.w, q.z);  // the lines at s
            float cx = Rx, cy = Ry;
            if constexpr (MODE == kBbdmas) {
              // sqrt(amplitude), phase kept: scale by |q|^(-1/2). |q|^2 carries
              // the smallest normal float, 2^-126, so that q = 0 gives a finite
              // scale (at most 2^31.5) times a zero sample, with no test and
              // select; above |q| = 2^-50 the added term lies below the float32
              // rounding of |q|^2
              const float m2 = fmaf(I, I, fmaf(Qv, Qv, 0x1p-126f));
              const float k = __builtin_amdgcn_rsqf(__builtin_amdgcn_sqrtf(m2));
              cx *= k;
              cy *= k;
            }
            S[a] = fmaf(cx, I, fmaf(-cy, Qv, S[a]));
            SI[a] = fmaf(cx, Qv, fmaf(cy, I, SI[a]));
          }
        }
      } else if constexpr (MODE == kPdas) {
        // sign(v) |v|^(1/p) = sign(v) 2^(log2|v| / p); |v| = 0 gives 2^-inf = 0.
        // p = 2 takes the square root instead: one transcendental operation per
        // gather instead of two
        const float ip = P.pdas_inv_p;
        if constexpr (decltype(sq)::value) {
#pragma unroll
          for (int a = 0; a < AM; ++a) {
            if (!PRED || a < A) {
              const float s = txl[a] + rxl;
              const int n = floor_i32(s);
              const float f = __builtin_amdgcn_fractf(s);
              const float2 p = *(const float2 *)(wb + kt8[WREF ? a : 0] + (n << 3));
              const float v = fmaf(f, p.y, p.x);
              S[a] = fmaf(w, copysignf(__builtin_amdgcn_sqrtf(fabsf(v)), v), S[a]);
            }
          }
        } else {
#pragma unroll
          for (int a = 0; a < AM; ++a) {
            if (!PRED || a < A) {
              const float s = txl[a] + rxl;
              const int n = floor_i32(s);
              const float f = __builtin_amdgcn_fractf(s);
              const float2 p = *(const float2 *)(wb + kt8[WREF ? a : 0] + (n << 3));
              const float v = fmaf(f, p.y, p.x);
              const float r = __builtin_amdgcn_exp2f(ip * __builtin_amdgcn_logf(fabsf(v)));
              S[a] = fmaf(w, copysignf(r, v), S[a]);
            }
          }
        }
      } else {
        float q = 0.f;
#pragma unroll
        for (int a = 0; a < AM; ++a) {
          if (!PRED || a < A) {
            const float s = txl[a] + rxl;
            const int n = floor_i32(s);
            const float f = __builtin_amdgcn_fractf(s);
            const float2 p = *(const float2 *)(wb + kt8[WREF ? a : 0] + (n << 3));
            const float v = fmaf(f, p.y, p.x);
            const float r = __builtin_amdgcn_sqrtf(fabsf(v));
            S[a] = fmaf(w, copysignf(r, v), S[a]);
            q += fabsf(v);
          }
        }
        Q = fmaf(w * w, q, Q);
      }
    };
    // One or two exact angles: two channels per iteration, so that the second
    // channel's table and window reads are in flight while the first computes
    // (one channel is a chain of two dependent LDS round trips, and a small
    // grid leaves few wavefronts per SIMD to hide them)
    auto channels = [&](auto sq) __attribute__((always_inline)) {
      if constexpr (AM <= 2 && !PRED) {
        int k = 0;
        for (; k + cpw < cnt; k += 2 * cpw) {
          channel(k, sq);
          channel(k + cpw, sq);
        }
        if (k < cnt) channel(k, sq);
      } else {
        for (int k = 0; k < cnt; k += cpw) channel(k, sq);
      }
    };
    if constexpr (MODE == kPdas) {
      if (P.pdas_p == 2.0f)
        channels(Flag<true>{});
      else
        channels(Flag<false>{});
    } else {
      channels(Flag<false>{});
    }
  }

  if constexpr (IQ) {
    // per angle: the transmit phasor exp(2 pi i r (LT + off_t + tx(p) - LT - off_t))
    // times the angle's sum; BB-DMAS squares it; the angles add
    float yr = 0.f, yi = 0.f;
#pragma unroll
    for (int a = 0; a < AM; ++a) {
      if (!PRED || a < A) {
        float tr = S[a], ti = SI[a];
        for (int off = ppw; off < kWave; off <<= 1) {
          tr += __shfl_xor(tr, off);
          ti += __shfl_xor(ti, off);
        }
        const float2 tp = s_tph[a];
        const float rho = P.iq_r * txl[a];
        const float ct = __builtin_amdgcn_cosf(rho), st = __builtin_amdgcn_sinf(rho);
        const float Tx = tp.x * ct - tp.y * st, Ty = tp.x * st + tp.y * ct;
        const float zr = Tx * tr - Ty * ti, zi = Tx * ti + Ty * tr;
        if constexpr (MODE == kBbdmas) {
          yr += zr * zr - zi * zi;
          yi += 2.f * zr * zi;
        } else {
          yr += zr;
          yi += zi;
        }
      }
    }
    const bool mine = grp == 0 && ix < P.nx && iz < P.nz;
    const float env = sqrtf(yr * yr + yi * yi);
    if (mine) {
      const size_t o = (size_t)ix * P.nz + iz;
      P.out[o] = yr;
      if (P.out_imag) P.out_imag[o] = yi;
      if (P.out_env) P.out_env[o] = env;
    }
    if (P.ws_max) {  // the frame maximum of |y| for the log image
      __shared__ float s_wmax[kMaxWavesPerBlock];
      float m = mine ? env : 0.f;
      for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
      if (lane == 0) s_wmax[wave] = m;
      __syncthreads();
      if (tid == 0) {
        for (int w = 1; w < (int)(blockDim.x / kWave); ++w) m = fmaxf(m, s_wmax[w]);
        frame_max_fold(P.ws_max, m);
      }
    }
    return;
  }

  float y;
  if constexpr (MODE == kDas) {
    for (int off = ppw; off < kWave; off <<= 1) total += __shfl_xor(total, off);
    y = total;
  } else if constexpr (MODE == kPdas) {
    // per angle the signed p-th power of the summed roots; the angles add
    y = 0.f;
#pragma unroll
    for (int a = 0; a < AM; ++a) {
      if (!PRED || a < A) {
        float t = S[a];
        for (int off = ppw; off < kWave; off <<= 1) t += __shfl_xor(t, off);
        y += P.pdas_p == 2.0f
                 ? t * fabsf(t)
                 : copysignf(__builtin_amdgcn_exp2f(P.pdas_p * __builtin_amdgcn_logf(fabsf(t))), t);
      }
    }
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

// The tile body for plan P. The exact-angle RF kernels of one lane group
// carry a second body without the aperture test in the weight (Hann, none),
// two fewer instructions per (pixel, channel); every other kernel and boxcar
// apodization take the general one. (The serve kernels call the general body
// directly: there the second body costs registers.)
template <int AM, bool PRED, int MODE, bool ONEGRP>
__device__ __forceinline__ void process_tile(const FramePlan &P, int tz, int tx,
                                             unsigned char *smem, int hull_lo = -1,
                                             int hull_hi = -1) {
  if constexpr ((MODE == kDas || MODE == kDmas || MODE == kPdas) && ONEGRP && !PRED) {
    if (P.apod != kBoxcar) {
      process_tile_body<AM, PRED, MODE, ONEGRP, false>(P, tz, tx, smem, hull_lo, hull_hi);
      return;
    }
  }
  process_tile_body<AM, PRED, MODE, ONEGRP, true>(P, tz, tx, smem, hull_lo, hull_hi);
}

}  // namespace dev
}  // namespace pwbf
