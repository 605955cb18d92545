#pragma once
// Block FFT in LDS for gfx950: Stockham autosort passes of radix 16 (the last
// pass takes the remaining 2, 4 or 8), so a 4096-point transform is three
// passes with the butterflies' values held in registers, natural order in and
// out, instead of twelve radix-2 stages.
//
// A pass of radix R over n = 2^L points with stride NS (the product of the
// earlier radices): butterfly j (0 <= j < n / R) reads x[j + r n / R],
// r < R, multiplies element r by W_{NS R}^{k r} with k = j mod NS, takes an
// R-point DFT in registers and writes element r to x[(j - k) R + k + r NS].
// Every butterfly of the pass reads before a barrier and writes after it, so
// the pass works in place. Several rows (transforms of the same length) can
// share a block: row q occupies x[q * padded(n) ...].
//
// LDS positions are padded by one element every 16 (pad(i) = i + i / 16): the
// first pass writes with a stride of 16 elements, which would otherwise put all
// lanes of a wave on the same bank. Twiddles come from one table of
// W_4096^i = exp(-2 pi i i / 4096), i < 2048 (W^{i + 2048} = -W^i), built at
// compile time and read through the vector cache: a butterfly reads w, w^2,
// w^4 and w^8 and forms the other powers with at most two products. The
// inverse transform (no 1/n) swaps real and imaginary parts around the
// forward DFT, which conjugates the twiddles.
#include <hip/hip_runtime.h>

#include "fft_twiddles.h"

namespace pwbf {
namespace fft {

constexpr int kThreads = 256;

__host__ __device__ constexpr int pad(int i) { return i + (i >> 4); }
__host__ __device__ constexpr int padded(int n) { return n + (n >> 4); }

// Distance between the rows of a multi-row block: one element more than the
// padded row, so that the same position of consecutive rows falls on different
// banks (transposing loads and stores walk down the rows)
__host__ __device__ constexpr int row_stride(int n, int rows) {
  return rows > 1 ? padded(n) + 1 : padded(n);
}

// LDS bytes of `rows` rows of n points
__host__ __device__ constexpr size_t lds_bytes(int n, int rows) {
  return (size_t)row_stride(n, rows) * rows * 8;
}

__device__ const detail::TwTable kTwTable = detail::TwTable();

// W_4096^i for 0 <= i < 4096
__device__ __forceinline__ float2 w4096(int i) {
  const detail::Tw t = kTwTable.v[i & (detail::kTwN / 2 - 1)];
  return i < detail::kTwN / 2 ? make_float2(t.c, t.s) : make_float2(-t.c, -t.s);
}

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// -i z and the swap of real and imaginary parts
__device__ __forceinline__ float2 mul_mi(float2 z) { return make_float2(z.y, -z.x); }
__device__ __forceinline__ float2 swap(float2 z) { return make_float2(z.y, z.x); }

// forward DFTs of 2, 4, 8 and 16 points in registers (radix-2 splits into even
// and odd halves; the twiddles of 8 and 16 points are cos and sin of multiples
// of pi / 8)
__device__ __forceinline__ void dft2(float2 &a, float2 &b) {
  const float2 t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

__device__ __forceinline__ void dft4(float2 &v0, float2 &v1, float2 &v2, float2 &v3) {
  const float2 t0 = cadd(v0, v2), t1 = csub(v0, v2), t2 = cadd(v1, v3), t3 = mul_mi(csub(v1, v3));
  v0 = cadd(t0, t2);
  v2 = csub(t0, t2);
  v1 = cadd(t1, t3);
  v3 = csub(t1, t3);
}

constexpr float kH = 0.70710678118654752f;   // cos(pi / 4)
constexpr float kC1 = 0.92387953251128674f;  // cos(pi / 8)
constexpr float kS1 = 0.38268343236508979f;  // sin(pi / 8)

template <int R>
__device__ __forceinline__ void dft(float2 (&v)[R]);

template <>
__device__ __forceinline__ void dft<2>(float2 (&v)[2]) {
  dft2(v[0], v[1]);
}

template <>
__device__ __forceinline__ void dft<4>(float2 (&v)[4]) {
  dft4(v[0], v[1], v[2], v[3]);
}

template <>
__device__ __forceinline__ void dft<8>(float2 (&v)[8]) {
  float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4(e0, e1, e2, e3);
  dft4(o0, o1, o2, o3);
  // W8^k, k = 1, 2, 3
  o1 = make_float2(kH * (o1.x + o1.y), kH * (o1.y - o1.x));
  o2 = mul_mi(o2);
  o3 = make_float2(kH * (o3.y - o3.x), -kH * (o3.x + o3.y));
  v[0] = cadd(e0, o0);
  v[4] = csub(e0, o0);
  v[1] = cadd(e1, o1);
  v[5] = csub(e1, o1);
  v[2] = cadd(e2, o2);
  v[6] = csub(e2, o2);
  v[3] = cadd(e3, o3);
  v[7] = csub(e3, o3);
}

template <>
__device__ __forceinline__ void dft<16>(float2 (&v)[16]) {
  float2 e[8], o[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    e[i] = v[2 * i];
    o[i] = v[2 * i + 1];
  }
  dft<8>(e);
  dft<8>(o);
  // W16^k = (cos(pi k / 8), -sin(pi k / 8)), k = 1..7
  const float2 w[8] = {make_float2(1.f, 0.f),  make_float2(kC1, -kS1), make_float2(kH, -kH),
                       make_float2(kS1, -kC1), make_float2(0.f, -1.f), make_float2(-kS1, -kC1),
                       make_float2(-kH, -kH),  make_float2(-kC1, -kS1)};
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const float2 t = k == 0 ? o[0] : (k == 4 ? mul_mi(o[4]) : cmul(o[k], w[k]));
    v[k] = cadd(e[k], t);
    v[k + 8] = csub(e[k], t);
  }
}

// w^r, r = 1 .. R - 1, for w = W_4096^b: w, w^2, w^4, w^8 from the table, the
// other powers as products of at most two of those
template <int R>
__device__ __forceinline__ void powers(int b, float2 (&t)[R]) {
  t[1] = w4096(b);
  if constexpr (R >= 4) {
    t[2] = w4096(2 * b);
    t[3] = cmul(t[2], t[1]);
  }
  if constexpr (R >= 8) {
    t[4] = w4096(4 * b);
    t[5] = cmul(t[4], t[1]);
    t[6] = cmul(t[4], t[2]);
    t[7] = cmul(t[4], t[3]);
  }
  if constexpr (R >= 16) {
    t[8] = w4096(8 * b);
#pragma unroll
    for (int r = 9; r < 16; ++r) t[r] = cmul(t[8], t[r - 8]);
  }
}

template <int R, int NS, int L, bool INV, int ROWS>
__device__ __forceinline__ void pass(float2 *x) {
  constexpr int n = 1 << L, nr = n / R, total = nr * ROWS;
  constexpr int K = (total + kThreads - 1) / kThreads;  // butterflies per thread
  static_assert(n <= detail::kTwN, "transforms up to 4096 points");
  // twiddle W_{NS R}^{k r} = W_4096^{k r tw4096}
  constexpr int stride = row_stride(n, ROWS), tw4096 = detail::kTwN / (NS * R);
  float2 v[K][R];
#pragma unroll
  for (int q = 0; q < K; ++q) {
    const int t = (int)threadIdx.x + q * kThreads;
    if (total % kThreads == 0 || t < total) {
      const int row = t / nr, j = t % nr, k = j & (NS - 1);
      const float2 *xr = x + row * stride;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const float2 a = xr[pad(j + r * nr)];
        v[q][r] = INV ? swap(a) : a;
      }
      if constexpr (NS > 1) {
        float2 t[R];
        powers<R>(k * tw4096, t);
#pragma unroll
        for (int r = 1; r < R; ++r)
          // inverse: swap(z conj(w)) = swap(z) w, so the swapped values take w itself
          v[q][r] = cmul(v[q][r], t[r]);
      }
      dft<R>(v[q]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < K; ++q) {
    const int t = (int)threadIdx.x + q * kThreads;
    if (total % kThreads == 0 || t < total) {
      const int row = t / nr, j = t % nr, k = j & (NS - 1);
      float2 *xr = x + row * stride;
      const int o = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) xr[pad(o + r * NS)] = INV ? swap(v[q][r]) : v[q][r];
    }
  }
  __syncthreads();
}

template <int L, int DONE, bool INV, int ROWS>
__device__ __forceinline__ void passes(float2 *x) {
  if constexpr (DONE < L) {
    constexpr int RB = (L - DONE) >= 4 ? 4 : (L - DONE);
    pass<1 << RB, 1 << DONE, L, INV, ROWS>(x);
    passes<L, DONE + RB, INV, ROWS>(x);
  }
}

// In-place transform of ROWS rows of 2^L points at x (padded layout, rows
// row_stride(2^L, ROWS) apart). Starts
// and ends with a barrier-consistent LDS state: callers write x and
// __syncthreads() before, read after.
template <int L, bool INV, int ROWS = 1>
__device__ __forceinline__ void transform(float2 *x) {
  passes<L, 0, INV, ROWS>(x);
}

// One row, L known only at run time (uniform over the block), 1 <= L <= 12.
template <bool INV>
__device__ __forceinline__ void transform_any(float2 *x, int L) {
  switch (L) {
    case 1: transform<1, INV>(x); break;
    case 2: transform<2, INV>(x); break;
    case 3: transform<3, INV>(x); break;
    case 4: transform<4, INV>(x); break;
    case 5: transform<5, INV>(x); break;
    case 6: transform<6, INV>(x); break;
    case 7: transform<7, INV>(x); break;
    case 8: transform<8, INV>(x); break;
    case 9: transform<9, INV>(x); break;
    case 10: transform<10, INV>(x); break;
    case 11: transform<11, INV>(x); break;
    default: transform<12, INV>(x); break;
  }
}

}  // namespace fft
}  // namespace pwbf
