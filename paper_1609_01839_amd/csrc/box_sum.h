// Building blocks of the streaming box sums of the guided filter and of its adjoint: a block
// of kGfThreads threads owns one column each, keeps compensated vertical running sums and
// forms horizontal window sums from them in LDS.
#pragma once
#include <hip/hip_runtime.h>

namespace gfd {

constexpr int kGfThreads = 256;
constexpr int kGfRmax = 8;
constexpr int kGfRun = 8;  // columns per thread in the horizontal sums (a multiple of 4)
constexpr int kGfRB = 2;   // rows per round of barriers

struct Kahan {
  float s, c;
};

// s += (xn - xo), compensated
__device__ __forceinline__ void kahan_slide(Kahan &k, float xn, float xo) {
  const float d = __fsub_rn(xn, xo);
  const float y = __fsub_rn(d, k.c);
  const float t = __fadd_rn(k.s, y);
  k.c = __fsub_rn(__fsub_rn(t, k.s), y);
  k.s = t;
}

// Pixels of the window of half-width R centred at c (a row or column index) inside [0, n).
template <int R>
__device__ __forceinline__ int clip_count(int c, int n) {
  return min(c + R, n - 1) - max(c - R, 0) + 1;
}

__device__ __forceinline__ int wrap(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

// Rows of vertical sums are kept in LDS with R zero columns on each side: column c of a
// row is at index c + R of a row of hs_pitch<R>() floats (a multiple of 4).  The padding
// columns are zeroed once and never written, so that runs at the strip's edges read finite
// values without clamped indices.
template <int R>
constexpr int hs_pitch() {
  return (kGfThreads + 2 * R + 3) & ~3;
}

// Horizontal window sums (half-width R) over rows of padded vertical sums: task `t` covers row
// t / runs and output columns [j0, j0 + kGfRun), j0 = run * kGfRun.  Its inputs, columns
// j0 - R .. j0 + kGfRun - 1 + R, start at the 16-byte aligned index j0 and are read as float4
// words; the outputs go out as float4 words into rows of kGfThreads floats.  Columns outside [R, used - R) produce don't-care
// values.
template <int R>
__device__ __forceinline__ void hsum_task(const float *__restrict__ src, float *__restrict__ dst, int task) {
  static_assert(kGfRun % 4 == 0, "outputs go out as float4");
  constexpr int runs = kGfThreads / kGfRun;
  constexpr int NX = kGfRun + 2 * R, NV = (NX + 3) / 4;
  const int row = task / runs, run = task - row * runs;
  const int j0 = run * kGfRun;
  const float4 *v4 = reinterpret_cast<const float4 *>(src + row * hs_pitch<R>() + j0);
  float x[4 * NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const float4 q = v4[k];
    x[4 * k] = q.x;
    x[4 * k + 1] = q.y;
    x[4 * k + 2] = q.z;
    x[4 * k + 3] = q.w;
  }
  float s = 0.0f;
#pragma unroll
  for (int i = 0; i <= 2 * R; ++i) s += x[i];
  float o[kGfRun];
  o[0] = s;
#pragma unroll
  for (int i = 1; i < kGfRun; ++i) {
    s += x[i + 2 * R] - x[i - 1];
    o[i] = s;
  }
  float4 *d4 = reinterpret_cast<float4 *>(dst + row * kGfThreads + j0);
#pragma unroll
  for (int k = 0; k < kGfRun / 4; ++k) d4[k] = make_float4(o[4 * k], o[4 * k + 1], o[4 * k + 2], o[4 * k + 3]);
}

// Zero the padding columns of `nrows` padded rows (every thread of the block calls this).
template <int R>
__device__ __forceinline__ void hs_zero_pads(float *buf, int nrows) {
  constexpr int P = hs_pitch<R>(), npad = P - kGfThreads;
  if constexpr (npad > 0) {
    for (int i = threadIdx.x; i < nrows * npad; i += blockDim.x) {
      const int r = i / npad, c = i - r * npad;
      buf[r * P + (c < R ? c : kGfThreads + c)] = 0.0f;
    }
  }
}

}  // namespace gfd
