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

// Column of the strip owned by thread l.  Rows of sums are stored with a gap of 4 floats after
// every 8 columns (hs_col), so 8-column block b of a wave's 64 columns starts at bank 12 b mod
// 32: blocks 0, 2, 4, 6 cover the 32 banks once, and so do blocks 1, 3, 5, 7.  Lanes 0-31 of a
// wave therefore own blocks 0, 2, 4, 6 and lanes 32-63 blocks 1, 3, 5, 7, which keeps the
// one-float accesses of a half wave (served together) free of bank conflicts; a wave's global
// loads and stores still cover its 64 contiguous columns.
__device__ __forceinline__ int gf_col(int l) {
  const int x = l & 63;
  return (l & ~63) + 8 * (2 * ((x >> 3) & 3) + (x >> 5)) + (x & 7);
}

// Running window sum moved by one row: the row xo leaves, xn enters.
__device__ __forceinline__ void slide(float &s, float xn, float xo) { s = __fadd_rn(s, __fsub_rn(xn, xo)); }

// Pixels of the window of half-width R centred at c (a row or column index) inside [0, n).
template <int R>
__device__ __forceinline__ int clip_count(int c, int n) {
  return min(c + R, n - 1) - max(c - R, 0) + 1;
}

__device__ __forceinline__ int wrap(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

// LDS layout of the rows that the horizontal sums read and write: column c of a row sits at
// hs_col(c) = c + 4 (c / 8), i.e. every run of 8 columns is followed by 4 unused floats.  A
// horizontal-sum task reads and writes whole runs as float4 words; with runs 48 bytes apart the
// eight lanes that one LDS cycle serves hit eight different groups of four banks (runs 32 bytes
// apart would put two lanes on every group), and every float4 offset inside a task is a
// compile-time constant.
__host__ __device__ constexpr int hs_col(int c) { return c + 4 * (c >> 3); }

// Rows of horizontal sums (outputs): kGfThreads columns.
constexpr int kHsOut = hs_col(kGfThreads - 1) + 1;
static_assert(kHsOut % 4 == 0, "float4 rows");

// Rows of vertical sums are kept with R zero columns on each side: column c of the block is
// padded column c + R, at hs_col(c + R) of a row of hs_pitch<R>() floats.  The padding columns
// are zeroed once and never written, so that runs at the strip's edges read finite values
// without clamped indices.
template <int R>
constexpr int hs_nv() {
  return (kGfRun + 2 * R + 3) / 4;  // float4 words a task reads
}
template <int R>
constexpr int hs_last_col() {
  return kGfThreads - kGfRun + 4 * hs_nv<R>() - 1;  // last padded column a task reads
}
template <int R>
constexpr int hs_pitch() {
  return (hs_col(hs_last_col<R>()) + 1 + 3) & ~3;
}

// Horizontal window sums (half-width R) over rows of padded vertical sums: task `t` covers row
// t / runs and output columns [j0, j0 + kGfRun), j0 = run * kGfRun.  Its inputs, padded columns
// j0 .. j0 + kGfRun - 1 + 2R, are read as float4 words; the outputs go out as float4 words into
// rows of kHsOut floats.  Columns outside [R, used - R) produce don't-care values.
template <int R>
__device__ __forceinline__ void hsum_task(const float *__restrict__ src, float *__restrict__ dst, int task) {
  static_assert(kGfRun == 8, "runs of 8 columns (the LDS layout)");
  constexpr int runs = kGfThreads / kGfRun;
  constexpr int NV = hs_nv<R>();
  const int row = task / runs, run = task - row * runs;
  const int j0 = run * kGfRun;
  const float *in = src + row * hs_pitch<R>() + hs_col(j0);
  float x[4 * NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const float4 q = *reinterpret_cast<const float4 *>(in + 4 * k + 4 * (k >> 1));
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
  float *out = dst + row * kHsOut + hs_col(j0);
  *reinterpret_cast<float4 *>(out) = make_float4(o[0], o[1], o[2], o[3]);
  *reinterpret_cast<float4 *>(out + 4) = make_float4(o[4], o[5], o[6], o[7]);
}

// Zero the padding columns of `nrows` padded rows (every thread of the block calls this).
template <int R>
__device__ __forceinline__ void hs_zero_pads(float *buf, int nrows) {
  constexpr int P = hs_pitch<R>(), lo = R, hi = hs_last_col<R>() - (kGfThreads + R) + 1, npad = lo + hi;
  if constexpr (npad > 0) {
    for (int i = threadIdx.x; i < nrows * npad; i += blockDim.x) {
      const int r = i / npad, c = i - r * npad;
      buf[r * P + hs_col(c < lo ? c : kGfThreads + R + (c - lo))] = 0.0f;
    }
  }
}

}  // namespace gfd
