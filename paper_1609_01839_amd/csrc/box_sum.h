// Building blocks of the streaming box sums of the guided filter and of its adjoint: a block
// of kGfThreads threads owns one column each, keeps compensated vertical running sums and
// forms horizontal window sums from them in LDS.
#pragma once
#include <hip/hip_runtime.h>

namespace gfd {

constexpr int kGfThreads = 256;
constexpr int kGfRmax = 8;
constexpr int kGfRun = 4;  // columns per thread in the horizontal sums
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

__device__ __forceinline__ int wrap(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

// Horizontal window sums (half-width R) of `ntask` rows of kGfThreads values: task `t` covers
// row t / runs and columns [run * kGfRun, run * kGfRun + kGfRun).  Columns outside [R, used - R)
// produce don't-care values.
template <int R>
__device__ __forceinline__ void hsum_task(const float *__restrict__ src, float *__restrict__ dst, int task) {
  constexpr int runs = kGfThreads / kGfRun;
  const int row = task / runs, run = task - row * runs;
  const float *v = src + row * kGfThreads;
  const int j0 = run * kGfRun;
  float x[kGfRun + 2 * R];
#pragma unroll
  for (int i = 0; i < kGfRun + 2 * R; ++i) x[i] = v[min(max(j0 - R + i, 0), kGfThreads - 1)];
  float s = 0.0f;
#pragma unroll
  for (int i = 0; i <= 2 * R; ++i) s += x[i];
  float *o = dst + row * kGfThreads + j0;
  o[0] = s;
#pragma unroll
  for (int i = 1; i < kGfRun; ++i) {
    s += x[i + 2 * R] - x[i - 1];
    o[i] = s;
  }
}

}  // namespace gfd
