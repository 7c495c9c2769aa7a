// Guided filter u = guidfilter(u_I, u_p, w, eps) on gfx950 (Sec. 2, Eqs.(3)-(5)).
//
// One block owns a strip of TX output columns and TY output rows and streams down its rows.
// Every thread owns one column of the strip extended by 2r on each side (r = (w-1)/2):
//   stage 1: vertical running sums over the last w rows of I, p, I*I, I*p (compensated FP32),
//            then horizontal sums of those across the block's columns -> w x w window sums,
//            giving a_k and b_k (Eqs.(3)-(4)) one row of windows at a time;
//   stage 2: the same two-direction running sums over a and b -> abar, bbar (Eq.(5)), and
//            u = abar * I + bbar.
// The last w rows of (I, p) and of (a, b) sit in LDS rings so that the rows leaving the
// vertical windows can be subtracted.  Windows wrap periodically in both directions.
// The inputs are shifted by constants (the image means when known) before the products
// are formed; the filter commutes with such shifts (u shifts by the input's constant).
#include "gfd_internal.h"

namespace gfd {

constexpr int kGfThreads = 256;
constexpr int kGfRmax = 8;
constexpr int kGfRun = 4;  // columns per thread in the horizontal sums

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

// Horizontal window sums of NQ rows of values held in LDS (row q at src + q * kGfThreads):
// thread (q, run) produces columns [run*kGfRun, run*kGfRun + kGfRun).
template <int NQ>
__device__ __forceinline__ void hsum_rows(const float *src, float *dst, int r) {
  const int t = threadIdx.x;
  constexpr int runs = kGfThreads / kGfRun;
  if (t >= NQ * runs) return;
  const int q = t / runs, run = t - q * runs;
  const float *v = src + q * kGfThreads;
  const int j0 = run * kGfRun;
  float s = 0.0f;
  for (int d = -r; d <= r; ++d) s += v[min(max(j0 + d, 0), kGfThreads - 1)];
  float *o = dst + q * kGfThreads + j0;
  o[0] = s;
#pragma unroll
  for (int i = 1; i < kGfRun; ++i) {
    s += v[min(j0 + i + r, kGfThreads - 1)] - v[max(j0 + i - 1 - r, 0)];
    o[i] = s;
  }
}

__global__ void __launch_bounds__(kGfThreads) k_guided_filter(const float *__restrict__ uI, const float *__restrict__ uP,
                                                              float *__restrict__ u, int M, int N, int r, float eps,
                                                              int TX, int TY, int nby, const float *__restrict__ cIp,
                                                              const float *__restrict__ cPp, int *iter_counter) {
  __shared__ float2 ringIP[(2 * kGfRmax + 1) * kGfThreads];
  __shared__ float2 ringAB[(2 * kGfRmax + 1) * kGfThreads];
  __shared__ float vbuf[4 * kGfThreads];
  __shared__ float hbuf[4 * kGfThreads];

  if (iter_counter != nullptr && blockIdx.x == 0 && threadIdx.x == 0) *iter_counter += 1;

  const int w = 2 * r + 1;
  const float inv_w2 = 1.0f / (float)(w * w);
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int bx = lb / nby, by = lb - bx * nby;
  const int x0 = bx * TX, y0 = by * TY;
  const int j = threadIdx.x;
  const int used = TX + 4 * r;
  const int gx = wrap(x0 - 2 * r + j, N);
  const float cI = *cIp, cP = *cPp;

  Kahan sI = {0, 0}, sP = {0, 0}, sII = {0, 0}, sIP = {0, 0}, sA = {0, 0}, sB = {0, 0};
  const int nrows = TY + 4 * r;
  for (int it = 0; it < nrows; ++it) {
    // ---- stage 1, vertical: add row `it`, drop row `it - w`
    const int gy = wrap(y0 - 2 * r + it, M);
    const int slot = it % w;
    if (j < used) {
      const size_t g = (size_t)gy * N + gx;
      const float I = __fsub_rn(uI[g], cI), p = __fsub_rn(uP[g], cP);
      float2 old = make_float2(0.0f, 0.0f);
      if (it >= w) old = ringIP[slot * kGfThreads + j];
      ringIP[slot * kGfThreads + j] = make_float2(I, p);
      kahan_slide(sI, I, old.x);
      kahan_slide(sP, p, old.y);
      kahan_slide(sII, I * I, old.x * old.x);
      kahan_slide(sIP, I * p, old.x * old.y);
      vbuf[0 * kGfThreads + j] = sI.s;
      vbuf[1 * kGfThreads + j] = sP.s;
      vbuf[2 * kGfThreads + j] = sII.s;
      vbuf[3 * kGfThreads + j] = sIP.s;
    }
    __syncthreads();
    if (it < w - 1) continue;  // no complete window yet (uniform across the block)
    // ---- stage 1, horizontal: window sums centred at row it - r
    hsum_rows<4>(vbuf, hbuf, r);
    __syncthreads();
    // ---- coefficients a, b (Eqs. 3-4) and stage 2, vertical
    const int it2 = it - (w - 1);  // index of this row of (a, b) in the stage-2 stream
    const int slot2 = it2 % w;
    if (j >= r && j < used - r) {
      const float mu = hbuf[j] * inv_w2;
      const float pb = hbuf[kGfThreads + j] * inv_w2;
      const float var = fmaxf(__fmaf_rn(-mu, mu, hbuf[2 * kGfThreads + j] * inv_w2), 0.0f);
      const float cov = __fmaf_rn(-mu, pb, hbuf[3 * kGfThreads + j] * inv_w2);
      const float a = cov / (var + eps);
      const float b = __fmaf_rn(-a, mu, pb);
      float2 old = make_float2(0.0f, 0.0f);
      if (it2 >= w) old = ringAB[slot2 * kGfThreads + j];
      ringAB[slot2 * kGfThreads + j] = make_float2(a, b);
      kahan_slide(sA, a, old.x);
      kahan_slide(sB, b, old.y);
      vbuf[j] = sA.s;
      vbuf[kGfThreads + j] = sB.s;
    }
    __syncthreads();
    if (it2 < w - 1) continue;
    // ---- stage 2, horizontal: window sums of a, b centred at row it - 2r
    hsum_rows<2>(vbuf, hbuf, r);
    __syncthreads();
    const int yo = y0 - 2 * r + it - 2 * r;  // output row
    const int xo = x0 - 2 * r + j;           // output column
    if (j >= 2 * r && j < TX + 2 * r && xo < N && yo < M && yo < y0 + TY) {
      const float abar = hbuf[j] * inv_w2, bbar = hbuf[kGfThreads + j] * inv_w2;
      const float I = ringIP[((it - 2 * r) % w) * kGfThreads + j].x;
      u[(size_t)yo * N + xo] = __fadd_rn(__fmaf_rn(abar, I, bbar), cP);
    }
  }
}

bool guided_filter_supported(int w) { return w >= 1 && (w % 2) == 1 && (w - 1) / 2 <= kGfRmax; }

hipError_t launch_guided_filter(const float *uI, const float *uP, float *u, int M, int N, int w, float eps,
                                const float *cI, const float *cP, int *iter_counter, hipStream_t st) {
  const int r = (w - 1) / 2;
  int TX = kGfThreads - 4 * r;
  if (TX > N) TX = N;
  int TY = 64;
  if (TY > M) TY = M;
  const int nbx = (N + TX - 1) / TX, nby = (M + TY - 1) / TY;
  hipLaunchKernelGGL(k_guided_filter, dim3(nbx * nby), dim3(kGfThreads), 0, st, uI, uP, u, M, N, r, eps, TX, TY, nby,
                     cI, cP, iter_counter);
  return hipGetLastError();
}

}  // namespace gfd
