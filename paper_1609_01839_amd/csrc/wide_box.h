// Separable box passes for guided-filter windows of any width (Sec. 2, Eqs.(3)-(5), with the
// box-filter remark of Sec. 3.1: the cost per pixel does not depend on w).
//
// The single-pass strip kernels keep the last w rows of their inputs in per-thread registers,
// which bounds them at r = kGfRmax.  Wider windows run each box stage as two launches:
//   k_wide_v: every thread owns one column of a strip of rows and slides a vertical window sum
//             of the stage's fields down it (FP64 accumulators: no drift however many slides);
//             the sums go to NF planes V of the image's size;
//   k_wide_h: one block per image row turns each V row into a FP64 prefix sum in LDS, takes the
//             horizontal window sums as differences of two prefixes (wrapped or clipped), stores
//             the window means back into V, then runs the stage's epilogue on every pixel of
//             the row.
// A stage is an Op (fields of the raw loads, an epilogue on the window means) like the ones of
// the strip kernels.  Windows wrap periodically (w <= min(M, N), so a window never holds a
// pixel twice) or, with CLIP, are clipped to the image and divided by their pixel counts; fields
// marked in Op::kT are transposed means (a gradient flowing back through B = D^-1 S): they are
// divided by the count of the input pixel's window before they are summed and their sums are
// used as they are.
#pragma once
#include <stddef.h>

#include <algorithm>

#include "box_sum.h"
#include "gfd_internal.h"

namespace gfd {

constexpr int kWideMaxN = 4096;   // widest row the horizontal pass holds in LDS
constexpr int kWideThreads = 256; // threads of a horizontal-pass block
constexpr int kWideVThreads = 64; // columns of a vertical-pass block

// Everything one wide stage reads and writes.  Pointers are device addresses.
struct WideArgs {
  const Img *d;          // the image's descriptor in the device table (reverse-mode stages), or null
  const float *src[4];   // input planes of the forward filter (guide and input, or guide channels + input)
  float *dst[4];         // coefficient planes between the two stages of the forward filter
  float *out;            // output plane of the forward filter
  float *V;              // NF planes of window sums, M * N floats apart
  const float *cen[4];   // device addresses of the centring constants (null: 0)
  float *eps_part;       // one partial sum of the eps gradient per image row (stages with kEps)
  double *pre;           // rows wider than kWideMaxN: M rows of N + 1 prefix sums (else unused)
  int M, N, r, clip;
  float eps;
  int table;             // 1: the forward filter's guide, input and output are d's u_I, u_p, u_E,
                         // read from the descriptor when the kernel runs
};

// The pointers a descriptor supplies, taken when the kernel runs (the reverse mode points its
// replay descriptors at other buffers between launches).
__device__ __forceinline__ void wide_resolve(WideArgs &a) {
  if (a.table) {
    a.src[0] = a.d->uI;
    a.src[1] = a.d->uP;
    a.out = a.d->uE;
  }
}

// Pixels of the window of half-width r centred at c inside [0, n).
__device__ __forceinline__ int wide_count(int c, int r, int n) { return min(c + r, n - 1) - max(c - r, 0) + 1; }

__device__ __forceinline__ void wide_centres(const WideArgs &a, float (&cen)[4]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) cen[k] = a.cen[k] ? *a.cen[k] : 0.0f;
}

// Vertical window sums of the stage's fields: block (bx, by) covers columns
// [bx * kWideVThreads, ...) and rows [by * TY, by * TY + TY).
template <class Op, bool CLIP>
__global__ void __launch_bounds__(kWideVThreads) k_wide_v(WideArgs a, int TY) {
  constexpr int NF = Op::NF, NR = Op::NR;
  wide_resolve(a);
  const int M = a.M, N = a.N, r = a.r;
  const int x = blockIdx.x * kWideVThreads + threadIdx.x;
  if (x >= N) return;  // no barriers in this kernel
  const int y0 = blockIdx.y * TY, y1 = min(y0 + TY, M);
  float cen[4];
  wide_centres(a, cen);
  const int cx = CLIP ? wide_count(x, r, N) : 1;
  // fields of image row y (any integer): wrapped into the image, or zero outside it with CLIP
  auto fields = [&](int y, double (&v)[NF]) {
    if (CLIP && (y < 0 || y >= M)) {
#pragma unroll
      for (int f = 0; f < NF; ++f) v[f] = 0.0;
      return;
    }
    const int yy = CLIP ? y : wrap(y, M);
    float raw[NR], fv[NF];
    Op::load(a, (size_t)yy * N + x, raw);
    Op::fields(raw, cen, fv);
    const float inv = CLIP ? 1.0f / (float)(wide_count(yy, r, M) * cx) : 1.0f;
#pragma unroll
    for (int f = 0; f < NF; ++f) v[f] = (double)(CLIP && ((Op::kT >> f) & 1u) ? fv[f] * inv : fv[f]);
  };
  double s[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) s[f] = 0.0;
  for (int y = y0 - r; y <= y0 + r; ++y) {
    double v[NF];
    fields(y, v);
#pragma unroll
    for (int f = 0; f < NF; ++f) s[f] += v[f];
  }
  const size_t P = (size_t)M * N;
  for (int y = y0; y < y1; ++y) {
#pragma unroll
    for (int f = 0; f < NF; ++f) a.V[f * P + (size_t)y * N + x] = (float)s[f];
    if (y + 1 < y1) {
      double vn[NF], vo[NF];
      fields(y + r + 1, vn);
      fields(y - r, vo);
#pragma unroll
      for (int f = 0; f < NF; ++f) s[f] += vn[f] - vo[f];
    }
  }
}

// Horizontal window sums, window means and the stage's epilogue for image row blockIdx.x.
// Rows of up to kWideMaxN pixels are staged in LDS with their FP64 prefix; longer rows (BIG,
// stand-alone filters only) read V directly and keep the prefix in a.pre, M rows of N + 1.
template <class Op, bool CLIP, bool BIG>
__global__ void __launch_bounds__(kWideThreads) k_wide_h(WideArgs a) {
  constexpr int NF = Op::NF, NR = Op::NR, NE = Op::NE;
  wide_resolve(a);
  constexpr int NW = kWideThreads / 64;
  __shared__ float row_lds[BIG ? 1 : kWideMaxN];
  __shared__ double pre_lds[BIG ? 1 : kWideMaxN + 1];
  __shared__ double wtot[NW];
  __shared__ float red[NW];
  const int M = a.M, N = a.N, r = a.r, y = blockIdx.x, t = threadIdx.x;
  const size_t P = (size_t)M * N, base = (size_t)y * N;
  double *pre = BIG ? a.pre + (size_t)y * (N + 1) : pre_lds;  // pre[x] = sum of the row's first x values
  const int chunk = (N + kWideThreads - 1) / kWideThreads;
  const int c0 = min(t * chunk, N), c1 = min(c0 + chunk, N);
  const int cy = CLIP ? wide_count(y, r, M) : 1;
  const float inv_w2 = 1.0f / ((float)(2 * r + 1) * (float)(2 * r + 1));
  for (int f = 0; f < NF; ++f) {
    float *Vf = a.V + f * P + base;
    const float *row = BIG ? Vf : row_lds;
    if (!BIG)
      for (int x = t; x < N; x += kWideThreads) row_lds[x] = Vf[x];
    __syncthreads();
    // exclusive prefix of this thread's chunk: scan of the chunk totals over the block
    double tot = 0.0;
    for (int x = c0; x < c1; ++x) tot += (double)row[x];
    double incl = tot;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const double u = __shfl_up(incl, o, 64);
      if ((t & 63) >= o) incl += u;
    }
    if ((t & 63) == 63) wtot[t >> 6] = incl;
    __syncthreads();
    double run = incl - tot;
    for (int k = 0; k < (t >> 6); ++k) run += wtot[k];
    for (int x = c0; x < c1; ++x) {
      pre[x] = run;
      run += (double)row[x];
    }
    if (t == kWideThreads - 1) pre[N] = run;  // the total (its chunk may be empty)
    __syncthreads();  // orders the prefix (LDS, or global within the block) before its reads
    for (int x = t; x < N; x += kWideThreads) {
      const int lo = x - r, hi = x + r;
      double S;
      if (CLIP) S = pre[min(hi, N - 1) + 1] - pre[max(lo, 0)];
      else if (lo < 0) S = pre[hi + 1] + (pre[N] - pre[N + lo]);
      else if (hi >= N) S = (pre[N] - pre[lo]) + pre[hi + 1 - N];
      else S = pre[hi + 1] - pre[lo];
      float nrm = inv_w2;
      if (CLIP) nrm = ((Op::kT >> f) & 1u) ? 1.0f : 1.0f / (float)(cy * wide_count(x, r, N));
      Vf[x] = (float)S * nrm;  // read back below by this same thread
    }
    __syncthreads();  // the row and its prefix are rewritten for the next field
  }
  float cen[4];
  wide_centres(a, cen);
  float eacc = 0.0f;
  for (int x = t; x < N; x += kWideThreads) {
    const size_t g = base + x;
    float B[NF], raw[NR], e[NE];
#pragma unroll
    for (int f = 0; f < NF; ++f) B[f] = a.V[f * P + g];
    Op::load(a, g, raw);
    Op::eload(a, g, e);
    Op::emit(a, g, B, raw, e, cen, eacc);
  }
  if (Op::kEps) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) eacc += __shfl_xor(eacc, o, 64);
    if ((t & 63) == 0) red[t >> 6] = eacc;
    __syncthreads();
    if (t == 0) {
      float h = 0.0f, l = 0.0f;
      for (int w = 0; w < NW; ++w) df_add(h, l, red[w], 0.0f);
      a.eps_part[y] = h + l;
    }
  }
}

// Rows per vertical-pass strip: the window's first sum (w loads) is amortised over at least
// 4r rows.
inline int wide_strip_rows(int M, int r) { return std::min(M, std::max(64, 4 * r)); }

// One stage: vertical sums, then horizontal sums and the epilogue (stream-ordered).
template <class Op, bool CLIP>
hipError_t wide_stage(const WideArgs &a, hipStream_t s) {
  const int TY = wide_strip_rows(a.M, a.r);
  hipLaunchKernelGGL((k_wide_v<Op, CLIP>), dim3((a.N + kWideVThreads - 1) / kWideVThreads, (a.M + TY - 1) / TY),
                     dim3(kWideVThreads), 0, s, a, TY);
  if (a.N > kWideMaxN) {
    if (a.pre == nullptr) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_wide_h<Op, CLIP, true>), dim3(a.M), dim3(kWideThreads), 0, s, a);
  } else {
    hipLaunchKernelGGL((k_wide_h<Op, CLIP, false>), dim3(a.M), dim3(kWideThreads), 0, s, a);
  }
  return hipGetLastError();
}

template <class Op>
hipError_t wide_stage(const WideArgs &a, hipStream_t s) {
  return a.clip ? wide_stage<Op, true>(a, s) : wide_stage<Op, false>(a, s);
}

// Device address of a field of an image's lambda state (no dereference on the host).
inline const float *state_field(const LamState *st, size_t offset) {
  return reinterpret_cast<const float *>(reinterpret_cast<const char *>(st) + offset);
}

}  // namespace gfd
