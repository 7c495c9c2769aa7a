// Guided filter with a three-channel guide on gfx950 (the colour case of Sec. 3.1's
// complexity remark; the multichannel form of Eqs.(3)-(5)).
//
// Per window k, with mu_k the guide's channel means and Sigma_k its 3 x 3 window covariance,
//   a_k = (Sigma_k + eps U)^-1 (mean_k(I p) - mu_k pbar_k),  b_k = pbar_k - a_k . mu_k,
//   u(i) = abar_i . I(i) + bbar_i,
// with abar, bbar the window means of a and b.  The kernel follows the grey filter's single
// streaming pass (one block per strip of TX columns and TY rows, two rows per round of
// barriers): stage 1 keeps compensated vertical running sums of the 13 products
// (I_c, p, I_c I_d for c <= d, I_c p), forms the horizontal window sums in LDS and solves each
// window's 3 x 3 system; stage 2 does the same over (a, b) and writes u.  The last w rows of the
// raw inputs and of (a, b) are held in per-thread register rings, so every input pixel is loaded
// once per strip.  The 3 x 3 systems are solved by cofactors in FP64: the covariance of strongly
// correlated channels is nearly singular at the scale of eps, and FP32 cofactors would lose
// most of their digits to cancellation.  Windows wrap periodically and every mean divides
// by w^2.  Inputs are shifted by their first pixels before products are formed.  Windows
// wider than the register rings hold (r > kGfRmax) run as two separable box stages
// (wide_box.h) with the same fields and the same FP64 solve.
#include "box_sum.h"
#include "gfd_internal.h"
#include "wide_box.h"

namespace gfd {

namespace {

constexpr int kC1 = 13;  // stage-1 fields
constexpr int kC2 = 4;   // stage-2 fields: a_r, a_g, a_b, b
// Rows per round: one for small radii (13 LDS rows per stream row: less LDS, more blocks per CU),
// two for wide windows, where the halo work dominates.
template <int R>
constexpr int gfc_rows() {
  return R <= 4 ? 1 : 2;
}

__device__ __forceinline__ void gfc_fields(const float (&x)[4], float (&v)[kC1]) {
  const float r = x[0], g = x[1], b = x[2], p = x[3];
  v[0] = r;
  v[1] = g;
  v[2] = b;
  v[3] = p;
  v[4] = r * r;
  v[5] = r * g;
  v[6] = r * b;
  v[7] = g * g;
  v[8] = g * b;
  v[9] = b * b;
  v[10] = r * p;
  v[11] = g * p;
  v[12] = b * p;
}

// (a_r, a_g, a_b, b) of one window from its 13 window means m (same order as gfc_fields).
__device__ __forceinline__ void gfc_coeffs(const float (&m)[kC1], float eps, float (&ab)[kC2]) {
  const double mr = m[0], mg = m[1], mb = m[2], pb = m[3];
  const double s00 = (double)m[4] - mr * mr + eps, s01 = (double)m[5] - mr * mg, s02 = (double)m[6] - mr * mb;
  const double s11 = (double)m[7] - mg * mg + eps, s12 = (double)m[8] - mg * mb;
  const double s22 = (double)m[9] - mb * mb + eps;
  const double c0 = (double)m[10] - mr * pb, c1 = (double)m[11] - mg * pb, c2 = (double)m[12] - mb * pb;
  // adjugate of the symmetric matrix
  const double A00 = s11 * s22 - s12 * s12, A01 = s02 * s12 - s01 * s22, A02 = s01 * s12 - s02 * s11;
  const double A11 = s00 * s22 - s02 * s02, A12 = s01 * s02 - s00 * s12, A22 = s00 * s11 - s01 * s01;
  const double det = s00 * A00 + s01 * A01 + s02 * A02;
  const double inv = 1.0 / det;
  const double a0 = (A00 * c0 + A01 * c1 + A02 * c2) * inv;
  const double a1 = (A01 * c0 + A11 * c1 + A12 * c2) * inv;
  const double a2 = (A02 * c0 + A12 * c1 + A22 * c2) * inv;
  ab[0] = (float)a0;
  ab[1] = (float)a1;
  ab[2] = (float)a2;
  ab[3] = (float)(pb - a0 * mr - a1 * mg - a2 * mb);
}

// The two stages as separable box stages: src = {I_r, I_g, I_b, p}, dst = {a_r, a_g, a_b, b},
// cen = the first pixels of the four inputs.
struct WideGfc1 {  // the 13 window means  ->  a, b
  static constexpr int NF = kC1, NR = 4, NE = 1;
  static constexpr unsigned kT = 0u;
  static constexpr bool kEps = false;
  __device__ static void load(const WideArgs &a, size_t g, float (&r)[NR]) {
#pragma unroll
    for (int c = 0; c < 4; ++c) r[c] = a.src[c][g];
  }
  __device__ static void eload(const WideArgs &, size_t, float (&e)[NE]) { e[0] = 0.0f; }
  __device__ static void fields(const float (&r)[NR], const float (&c)[4], float (&v)[NF]) {
    float x[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) x[k] = __fsub_rn(r[k], c[k]);
    gfc_fields(x, v);
  }
  __device__ static void emit(const WideArgs &a, size_t g, const float (&B)[NF], const float (&)[NR],
                              const float (&)[NE], const float (&)[4], float &) {
    float ab[kC2];
    gfc_coeffs(B, a.eps, ab);
#pragma unroll
    for (int k = 0; k < kC2; ++k) a.dst[k][g] = ab[k];
  }
};

struct WideGfc2 {  // window means of a, b  ->  u = abar . I + bbar
  static constexpr int NF = kC2, NR = kC2, NE = 3;
  static constexpr unsigned kT = 0u;
  static constexpr bool kEps = false;
  __device__ static void load(const WideArgs &a, size_t g, float (&r)[NR]) {
#pragma unroll
    for (int k = 0; k < kC2; ++k) r[k] = a.dst[k][g];
  }
  __device__ static void eload(const WideArgs &a, size_t g, float (&e)[NE]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) e[c] = a.src[c][g];
  }
  __device__ static void fields(const float (&r)[NR], const float (&)[4], float (&v)[NF]) {
#pragma unroll
    for (int k = 0; k < kC2; ++k) v[k] = r[k];
  }
  __device__ static void emit(const WideArgs &a, size_t g, const float (&B)[NF], const float (&)[NR],
                              const float (&e)[NE], const float (&c)[4], float &) {
    float acc = B[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) acc = __fmaf_rn(B[k], __fsub_rn(e[k], c[k]), acc);
    a.out[g] = __fadd_rn(acc, c[3]);
  }
};

}  // namespace

// One strip (logical block lb of an nbx x nby grid, nby strips per column).  Thread j owns
// column x0 - 2r + j of the strip extended by 2r on each side.
template <int R>
__device__ __forceinline__ void gfc_strip(const GFD_AS1 float *__restrict__ I3, const GFD_AS1 float *__restrict__ up,
                                          GFD_AS1 float *__restrict__ u, int M, int N, float eps, int TX, int TY,
                                          int nby, int lb, const float (&cen)[4], float *__restrict__ vbuf,
                                          float *__restrict__ hbuf) {
  constexpr int W = 2 * R + 1, RB = gfc_rows<R>(), VP = hs_pitch<R>();
  hs_zero_pads<R>(vbuf, RB * kC1);  // ordered before the first reads by the first barrier
  const float inv_w2 = 1.0f / (float)(W * W);
  const size_t plane = (size_t)M * N;
  const int bx = lb / nby, by = lb - bx * nby;
  const int x0 = bx * TX, y0 = by * TY;
  const int j = threadIdx.x, used = TX + 4 * R;
  const bool active = j < used;
  const int gx = wrap(x0 - 2 * R + j, N);
  const int nrows = TY + 4 * R, ybase = y0 - 2 * R;  // stream row it is image row ybase + it
  // Rows are fetched in stream order: the wrapped image row of the next fetch is carried from
  // one fetch to the next (no division per row); stream rows past the end repeat the last.
  int f_it = 0, f_row = wrap(ybase, M);
  auto fetch_next = [&](float (&x)[4]) {
    const size_t g = (size_t)f_row * N + gx;
    x[0] = I3[g];
    x[1] = I3[plane + g];
    x[2] = I3[2 * plane + g];
    x[3] = up[g];
    if (f_it < nrows - 1) {
      ++f_it;
      if (++f_row == M) f_row = 0;
    }
  };
  Kahan s1[kC1], s2[kC2];
#pragma unroll
  for (int f = 0; f < kC1; ++f) s1[f] = Kahan{0.0f, 0.0f};
#pragma unroll
  for (int f = 0; f < kC2; ++f) s2[f] = Kahan{0.0f, 0.0f};
  // Rings (slot = stream row mod W; the row loop is unrolled over RB * W rows so that slots are
  // compile-time indices): centred raw inputs of the last W stream rows, and the coefficients
  // of the last W rows of windows.
  float rx[W][4], rab[W][kC2];
#pragma unroll
  for (int k = 0; k < W; ++k) {
#pragma unroll
    for (int x = 0; x < 4; ++x) rx[k][x] = 0.0f;
#pragma unroll
    for (int x = 0; x < kC2; ++x) rab[k][x] = 0.0f;
  }
  float nx[RB][4];
#pragma unroll
  for (int q = 0; q < RB; ++q) fetch_next(nx[q]);  // stream rows 0 .. RB - 1
  for (int base0 = 0; base0 < nrows; base0 += RB * W) {
#pragma unroll
    for (int r = 0; r < W; ++r) {
      const int base = base0 + RB * r;
      if (base >= nrows) break;  // uniform
      float guide[RB][3];
      // ---- stage 1, vertical
#pragma unroll
      for (int q = 0; q < RB; ++q) {
        const int s = (RB * r + q) % W, sg = (RB * r + q + 1) % W;
        float xo[4], vn[kC1], vo[kC1];
#pragma unroll
        for (int x = 0; x < 4; ++x) {
          xo[x] = rx[s][x];  // stream row it - W (zeros while it < W)
          rx[s][x] = __fsub_rn(nx[q][x], cen[x]);
        }
#pragma unroll
        for (int x = 0; x < 3; ++x) guide[q][x] = rx[sg][x];  // stream row it - 2r
        gfc_fields(rx[s], vn);
        gfc_fields(xo, vo);
        float *vb = vbuf + q * kC1 * VP + hs_col(j + R);
        if (active && base + q < nrows) {
#pragma unroll
          for (int f = 0; f < kC1; ++f) {
            kahan_slide(s1[f], vn[f], vo[f]);
            vb[f * VP] = s1[f].s;
          }
        } else {
#pragma unroll
          for (int f = 0; f < kC1; ++f) vb[f * VP] = 0.0f;
        }
      }
#pragma unroll
      for (int q = 0; q < RB; ++q) fetch_next(nx[q]);  // stream rows base + RB + q
      __syncthreads();
      if (base + RB - 1 < W - 1) continue;  // no complete window in this round (uniform)
      // ---- stage 1, horizontal
      for (int t = j; t < RB * kC1 * (kGfThreads / kGfRun); t += kGfThreads) hsum_task<R>(vbuf, hbuf, t);
      __syncthreads();
      // ---- coefficients (one row of windows per stream row) and stage 2, vertical; the rows of
      // vbuf are reused, with the same padding, now that the stage-1 sums have been read
#pragma unroll
      for (int q = 0; q < RB; ++q) {
        const int it = base + q, it2 = it - (W - 1);  // row of (a, b) in the stage-2 stream
        float *vb = vbuf + q * kC2 * VP + hs_col(j + R);
        if (it < nrows && it2 >= 0 && j >= R && j < used - R) {
          const int slot = (RB * r + q + 1) % W;  // it2 mod W
          float m[kC1], ab[kC2];
#pragma unroll
          for (int f = 0; f < kC1; ++f) m[f] = hbuf[(q * kC1 + f) * kHsOut + hs_col(j)] * inv_w2;
          gfc_coeffs(m, eps, ab);
#pragma unroll
          for (int f = 0; f < kC2; ++f) {
            kahan_slide(s2[f], ab[f], it2 >= W ? rab[slot][f] : 0.0f);
            rab[slot][f] = ab[f];
            vb[f * VP] = s2[f].s;
          }
        } else {
          // columns without coefficients enter the first window of a sliding run: keep them zero
#pragma unroll
          for (int f = 0; f < kC2; ++f) vb[f * VP] = 0.0f;
        }
      }
      __syncthreads();
      if (base + RB - 1 < 4 * R) continue;  // no complete stage-2 window yet (uniform)
      // ---- stage 2, horizontal
      for (int t = j; t < RB * kC2 * (kGfThreads / kGfRun); t += kGfThreads) hsum_task<R>(vbuf, hbuf, t);
      __syncthreads();
      // ---- output rows
#pragma unroll
      for (int q = 0; q < RB; ++q) {
        const int it = base + q;
        const int yo = ybase + it - 2 * R, xo = x0 - 2 * R + j;
        if (it < nrows && it >= 4 * R && j >= 2 * R && j < TX + 2 * R && xo < N && yo < M && yo < y0 + TY) {
          const float *hb = hbuf + q * kC2 * kHsOut + hs_col(j);
          float acc = hb[3 * kHsOut] * inv_w2;
#pragma unroll
          for (int c = 0; c < 3; ++c) acc = __fmaf_rn(hb[c * kHsOut] * inv_w2, guide[q][c], acc);
          u[(size_t)yo * N + xo] = __fadd_rn(acc, cen[3]);
        }
      }
      // the next round's first barrier orders these hbuf reads before hbuf is rewritten
    }
  }
}

template <int R>
__global__ void __launch_bounds__(kGfThreads) k_gfc_plain(const float *__restrict__ I3, const float *__restrict__ up,
                                                          float *__restrict__ u, int M, int N, float eps, int TX,
                                                          int TY, int nby) {
  __shared__ __align__(16) float vbuf[gfc_rows<R>() * kC1 * hs_pitch<R>()];
  __shared__ __align__(16) float hbuf[gfc_rows<R>() * kC1 * kHsOut];
  const size_t plane = (size_t)M * N;
  const float cen[4] = {I3[0], I3[plane], I3[2 * plane], up[0]};
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  gfc_strip<R>(G(I3), G(up), G(u), M, N, eps, TX, TY, nby, lb, cen, vbuf, hbuf);
}

hipError_t launch_guided_filter_color(const float *I3, const float *up, float *u, int M, int N, int w, float eps,
                                      hipStream_t s) {
  const int r = (w - 1) / 2;
  if (!guided_filter_supported(w)) return hipErrorInvalidValue;
  if (gf_wide(w)) {
    // separable passes: 13 planes of window sums and the 4 coefficient planes (and the row
    // prefixes of rows wider than kWideMaxN), stream-ordered temporaries
    const size_t P = (size_t)M * N;
    const size_t npre = N > kWideMaxN ? (size_t)M * (N + 1) : 0;
    float *tmp = nullptr;
    hipError_t e = hipMallocAsync((void **)&tmp, (kC1 + kC2) * P * sizeof(float) + npre * sizeof(double), s);
    if (e != hipSuccess) return e;
    WideArgs a = {};
    a.pre = npre ? reinterpret_cast<double *>(tmp + (kC1 + kC2) * P) : nullptr;
    a.V = tmp;
    for (int c = 0; c < 3; ++c) {
      a.src[c] = I3 + c * P;
      a.cen[c] = I3 + c * P;  // the first pixels, like the strip kernel
    }
    a.src[3] = up;
    a.cen[3] = up;
    for (int k = 0; k < kC2; ++k) a.dst[k] = tmp + (kC1 + k) * P;
    a.out = u;
    a.M = M;
    a.N = N;
    a.r = r;
    a.clip = 0;
    a.eps = eps;
    e = wide_stage<WideGfc1>(a, s);
    if (e == hipSuccess) e = wide_stage<WideGfc2>(a, s);
    const hipError_t ef = hipFreeAsync(tmp, s);
    return e != hipSuccess ? e : ef;
  }
  int TX = kGfThreads - 4 * r, TY = 64;
  if (TX > N) TX = N;
  if (TY > M) TY = M;
  const int nbx = (N + TX - 1) / TX, nby = (M + TY - 1) / TY;
#define GFD_LAUNCH_GFC(RR) \
  hipLaunchKernelGGL(k_gfc_plain<RR>, dim3(nbx * nby), dim3(kGfThreads), 0, s, I3, up, u, M, N, eps, TX, TY, nby)
  switch (r) {
    case 0: GFD_LAUNCH_GFC(0); break;
    case 1: GFD_LAUNCH_GFC(1); break;
    case 2: GFD_LAUNCH_GFC(2); break;
    case 3: GFD_LAUNCH_GFC(3); break;
    case 4: GFD_LAUNCH_GFC(4); break;
    case 5: GFD_LAUNCH_GFC(5); break;
    case 6: GFD_LAUNCH_GFC(6); break;
    case 7: GFD_LAUNCH_GFC(7); break;
    case 8: GFD_LAUNCH_GFC(8); break;
    default: return hipErrorInvalidValue;
  }
#undef GFD_LAUNCH_GFC
  return hipGetLastError();
}

}  // namespace gfd
