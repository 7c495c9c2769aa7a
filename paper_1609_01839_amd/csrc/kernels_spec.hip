// Spectral part of the iteration on gfx950: row / column FFT passes over a tile-major half
// spectrum, the residual and lambda reductions (Sec. 3.2, Eqs.(10)-(11)), the two Fourier
// solves (Sec. 3.1, Eqs.(8)-(9)) and the per-image set-up.
//
// Hot-path kernels take a device table of image descriptors (Img) and a work list of
// (image, block) items: one launch serves every image of a batch that shares the kernel
// variant, and a single image is a batch of one.  Work lists are padded per image to a
// multiple of 8 items and each image's blocks are permuted so that the blocks the hardware
// sends to one XCD (every 8th) are neighbouring tiles or rows sharing that XCD's L2.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <tuple>
#include <type_traits>

#include "gfd_internal.h"

namespace gfd {

// ============================================================================ reductions

// Plain FP32 butterfly over the wave, then compensated across the waves in wave order by NV
// threads in parallel: thread v (< NV) ends with value v in (h, l).  A block of fewer than 64
// threads (a power of two: the register-resident column pass at 256 rows and two columns has
// 32) is one partial wave, and its butterfly stays within its lanes.
template <int NV>
__device__ __forceinline__ void block_sum_plain_then_df(float (&acc)[NV], float &h, float &l, float *scratch) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    if (off >= (int)blockDim.x) continue;  // uniform
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] += __shfl_xor(acc[v], off, 64);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) scratch[wid * NV + v] = acc[v];
  }
  __syncthreads();
  h = 0.0f;
  l = 0.0f;
  if ((int)threadIdx.x < NV) {
    for (int w = 0; w < nw; ++w) df_add(h, l, scratch[w * NV + threadIdx.x], 0.0f);
  }
}

// Partial sums are stored structure-of-arrays, part[(2 a + {0: hi, 1: lo}) * npart + block];
// thread a (< nv) stores value a.
__device__ __forceinline__ void store_partial(GFD_AS1 float *part, int npart, int blk, int nv, float h, float l) {
  const int a = threadIdx.x;
  if (a < nv) {
    part[(size_t)(2 * a) * npart + blk] = h;
    part[(size_t)(2 * a + 1) * npart + blk] = l;
  }
}

// Compensated sums of the NV values of the partials of `nparts` blocks.  Wave w takes values
// w, w + nwaves, ... in pairs (w and w + nwaves, then w + 2 nwaves and w + 3 nwaves, ...): each
// lane accumulates the partials lane, lane + 64, ... of both values in order (loaded U at a time
// for both values before either is added, so that a pair of values with up to 64 U partials
// costs one memory round trip), then the wave combines its lanes by shuffles.  A wave whose pair
// has no second value loads the first one twice and keeps one result.  Deterministic order (each
// value's additions are the same as with one value per pass); thread 0 receives all NV sums.
// `scratch` must hold 2 NV floats.  U: partials per lane and value loaded together (4 U
// registers).
template <int NV, int U = 32>
__device__ __forceinline__ void reduce_partials(const GFD_AS1 float *__restrict__ part, int npart, int nparts, float (&hi)[NV],
                                float (&lo)[NV], float *scratch) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = max((int)(blockDim.x >> 6), 1);
  for (int v = wid; v < NV; v += 2 * nw) {
    const bool two = v + nw < NV;  // uniform in the wave
    const int v2 = two ? v + nw : v;
    const GFD_AS1 float *ph = part + (size_t)(2 * v) * npart, *pl = part + (size_t)(2 * v + 1) * npart;
    const GFD_AS1 float *qh = part + (size_t)(2 * v2) * npart, *ql = part + (size_t)(2 * v2 + 1) * npart;
    float h = 0.0f, l = 0.0f, h2 = 0.0f, l2 = 0.0f;
    for (int p0 = lane; p0 < nparts; p0 += 64 * U) {
      float xh[U], xl[U], yh[U], yl[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int p = p0 + 64 * u;
        xh[u] = p < nparts ? ph[p] : 0.0f;
        xl[u] = p < nparts ? pl[p] : 0.0f;
        yh[u] = p < nparts ? qh[p] : 0.0f;
        yl[u] = p < nparts ? ql[p] : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        df_add(h, l, xh[u], xl[u]);
        df_add(h2, l2, yh[u], yl[u]);
      }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const float oh = __shfl_down(h, off, 64), ol = __shfl_down(l, off, 64);
      const float oh2 = __shfl_down(h2, off, 64), ol2 = __shfl_down(l2, off, 64);
      df_add(h, l, oh, ol);
      df_add(h2, l2, oh2, ol2);
    }
    if (lane == 0) {
      scratch[2 * v] = h;
      scratch[2 * v + 1] = l;
      if (two) {
        scratch[2 * v2] = h2;
        scratch[2 * v2 + 1] = l2;
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      hi[v] = scratch[2 * v];
      lo[v] = scratch[2 * v + 1];
    }
  }
  __syncthreads();
}

// Commit the lambda of this iteration (one thread, once the search is finished).  The search
// state is a private copy `st` that the caller writes back.  With `advance` the iteration's
// bookkeeping is closed as well: the counter moves on and the first candidates of the next
// search are seeded (nothing later in the iteration reads the counter or the candidates).
// A search that precedes the first iteration (a warm start, `advance` = 0) keeps the counter;
// the next search has the same estimate and hence the same root, so its candidates are seeded
// around lambda_star with the narrowest spacing.
__device__ __forceinline__ void lam_commit(const Img &d, LamState &st, int advance) {
  const float ls = st.lam_star;
  float lam = ls;
  if (!isinf(ls)) {
    const float sc = (d.scales != nullptr && st.k < st.nscale) ? d.scales[st.k] : 1.0f;
    lam = sc * ls;
    if (!(st.flags & kFlagNoRoot)) {
      st.lam_prev2 = st.lam_prev;
      st.lam_prev = ls;
    }
  }
  st.lam = lam;
  st.flags_all |= (unsigned)st.flags;
  if (d.lam_hist != nullptr && st.k < d.hist_cap) {
    d.lam_hist[st.k] = lam;
    d.flag_hist[st.k] = st.flags;
    if (d.lam_star_hist != nullptr) d.lam_star_hist[st.k] = ls;
  }
  if (advance) {
    st.k += 1;
    lam_first_candidates(st);
  } else if (!isinf(ls) && !(st.flags & kFlagNoRoot)) {
    st.lam_prev2 = st.lam_prev;
    lam_first_candidates(st);
  }
}

// Per-bin contribution to the first lambda round: Einf, the floor and the candidates.
template <int NC>
__device__ __forceinline__ void first_round_terms(float qq, float t2, const float (&mu)[NC],
                                                  float (&acc)[2 + 2 * NC]) {
  acc[0] += qq;
  {
    const float r = __builtin_amdgcn_rcpf(__fmaf_rn(t2, 1.0f / kLamFloor, 1.0f));
    acc[1] = __fmaf_rn(qq, r * r, acc[1]);
  }
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    const float r = __builtin_amdgcn_rcpf(__fmaf_rn(t2, mu[j], 1.0f));
    const float qg = qq * (r * r);
    acc[2 + j] += qg;
    acc[2 + NC + j] = __fmaf_rn(qg, 1.0f - r, acc[2 + NC + j]);
  }
}

// The residual pass opens the image's search for the rounds launch that follows it (the kernel
// boundary orders these stores before that launch's reads): lambda not fixed, no round folded.
__device__ __forceinline__ void lam_open(LamState *st) {
  st->phase = 0;
  st->round = -1;
}

// ============================================================================ device bodies (any length)

// Row pass, forward, rows [r0, r0 + R): rows are paired into complex sequences z = x_a + i x_b,
// transformed in LDS, and separated into the two half spectra
// X_a[k] = (Z[k] + conj Z[N-k]) / 2, X_b[k] = (Z[k] - conj Z[N-k]) / 2i, written tile-major.
template <class T, int E, class XP, class SP>
__device__ __forceinline__ void row_fwd_body(XP x, const Layout &lay, const FftPlan &pn,
                                             const GFD_AS1 cpx<T> *__restrict__ tw, SP S, int blk, cpx<T> *buf) {
  const int M = lay.M, N = lay.N, R = lay.R, LP = N + 1;
  const int npair = R >> 1;
  const int r0 = blk * R;
#pragma unroll 8
  for (int e = threadIdx.x; e < npair * N; e += blockDim.x) {
    const int b = fdiv(e, lay.Ndiv), n = e - b * N;
    const int ra = r0 + 2 * b, rb = ra + 1;
    T re = ra < M ? (T)x[(size_t)ra * N + n] : (T)0;
    T im = rb < M ? (T)x[(size_t)rb * N + n] : (T)0;
    buf[b * LP + n] = cpx<T>{re, im};
  }
  __syncthreads();
  lds_fft<T, E, -1, false>(buf, npair, 0, 1, LP, pn, tw);
  const int C = lay.C, per_t = R * C, Wh = lay.Wh;
  const int total = lay.NT * per_t;
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    const int t = fdiv(e, lay.RCdiv), rem = e - t * per_t;
    const int rho = rem >> lay.logC, c = rem & (C - 1);
    const int m = r0 + rho;
    if (m >= M) continue;
    const int k = t * C + c;
    cpx<T> X = {(T)0, (T)0};
    if (k < Wh) {
      const cpx<T> *z = buf + (rho >> 1) * LP;
      cpx<T> Zk = z[k], Zn = z[k == 0 ? 0 : N - k];
      if ((rho & 1) == 0) X = cpx<T>{(Zk.re + Zn.re) * (T)0.5, (Zk.im - Zn.im) * (T)0.5};
      else X = cpx<T>{(Zk.im + Zn.im) * (T)0.5, (Zn.re - Zk.re) * (T)0.5};
    }
    S[(size_t)t * lay.TS + (size_t)m * C + c] = X;
  }
}

// Column pass, forward, of one tile: its C columns are transformed in LDS.
template <class T, int E, class TP>
__device__ __forceinline__ void col_fwd_load_fft(TP tile, const Layout &lay, const FftPlan &pm,
                                                 const GFD_AS1 cpx<T> *__restrict__ tw, cpx<T> *buf) {
  const int n = lay.M * lay.C;
#pragma unroll 8
  for (int e = threadIdx.x; e < n; e += blockDim.x) buf[e] = tile[e];
  __syncthreads();
  lds_fft<T, E, -1, true>(buf, lay.C, lay.logC, lay.C, 1, pm, tw);
}

// Spectral solves of Eqs.(8)-(9) for one bin:
//   F(u_p) = (conj(H) Y + lam F(u_E)) / (|H|^2 + lam)
//   F(u_I) = (conj(H) Y + lam D2 F(u_E)) / (|H|^2 + lam D2),  D2 = |F(grad)|^2,
// written with mu = 1/lam when lam >= 1 so that nothing overflows for large lam; lam = +inf
// copies F(u_E) to both.  The 1/P of the inverse transform is folded in.
struct SolveParams {
  float lam, invP, mu;
  bool inf_branch, big;
};
__device__ __forceinline__ SolveParams solve_params(const LamState *st) {
  SolveParams s;
  s.lam = st->lam;
  s.invP = st->invP;
  s.inf_branch = isinf(s.lam);
  s.big = s.lam >= 1.0f;
  s.mu = s.big ? 1.0f / s.lam : 0.0f;
  return s;
}
// MODE 0: lambda = +inf, 1: lambda >= 1 (written with mu = 1/lambda), 2: lambda < 1.
template <int MODE>
__device__ __forceinline__ void solve_bin_mode(const SolveParams &sp, cf U, cf hy, float t2, float d2, cf &Up,
                                               cf &Ui) {
  if constexpr (MODE == 0) {
    Up = cscale(U, sp.invP);
    Ui = Up;
  } else if constexpr (MODE == 1) {
    const float ip = sp.invP * __builtin_amdgcn_rcpf(__fmaf_rn(sp.mu, t2, 1.0f));
    const float ii = sp.invP * __builtin_amdgcn_rcpf(__fmaf_rn(sp.mu, t2, d2));
    Up = cf{(__fmaf_rn(sp.mu, hy.re, U.re)) * ip, (__fmaf_rn(sp.mu, hy.im, U.im)) * ip};
    Ui = cf{(__fmaf_rn(sp.mu, hy.re, d2 * U.re)) * ii, (__fmaf_rn(sp.mu, hy.im, d2 * U.im)) * ii};
  } else {
    const float ip = sp.invP * __builtin_amdgcn_rcpf(t2 + sp.lam);
    const float ld = sp.lam * d2;
    const float ii = sp.invP * __builtin_amdgcn_rcpf(t2 + ld);
    Up = cf{__fmaf_rn(sp.lam, U.re, hy.re) * ip, __fmaf_rn(sp.lam, U.im, hy.im) * ip};
    Ui = cf{__fmaf_rn(ld, U.re, hy.re) * ii, __fmaf_rn(ld, U.im, hy.im) * ii};
  }
}

__device__ __forceinline__ void solve_bin(const SolveParams &sp, cf U, cf hy, float t2, float d2, cf &Up, cf &Ui) {
  if (sp.inf_branch) solve_bin_mode<0>(sp, U, hy, t2, d2, Up, Ui);
  else if (sp.big) solve_bin_mode<1>(sp, U, hy, t2, d2, Up, Ui);
  else solve_bin_mode<2>(sp, U, hy, t2, d2, Up, Ui);
}

// ============================================================================ hot-path kernels, any length

#define GFD_ITEM_LOOP                                        \
  for (int ii = blockIdx.x; ii < nitems; ii += gridDim.x) { \
    const Item wi = W[ii];                                   \
    if (wi.blk < 0) continue;                                \
    const Img &d = D[wi.img];
#define GFD_ITEM_END \
  __syncthreads();   \
  }

template <int E>
__global__ void __launch_bounds__(1024) k_row_fwd_g(const Img *__restrict__ D, const Item *__restrict__ W, int nitems) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cf *buf = reinterpret_cast<cf *>(smem_raw);
  GFD_ITEM_LOOP
  row_fwd_body<float, E>(G(d.uE), d.L, d.pn, G(d.twN), G(d.S1), wi.blk, buf);
  GFD_ITEM_END
}

template <int E, bool RESID>
__global__ void __launch_bounds__(1024) k_col_fwd_g(const Img *__restrict__ D, const Item *__restrict__ W, int nitems) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cf *buf = reinterpret_cast<cf *>(smem_raw);
  __shared__ float scratch[kLamAcc * 16];
  GFD_ITEM_LOOP
  const Layout &lay = d.L;
  const int n = lay.M * lay.C, C = lay.C;
  const size_t off = (size_t)wi.blk * lay.TS;
  GFD_AS1 cf *tile = G(d.S1) + off;
  // F(h) and F(y) of this thread's bins do not depend on the transform: their loads are issued
  // first so that they travel while the column transform runs
  cf hv[RESID ? E : 1], yv[RESID ? E : 1];
  if (RESID) {
#pragma unroll
    for (int u = 0; u < E; ++u) {
      const int e = min((int)threadIdx.x + u * (int)blockDim.x, n - 1);
      hv[u] = G(d.H)[off + e];
      yv[u] = G(d.Y)[off + e];
    }
  }
  col_fwd_load_fft<float, E>(tile, lay, d.pm, G(d.twM), buf);
  if (!RESID) {
    for (int e = threadIdx.x; e < n; e += blockDim.x) tile[e] = buf[e];
  } else {
    // fused with the residual R = H U_E - Y of Eq.(10), q = w |R|^2 (w = 1 on columns 0 and
    // N/2, else 2), Einf = sum q / P and the first lambda candidates
    constexpr int NC = kLamFirstCand;
    float mu[NC];
#pragma unroll
    for (int j = 0; j < NC; ++j) mu[j] = d.st->mu[j];
    float acc[2 + 2 * NC];
#pragma unroll
    for (int a = 0; a < 2 + 2 * NC; ++a) acc[a] = 0.0f;
    const int kbase = wi.blk * C;
#pragma unroll
    for (int u = 0; u < E; ++u) {
      const int e = threadIdx.x + u * blockDim.x;
      if (e < n) {
        const cf U = buf[e];
        tile[e] = U;
        const int k = kbase + (e & (C - 1));
        float qq = 0.0f, t2 = 0.0f;
        if (k < lay.Wh) {  // padding columns hold zeros in H and Y
          const cf r = cmul(hv[u], U) - yv[u];
          qq = ((k == 0 || 2 * k == lay.N) ? 1.0f : 2.0f) * abs2f(r);
          t2 = abs2f(hv[u]);
        }
        G(d.q)[off + e] = qq;
        first_round_terms<NC>(qq, t2, mu, acc);
      }
    }
    float h, l;
    block_sum_plain_then_df<2 + 2 * NC>(acc, h, l, scratch);
    store_partial(G(d.part), d.npart, wi.blk, 2 + 2 * NC, h, l);
    if (wi.blk == 0 && threadIdx.x == 0) lam_open(d.st);
  }
  GFD_ITEM_END
}

template <int E>
__global__ void __launch_bounds__(1024) k_col_inv_g(const Img *__restrict__ D, const Item *__restrict__ W, int nitems) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cf *buf = reinterpret_cast<cf *>(smem_raw);
  GFD_ITEM_LOOP
  const Layout &lay = d.L;
  const int n = lay.M * lay.C, C = lay.C;
  const size_t off = (size_t)wi.blk * lay.TS;
  const SolveParams sp = solve_params(d.st);
  const int kbase = wi.blk * C;
  // straight-line elements (case split outside the loop, clamped indices, padding columns
  // zeroed by a select, the means written afterwards) so that their loads issue together
  cf ui[E], up[E];
  auto elems = [&](auto mode) {
    constexpr int MODE = decltype(mode)::value;
#pragma unroll
    for (int u = 0; u < E; ++u) {
      const int e = min((int)threadIdx.x + u * (int)blockDim.x, n - 1);
      const int k = kbase + (e & (C - 1)), m = e >> lay.logC;
      cf Up, Ui;
      solve_bin_mode<MODE>(sp, G(d.S1)[off + e], G(d.HY)[off + e], G(d.H2)[off + e],
                           G(d.dM)[m] + G(d.dN)[min(k, lay.Wh - 1)], Up, Ui);
      const bool ok = k < lay.Wh;
      up[u] = ok ? Up : cf{0.0f, 0.0f};
      ui[u] = ok ? Ui : cf{0.0f, 0.0f};
    }
  };
  if (sp.inf_branch) elems(std::integral_constant<int, 0>{});
  else if (sp.big) elems(std::integral_constant<int, 1>{});
  else elems(std::integral_constant<int, 2>{});
  if (threadIdx.x == 0 && wi.blk == 0) {  // zero frequency (row 0, column 0): the means
    d.st->meanP = up[0].re;
    d.st->meanI = ui[0].re;
  }
#pragma unroll
  for (int u = 0; u < E; ++u) {
    const int e = threadIdx.x + u * blockDim.x;
    if (e < n) buf[e] = up[u];
  }
  __syncthreads();
  lds_fft<float, E, +1, true>(buf, C, lay.logC, C, 1, d.pm, G(d.twM));
  for (int e = threadIdx.x; e < n; e += blockDim.x) G(d.SIP)[2 * (off + e) + 1] = buf[e];
  __syncthreads();
#pragma unroll
  for (int u = 0; u < E; ++u) {
    const int e = threadIdx.x + u * blockDim.x;
    if (e < n) buf[e] = ui[u];
  }
  __syncthreads();
  lds_fft<float, E, +1, true>(buf, C, lay.logC, C, 1, d.pm, G(d.twM));
  for (int e = threadIdx.x; e < n; e += blockDim.x) G(d.SIP)[2 * (off + e)] = buf[e];
  GFD_ITEM_END
}

// Row pass, inverse: row m of the two half spectra A (of u_I) and B (of u_p) are combined into
// the full spectrum Z = A + iB (with Z[N-k] = conj A[k] + i conj B[k]); its inverse transform is
// u_I + i u_p.  Columns 0 and N/2 of a real row's spectrum are real: their imaginary parts
// (rounding residue) are dropped.
template <int E>
__global__ void __launch_bounds__(1024) k_row_inv_g(const Img *__restrict__ D, const Item *__restrict__ W, int nitems) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cf *buf = reinterpret_cast<cf *>(smem_raw);
  GFD_ITEM_LOOP
  const Layout &lay = d.L;
  const int M = lay.M, N = lay.N, R = lay.R, Wh = lay.Wh, LP = N + 1;
  const int r0 = wi.blk * R;
  for (int rho = 0; rho < R; ++rho) {
    const int m = r0 + rho;
    if (m >= M) break;
    cf *z = buf + rho * LP;
#pragma unroll 4
    for (int k = threadIdx.x; k < Wh; k += blockDim.x) {
      const size_t g = lay.tpos(m, k);
      cf A = G(d.SIP)[2 * g], B = G(d.SIP)[2 * g + 1];
      if (k == 0 || 2 * k == N) {
        A.im = 0.0f;
        B.im = 0.0f;
      }
      z[k] = cf{A.re - B.im, A.im + B.re};
      if (k > 0 && N - k >= Wh) z[N - k] = cf{A.re + B.im, B.re - A.im};
    }
  }
  __syncthreads();
  lds_fft<float, E, +1, false>(buf, R, 0, 1, LP, d.pn, G(d.twN));
  for (int e = threadIdx.x; e < R * N; e += blockDim.x) {
    const int rho = fdiv(e, lay.Ndiv), nn = e - rho * N;
    const int m = r0 + rho;
    if (m >= M) continue;
    const cf z = buf[rho * LP + nn];
    G(d.uI)[(size_t)m * N + nn] = z.re;
    G(d.uP)[(size_t)m * N + nn] = z.im;
  }
  GFD_ITEM_END
}

// ============================================================================ hot-path kernels, power-of-two lengths
// Register-resident radix-16 transforms (fft_reg.h): two LDS exchanges per transform, first
// and last passes straight from / to global memory.  Threads beyond an image's need (blocks
// sized for a larger image of the batch) only join the barriers.

// The compile-time row transforms and the forward column pass take their twiddles from two
// 64-entry tables in LDS (TwSplit), written here from the image's FP32 table at the block's start into tab[0 .. 128),
// a region no exchange touches; the first pass of a transform needs no twiddles and ends with
// a barrier, which makes the tables visible before they are read.
template <int L>
__device__ __forceinline__ void load_tw_split(cf *tab, const cf *tw) {
  // (entries 64 j with j >= L / 64 are never used: they are read at 64 j mod L, inside the table)
  // One load per thread, written at once, wherever the block has 128 threads (always at
  // L >= 2048, T = L / 16 threads per sequence): a loop here let the compiler defer the write
  // behind the pass's own loads (7-10 us more per pass at 4096, 3 % of the batch).
  if (L >= 2048 || blockDim.x >= 128) {
    if (threadIdx.x < 128) {
      const int j = threadIdx.x & 63;
      tab[threadIdx.x] = E(G(tw), (uint32_t)(threadIdx.x < 64 ? j : (64 * j) & (L - 1)));
    }
  } else {
    // blocks of short rows can have fewer than 128 threads
    for (int i = threadIdx.x; i < 128; i += blockDim.x) {
      const int j = i & 63;
      tab[i] = E(G(tw), (uint32_t)(i < 64 ? j : (64 * j) & (L - 1)));
    }
  }
}

template <int LF>
__global__ void __launch_bounds__(1024) k_row_fwd_r16(const Img *__restrict__ D, const Item *__restrict__ W,
                                                     int nitems, int tw_off) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cf *lds = reinterpret_cast<cf *>(smem_raw);
  if constexpr (LF != 0) {
    if ((int)blockIdx.x < nitems) load_tw_split<LF>(lds + tw_off, D[W[blockIdx.x].img].twN);
  }
  GFD_ITEM_LOOP
  const Layout &lay = d.L;
  const int M = lay.M, N = lay.N, R = lay.Rf, T = d.rn.T;
  const int LP = reg_row_pitch(N);
  const int seq = threadIdx.x / T, t = threadIdx.x - seq * T;
  const bool active = seq < (R >> 1);
  const int r0 = wi.blk * R;
  const int ra = r0 + 2 * seq, rb = ra + 1;
  cf v[16];
  {  // every load is issued (rows clamped into the image), the values are selected afterwards
    const GFD_AS1 float *u = G(d.uE);
    const uint32_t oa = (uint32_t)min(ra, M - 1) * (uint32_t)N + (uint32_t)t;
    const uint32_t ob = (uint32_t)min(rb, M - 1) * (uint32_t)N + (uint32_t)t;
    const bool ua = active && ra < M, ub = active && rb < M;
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const float a = E(u + (size_t)T * m, oa), b = E(u + (size_t)T * m, ob);
      v[m] = cf{ua ? a : 0.0f, ub ? b : 0.0f};
    }
  }
  cf *my = lds + seq * LP;
  if constexpr (LF != 0) reg_fft_c<LF, -1, 1>(v, t, active, my, TwSplit{lds + tw_off, lds + tw_off + 64});
  else reg_fft<-1>(v, t, active, d.rn, my, 1, G(d.twN));
  if (active) {
    cf *w0 = my + lds_pad(t);
    const int st = T + T / 16;  // T is a multiple of 16
#pragma unroll
    for (int m = 0; m < 16; ++m) w0[m * st] = v[m];
  }
  __syncthreads();
  const int C = lay.C, per_t = R * C, Wh = lay.Wh;
  if ((blockDim.x & (per_t - 1)) == 0) {
    // every thread keeps one (row, column-in-tile) pair and walks the tiles
    const int lp = __ffs(per_t) - 1;
    const int rem = threadIdx.x & (per_t - 1);
    const int rho = rem >> lay.logC, c = rem & (C - 1);
    const int m = r0 + rho;
    if (m < M) {
      const int tstep = blockDim.x >> lp, tt0 = threadIdx.x >> lp;
      const cf *z = lds + (rho >> 1) * LP;
      const bool odd = (rho & 1) != 0;
      const uint32_t ostep = (uint32_t)tstep * (uint32_t)lay.TS;
      uint32_t o = (uint32_t)tt0 * (uint32_t)lay.TS + (uint32_t)m * (uint32_t)C + (uint32_t)c;
      for (int tt = tt0; tt < lay.NT; tt += tstep, o += ostep) {
        const int k = tt * C + c;
        cf X = {0.0f, 0.0f};
        if (k < Wh) {
          const cf Zk = z[lds_pad(k)], Zn = z[lds_pad(k == 0 ? 0 : N - k)];
          X = odd ? cf{(Zk.im + Zn.im) * 0.5f, (Zn.re - Zk.re) * 0.5f}
                  : cf{(Zk.re + Zn.re) * 0.5f, (Zk.im - Zn.im) * 0.5f};
        }
        E(G(d.S1), o) = X;
      }
    }
  } else {
    const int total = lay.NT * per_t;
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
      const int tt = fdiv(e, lay.RfCdiv), rem = e - tt * per_t;
      const int rho = rem >> lay.logC, c = rem & (C - 1);
      const int m = r0 + rho;
      if (m >= M) continue;
      const int k = tt * C + c;
      cf X = {0.0f, 0.0f};
      if (k < Wh) {
        const cf *z = lds + (rho >> 1) * LP;
        const cf Zk = z[lds_pad(k)], Zn = z[lds_pad(k == 0 ? 0 : N - k)];
        if ((rho & 1) == 0) X = cf{(Zk.re + Zn.re) * 0.5f, (Zk.im - Zn.im) * 0.5f};
        else X = cf{(Zk.im + Zn.im) * 0.5f, (Zn.re - Zk.re) * 0.5f};
      }
      G(d.S1)[(size_t)tt * lay.TS + (size_t)m * C + c] = X;
    }
  }
  GFD_ITEM_END
}

// With RESID and Layout::fold the block of tile 0 also transforms column N/2 (column 0 of the
// last tile, which then has no block): after the row transforms columns 0 and N/2 are real, so
// column N/2 rides in the imaginary part of column 0 and the two are separated after the
// transform by the symmetry of real-input transforms, F(x)[-k] = conj F(x)[k].  Its residual
// and first-round terms are added to the block's partial sums.
template <bool RESID, int LF>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4, 8))) k_col_fwd_r16(const Img *__restrict__ D, const Item *__restrict__ W,
                                                     int nitems, int tw_off) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cf *lds = reinterpret_cast<cf *>(smem_raw);
  __shared__ float scratch[kLamAcc * 16];
  if constexpr (LF != 0) {
    if ((int)blockIdx.x < nitems) load_tw_split<LF>(lds + tw_off, D[W[blockIdx.x].img].twM);
  }
  GFD_ITEM_LOOP
  const Layout &lay = d.L;
  const int C = lay.C, T = d.rm.T;
  const int c = threadIdx.x & (C - 1), t = threadIdx.x >> lay.logC;
  const bool active = t < T;
  // element m of this thread's column sits at byte to + sm * m of the tile: sm * m is the same
  // for the whole block, to a 32-bit per-thread offset (inactive threads read a valid element
  // and never use it)
  const size_t tb = (size_t)wi.blk * lay.TS, tbN = (size_t)(lay.NT - 1) * lay.TS;
  const uint32_t sm = (uint32_t)(T * C * sizeof(cf));
  const uint32_t to = (uint32_t)(((active ? t : 0) * C + c) * sizeof(cf));
  const auto rS = gbytes(d.S1 + tb);
  const bool fold = RESID && lay.fold && wi.blk == 0;  // uniform over the block
  const bool fc = fold && c == 0 && active;
  cf v[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) v[m] = ld_cf(rS, to, sm * m);
  if (fc) {  // column N/2 (real) as the imaginary part of column 0 (real)
    const auto rN = gbytes(d.S1 + tbN);
#pragma unroll
    for (int m = 0; m < 16; ++m) v[m].im = ld_f(rN, to, sm * m);
  }
  if constexpr (LF != 0) reg_fft_c<LF, -1, col_ls(LF), false>(v, t, active, lds + c, TwSplit{lds + tw_off, lds + tw_off + 64});
  else reg_fft<-1>(v, t, active, d.rm, lds + c, C, G(d.twM));
  if (!RESID) {
    if (active) {
#pragma unroll
      for (int m = 0; m < 16; ++m) st_cf(v[m], rS, to, sm * m);
    }
  } else {
    cf *zB = lds + lay.M;  // column N/2 after the separation (the exchange area is free now)
    if (fold) {
      cf *zA = lds;
      if (fc) {
#pragma unroll
        for (int m = 0; m < 16; ++m) zA[t + T * m] = v[m];
      }
      __syncthreads();
      if (fc) {
#pragma unroll
        for (int m = 0; m < 16; ++m) {
          const int row = t + T * m;
          const cf zm = zA[(lay.M - row) & (lay.M - 1)];  // Z[-k]
          const cf d = cf{v[m].re - zm.re, v[m].im + zm.im};  // Z[k] - conj Z[-k] = 2i F(x_N/2)[k]
          v[m] = cf{0.5f * (v[m].re + zm.re), 0.5f * (v[m].im - zm.im)};
          zB[row] = cf{0.5f * d.im, -0.5f * d.re};
        }
      }
    }
    constexpr int NC = kLamFirstCand;
    float mu[NC];
#pragma unroll
    for (int j = 0; j < NC; ++j) mu[j] = d.st->mu[j];
    float acc[2 + 2 * NC];
#pragma unroll
    for (int a = 0; a < 2 + 2 * NC; ++a) acc[a] = 0.0f;
    const int k = wi.blk * C + c;
    const bool valid = active && k < lay.Wh;
    const float wgt = (k == 0 || 2 * k == lay.N) ? 1.0f : 2.0f;
    __builtin_amdgcn_sched_barrier(0);  // H and Y are not loaded before the transform is done
    // R = H U_E - Y, q = w |R|^2 and the first-round terms of a column of one tile, in two
    // halves of eight bins: the 16 loads of a half are in flight together, and each bin's U_E
    // and q are stored as soon as q is known (padding columns hold zeros in H and Y, so they
    // are loaded like the others)
    auto residual = [&](size_t tile, auto value, float w, bool ok) {
      const auto rU = gbytes(d.S1 + tile), rH = gbytes(d.H + tile), rY = gbytes(d.Y + tile), rq = gbytes(d.q + tile);
#pragma unroll
      for (int h0 = 0; h0 < 16; h0 += 8) {
        cf hv[8], yv[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          hv[i] = ld_cf(rH, to, sm * (h0 + i));
          yv[i] = ld_cf(rY, to, sm * (h0 + i));
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int m = h0 + i;
          const cf u = value(m);
          const cf r = cmul(hv[i], u) - yv[i];
          const float qq = ok ? w * abs2f(r) : 0.0f;
          st_cf(u, rU, to, sm * m);
          st_f(qq, rq, to / 2, sm / 2 * m);
          first_round_terms<NC>(qq, abs2f(hv[i]), mu, acc);
        }
      }
    };
    if (active) residual(tb, [&](int m) { return v[m]; }, wgt, valid);
    if (fc) residual(tbN, [&](int m) { return zB[t + T * m]; }, 1.0f, true);
    float h, l;
    block_sum_plain_then_df<2 + 2 * NC>(acc, h, l, scratch);
    store_partial(G(d.part), d.npart, wi.blk, 2 + 2 * NC, h, l);
    if (wi.blk == 0 && threadIdx.x == 0) lam_open(d.st);
  }
  GFD_ITEM_END
}

// With Layout::fold the block of tile 0 also solves column N/2 (column 0 of the last tile,
// which no block owns) and transforms it as the imaginary part of column 0: both solved columns
// are Hermitian, so their inverse transforms are real and the real and imaginary parts of the
// one transform are the two columns.  The folded column is solved first and parked in LDS, so
// that it adds no registers to the main solve.
template <int LF>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4, 8))) k_col_inv_r16(const Img *__restrict__ D, const Item *__restrict__ W,
                                                     int nitems) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cf *lds = reinterpret_cast<cf *>(smem_raw);
  GFD_ITEM_LOOP
  const Layout &lay = d.L;
  const int C = lay.C, T = d.rm.T;
  const int c = threadIdx.x & (C - 1), t = threadIdx.x >> lay.logC;
  const bool active = t < T;
  const size_t off = (size_t)wi.blk * lay.TS;
  const SolveParams sp = solve_params(d.st);
  const int k = wi.blk * C + c;
  const bool valid = active && k < lay.Wh;
  const float dk = valid ? G(d.dN)[k] : 0.0f;
  const bool fold = lay.fold && wi.blk == 0;  // uniform over the block
  const bool fc = fold && c == 0 && active;
  if (fc) {  // column N/2, parked in LDS (free until the transforms)
    const size_t offN = (size_t)(lay.NT - 1) * lay.TS;
    const float dN2 = G(d.dN)[lay.N / 2];
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const int row = t + T * m;
      const size_t e = offN + (size_t)row * C;
      cf Up, Ui;
      solve_bin(sp, G(d.S1)[e], G(d.HY)[e], G(d.H2)[e], G(d.dM)[row] + dN2, Up, Ui);
      lds[row] = Up;
      lds[lay.M + row] = Ui;
    }
  }
  // all loads first (no store in between), then the solves
  // Straight-line rows (the solve's case split is taken once, outside the loop; padding columns
  // are computed and then zeroed; the means are written after the loop), so the compiler can
  // issue the loads of later rows ahead of the arithmetic of earlier ones.
  cf vp[16], vi[16];
  // element m of this thread's column: element to + sm * m of the tile (sm * m the same for the
  // whole block, to a 32-bit per-thread offset)
  const uint32_t sm = (uint32_t)(T * C), to = (uint32_t)(t * C + c);
  const auto rS = gbytes(d.S1 + off), rHY = gbytes(d.HY + off);
  const auto rH2 = gbytes(d.H2 + off), rdM = gbytes(d.dM);
  auto rows = [&](auto mode) {
    constexpr int MODE = decltype(mode)::value;
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      cf Up, Ui;
      solve_bin_mode<MODE>(sp, ld_cf(rS, 8 * to, 8 * sm * m), ld_cf(rHY, 8 * to, 8 * sm * m),
                           ld_f(rH2, 4 * to, 4 * sm * m), ld_f(rdM, 4 * (uint32_t)t, 4 * (uint32_t)(T * m)) + dk,
                           Up, Ui);
      vp[m] = valid ? Up : cf{0.0f, 0.0f};
      vi[m] = valid ? Ui : cf{0.0f, 0.0f};
      // two groups of eight rows: the second group's loads are issued after the first group's
      // solves, which bounds the loaded operands held in registers
      if (m == 7) __builtin_amdgcn_sched_barrier(0);
    }
  };
  if (!active) {
#pragma unroll
    for (int m = 0; m < 16; ++m) vp[m] = vi[m] = cf{0.0f, 0.0f};
  } else if (sp.inf_branch) {
    rows(std::integral_constant<int, 0>{});
  } else if (sp.big) {
    rows(std::integral_constant<int, 1>{});
  } else {
    rows(std::integral_constant<int, 2>{});
  }
  if (valid && k == 0 && t == 0) {  // zero frequency (row 0, column 0): the means of u_p and u_I
    d.st->meanP = vp[0].re;
    d.st->meanI = vi[0].re;
  }
  if (fold) {
    if (fc) {  // U_0 + i U_N
#pragma unroll
      for (int m = 0; m < 16; ++m) {
        const cf np = lds[t + T * m], ni = lds[lay.M + t + T * m];
        vp[m] = cf{vp[m].re - np.im, vp[m].im + np.re};
        vi[m] = cf{vi[m].re - ni.im, vi[m].im + ni.re};
      }
    }
    __syncthreads();  // the parked column is read before the transforms use the LDS
  }
  // both transforms, then one 16-byte store per bin (U_I, U_p): the two columns of the tile give
  // 32 contiguous bytes per row
  if constexpr (LF != 0) {
    // (twiddles from the butterfly-major global table: the two products per twiddle of the LDS
    // tables, or an index per twiddle into the plain table, cost this kernel's register budget
    // more than the loads' latency)
    reg_fft_c<LF, +1, col_ls(LF), false>(vp, t, active, lds + c, TwTable{G(d.twB)});
    // the second transform loads its twiddles again: an opaque copy of the table pointer keeps
    // the compiler from holding the first transform's twiddles in registers across both
    const cf *tw2 = d.twB;
    asm volatile("" : "+s"(tw2));
    reg_fft_c<LF, +1, col_ls(LF), false>(vi, t, active, lds + c, TwTable{G(tw2)});
  } else {
    reg_fft<+1>(vp, t, active, d.rm, lds + c, C, G(d.twM));
    reg_fft<+1>(vi, t, active, d.rm, lds + c, C, G(d.twM));
  }
  if (active) {
    // the solved spectra are tile-major like the inputs: the bins of this thread sit at the
    // same elements to + sm * m of the tile, and a wave's 16-byte stores are contiguous
    const auto rO = gbytes(reinterpret_cast<float4 *>(d.SIP) + off);
    if (fc) {  // real parts: column 0 (this tile); imaginary parts: column N/2 (column 0 of the last tile)
      const auto rN = gbytes(reinterpret_cast<float4 *>(d.SIP) + (size_t)(lay.NT - 1) * lay.TS);
#pragma unroll
      for (int m = 0; m < 16; ++m) {
        st_f4(vi[m].re, 0.0f, vp[m].re, 0.0f, rO, 16 * to, 16 * sm * m);
        st_f4(vi[m].im, 0.0f, vp[m].im, 0.0f, rN, 16 * to, 16 * sm * m);
      }
    } else {
#pragma unroll
      for (int m = 0; m < 16; ++m) st_f4(vi[m].re, vi[m].im, vp[m].re, vp[m].im, rO, 16 * to, 16 * sm * m);
    }
  }
  GFD_ITEM_END
}

// Row pass, inverse; the Hermitian completion is gathered straight from the tile-major spectra.
template <int LF>
__global__ void __launch_bounds__(1024) k_row_inv_r16(const Img *__restrict__ D, const Item *__restrict__ W,
                                                     int nitems, int tw_off) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cf *lds = reinterpret_cast<cf *>(smem_raw);
  if constexpr (LF != 0) {
    if ((int)blockIdx.x < nitems) load_tw_split<LF>(lds + tw_off, D[W[blockIdx.x].img].twN);
  }
  GFD_ITEM_LOOP
  const Layout &lay = d.L;
  const int M = lay.M, N = lay.N, Wh = lay.Wh, T = d.rn.T;
  const int LP = reg_row_pitch(N);
  const int seq = threadIdx.x / T, t = threadIdx.x - seq * T;
  const bool active = seq < lay.Ri;
  const int row = wi.blk * lay.Ri + seq;
  cf v[16];
  {
    // The block's Ri rows are gathered together: in every tile they are Ri C consecutive 16-byte
    // words (bins of Ri rows, C columns), so each word is loaded once (a row's bins k and N - k
    // share one) in runs of Ri C words, and staged in LDS (rows past the end load a copy of the
    // last row, never stored); then every thread picks its bins with the Hermitian completion.
    // The staging memory is the transform's exchange area, free until the transform.
    const int Ri = lay.Ri, C = lay.C, logC = lay.logC;
    const int per = Ri << logC, lper = __ffs(per) - 1;  // words per tile (a power of two)
    // SP: staged row pitch in words, with SP = 8 / Ri (mod 8) so that the eight words one LDS
    // cycle writes (8 / Ri consecutive words of each of the Ri rows) cover the banks once
    const int want = Ri <= 8 ? (8 / Ri) & 7 : 0;
    const int total = lay.NT * per, SP = lay.RP + ((want - lay.RP) & 7);
    float4 *stage = reinterpret_cast<float4 *>(smem_raw);
    const GFD_AS1 float4 *sip = reinterpret_cast<const GFD_AS1 float4 *>(G(d.SIP));
    const int r0 = wi.blk * Ri;
    // kU words per thread in one batch of loads (with 8 a second batch waited a whole memory
    // latency for the few words of the last tile; indices past the end repeat the last word)
    constexpr int kU = 9;
    for (int e0 = threadIdx.x; e0 < total; e0 += kU * blockDim.x) {
      float4 w[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {  // loads first: they are in flight together
        const int e = min(e0 + u * (int)blockDim.x, total - 1);
        const int tile = e >> lper, rem = e & (per - 1);
        const uint32_t m = (uint32_t)min(r0 + (rem >> logC), M - 1);
        w[u] = E(sip, (uint32_t)tile * (uint32_t)lay.TS + m * (uint32_t)C + (uint32_t)(rem & (C - 1)));
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int e = e0 + u * (int)blockDim.x;
        if (e < total) {
          const int tile = e >> lper, rem = e & (per - 1);
          stage[(rem >> logC) * SP + (tile << logC) + (rem & (C - 1))] = w[u];
        }
      }
    }
    __syncthreads();
    if (active) {
      const float4 *my = stage + seq * SP;
#pragma unroll
      for (int m = 0; m < 16; ++m) {
        const int n = t + T * m;
        const bool direct = n < Wh;
        const int kk = direct ? n : N - n;
        const float4 ab = my[kk];
        const bool real_col = kk == 0 || 2 * kk == N;
        const float ai = real_col ? 0.0f : ab.y, bi = real_col ? 0.0f : ab.w;
        v[m] = direct ? cf{ab.x - bi, ai + ab.z} : cf{ab.x + bi, ab.z - ai};
      }
    }
    __syncthreads();  // the staged words are read before the transform writes the LDS
  }
  if constexpr (LF != 0) reg_fft_c<LF, +1, 1>(v, t, active, lds + seq * LP, TwSplit{lds + tw_off, lds + tw_off + 64});
  else reg_fft<+1>(v, t, active, d.rn, lds + seq * LP, 1, G(d.twN));
  if (active && row < M) {
    const uint32_t g0 = (uint32_t)row * (uint32_t)N + (uint32_t)t;
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      E(G(d.uI) + (size_t)T * m, g0) = v[m].re;
      E(G(d.uP) + (size_t)T * m, g0) = v[m].im;
    }
  }
  GFD_ITEM_END
}

// ============================================================================ lambda search kernels
// The search kernels work on a private copy of the image's state (one thread) and write it
// back, so that the serial search code does not wait on memory at every field access.
// `stv` is the array of the states of the set's images (index = image), read first so that an
// image whose lambda is already fixed skips the round after one load.

// The lambda search after the residual pass, for every image of the launch, as one work queue.
// Entries 0 .. nimg-1 start the images' searches (reduce the residual pass's per-tile partial
// sums, then lam_begin on one thread); a start that leaves the search open appends its image to
// the queue's open list.  The entries after them are the evaluation rounds of the open images
// only, round-major: entry nimg + q is round q / S, chunk q % S of the open images' chunks laid
// end to end (S chunks per round).  A block takes entries in queue order.  Before a round entry
// it waits until every start is done (the open list is then final), and before a chunk of round
// r it waits until the image's round r has been published (by the start for r = 0, by the fold
// of round r - 1 after that) or its lambda fixed.  The waits cannot deadlock: every entry a
// block waits on was taken earlier by a block that is running, and those finish without waiting
// on later entries.  Per chunk: sums of q g_j and q g_j (1 - r_j) over its bins; the image's last
// block to store a round's sums (the count in the image's state, fenced on both sides) folds the
// round into the bracket.  An open search's state is stored first and published after a fence
// (round r + 1); a fixed lambda is published as phase = 1 without one (lam_publish).  Blocks leave when their entry is past the last round
// or every image's lambda is fixed; the last to leave clears the queue for the next launch.
// A single image skips the start entry: every block reduces the partials and runs the start
// itself (the same sums in the same order give the same decision in every block), so no block
// waits for another to start the search.  When the first round decides, block 0 commits lambda
// and no block touches the queue; otherwise each block evaluates round 0 with its own copy of the
// start's candidates, and the fold of round 0 starts from the folding block's copy.
constexpr int kLamSpinLimit = 1 << 20;  // bounded wait (about 50 ms); never reached in practice
constexpr int kLamOpenLds = 4096;       // open images a block can map (every image of a batch)

// A fixed lambda is read only by later launches (the launch boundary orders those reads); the
// blocks of this launch only learn that the image is closed (its phase, the closed count) and
// read nothing else of its state, so that path has no fence.  A fence is a write-back of the
// L2's dirty lines, which after the residual pass costs microseconds.  An open search's state
// (the next candidates) is read by the blocks of the next round: it is fenced before the round
// is published.
__device__ __forceinline__ void lam_publish(LamState *sp, LamState &st, int fixed, int next_round, LamQueue *lq) {
  st.round = next_round - 1;
  if (fixed) {
    st.phase = 1;  // the plain copy and the flag agree, whichever reaches memory first
    *sp = st;
    __hip_atomic_store(&sp->phase, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    atomicAdd(&lq->closed, 1);
  } else {
    st.phase = 0;
    *sp = st;
    __threadfence();
    __hip_atomic_store(&sp->round, next_round, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__device__ __forceinline__ int ld_agent(const int *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void __launch_bounds__(512) k_lam_rounds(const Img *__restrict__ D, const Item *__restrict__ W1, int nimg,
                                                    LamState *stv, LamQueue *lq, int rounds, int advance) {
  __shared__ float scratch[kLamAcc * 8];
  __shared__ int s_item, s_go, is_last, s_fixed, s_img, s_chunk, s_nopen, s_S;
  __shared__ float s_mu[kLamMaxCand], s_mu0[kLamMaxCand];
  __shared__ LamState sst;  // single image: this block's copy of the start of the search
  __shared__ int s_open[kLamOpenLds], s_pre[kLamOpenLds + 1];  // open images, prefix sums of their chunks
  constexpr int NC = kLamMaxCand, NC1 = kLamFirstCand;
  const bool single = nimg == 1;
  if (threadIdx.x == 0) s_nopen = -1;  // open list not read yet
  if (single) {
    const Item w0 = W1[0];
    const Img &d = D[w0.img];
    // thread 0 loads the state before the reduction, so that the load's latency overlaps it
    LamState st;
    if (threadIdx.x == 0) st = stv[w0.img];
    float hi[2 + 2 * NC1], lo[2 + 2 * NC1];
    reduce_partials<2 + 2 * NC1, 16>(G(d.part), d.npart, d.L.col_blocks(), hi, lo, scratch);
    if (threadIdx.x == 0) {
      st.done = 0;
      st.flags = 0;
      float cand[NC1];
      for (int j = 0; j < NC1; ++j) cand[j] = st.cand[j];
      const int fixed = lam_begin(st, hi[0], lo[0], hi[1], lo[1], NC1, cand, hi + 2, lo + 2, hi + 2 + NC1);
      if (fixed) {
        if (blockIdx.x == 0) {
          lam_commit(d, st, advance);
          stv[w0.img] = st;
        }
      } else {
        for (int j = 0; j < NC; ++j) s_mu0[j] = st.mu[j];
        sst = st;
        s_open[0] = w0.img;
        s_pre[0] = 0;
        s_pre[1] = d.nchunk;
        s_nopen = 1;
        s_S = d.nchunk;
      }
      s_fixed = fixed;
    }
    __syncthreads();
    if (s_fixed) return;  // uniform (and the same in every block)
  }
  for (;;) {
    if (threadIdx.x == 0) s_item = ld_agent(&lq->closed) < nimg ? atomicAdd(&lq->next, 1) : -1;
    __syncthreads();
    const int qi = s_item;
    if (qi < 0) break;  // uniform: every image's lambda is fixed
    if (qi < nimg) {    // start of an image's search: the first round was evaluated in the residual pass
      if (single) continue;  // every block started the search itself
      const Item wi = W1[qi];
      const Img &d = D[wi.img];
      float hi[2 + 2 * NC1], lo[2 + 2 * NC1];
      // (one batch of 16 partials per lane and value: one memory round trip per value)
      reduce_partials<2 + 2 * NC1, 16>(G(d.part), d.npart, d.L.col_blocks(), hi, lo, scratch);
      if (threadIdx.x == 0) {
        // the serial search works on a copy in registers
        LamState st = stv[wi.img];
        st.done = 0;
        st.flags = 0;
        float cand[NC1];
        for (int j = 0; j < NC1; ++j) cand[j] = st.cand[j];
        const int fixed = lam_begin(st, hi[0], lo[0], hi[1], lo[1], NC1, cand, hi + 2, lo + 2, hi + 2 + NC1);
        if (fixed) lam_commit(d, st, advance);
        lam_publish(stv + wi.img, st, fixed, 0, lq);
        if (!fixed) {  // the open list entry is read once the starts are counted
          __hip_atomic_store(&lq->open[atomicAdd(&lq->nopen, 1)], wi.img, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __threadfence();
        }
        atomicAdd(&lq->begun, 1);
      }
      __syncthreads();
      continue;
    }
    if (s_nopen < 0) {  // first round entry of this block: the final open list (uniform)
      if (threadIdx.x == 0) {
        for (int spin = 0; ld_agent(&lq->begun) < nimg; ++spin) {
          if (spin >= kLamSpinLimit) break;  // (the list below then covers the starts done so far)
          __builtin_amdgcn_s_sleep(2);
        }
        __threadfence();
        s_nopen = min(ld_agent(&lq->nopen), kLamOpenLds);
      }
      __syncthreads();
      for (int k = threadIdx.x; k < s_nopen; k += blockDim.x) {
        const int img = ld_agent(&lq->open[k]);
        s_open[k] = img;
        s_pre[k + 1] = D[img].nchunk;
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        s_pre[0] = 0;
        for (int k = 0; k < s_nopen; ++k) s_pre[k + 1] += s_pre[k];
        s_S = s_pre[s_nopen];
      }
      __syncthreads();
    }
    const int q = qi - nimg, S = s_S;
    if (q >= rounds * S) break;  // uniform: past the last round
    const int r = q / S, rem = q - r * S;
    if (threadIdx.x == 0) {  // the open image and chunk of this entry
      int lo = 0, hi = s_nopen - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_pre[mid] <= rem) lo = mid;
        else hi = mid - 1;
      }
      s_img = s_open[lo];
      s_chunk = rem - s_pre[lo];
      int go = 0;
      if (single && r == 0) {  // round 0 of a single image: this block's own candidates
        go = 1;
        for (int j = 0; j < NC; ++j) s_mu[j] = s_mu0[j];
      } else {
        LamState *sp = stv + s_img;
        for (int spin = 0;; ++spin) {
          if (ld_agent(&sp->phase) != 0) break;
          if (ld_agent(&sp->round) >= r) {
            go = 1;
            break;
          }
          if (spin >= kLamSpinLimit) {
            atomicOr(&sp->flags_all, (unsigned)kFlagUnconverged);
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
        if (go) {
          __threadfence();
#pragma unroll
          for (int j = 0; j < NC; ++j) s_mu[j] = __hip_atomic_load(&sp->mu[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      s_go = go;
    }
    __syncthreads();
    if (!s_go) continue;  // uniform
    const int img = s_img, blk = s_chunk;
    const Img &d = D[img];
    float mu[NC];
#pragma unroll
    for (int j = 0; j < NC; ++j) mu[j] = s_mu[j];
    float acc[2 * NC];
#pragma unroll
    for (int v = 0; v < 2 * NC; ++v) acc[v] = 0.0f;
    const size_t nbins = d.L.bins(), n4 = nbins / 4;
    const GFD_AS1 float4 *q4 = reinterpret_cast<const GFD_AS1 float4 *>(G(d.q));
    const GFD_AS1 float4 *h4 = reinterpret_cast<const GFD_AS1 float4 *>(G(d.H2));
    for (size_t i = (size_t)blk * blockDim.x + threadIdx.x; i < n4; i += (size_t)d.nchunk * blockDim.x) {
      const float4 qa = q4[i], ta = h4[i];
      const float qs[4] = {qa.x, qa.y, qa.z, qa.w}, ts[4] = {ta.x, ta.y, ta.z, ta.w};
#pragma unroll
      for (int u = 0; u < 4; ++u) {
#pragma unroll
        for (int j = 0; j < NC; ++j) {
          const float rr = __builtin_amdgcn_rcpf(__fmaf_rn(ts[u], mu[j], 1.0f));
          const float qg = qs[u] * (rr * rr);
          acc[j] += qg;
          acc[NC + j] = __fmaf_rn(qg, 1.0f - rr, acc[NC + j]);
        }
      }
    }
    if (blk == 0) {  // bins that do not fill a float4
      for (size_t i = n4 * 4 + threadIdx.x; i < nbins; i += blockDim.x) {
#pragma unroll
        for (int j = 0; j < NC; ++j) {
          const float rr = __builtin_amdgcn_rcpf(__fmaf_rn(G(d.H2)[i], mu[j], 1.0f));
          const float qg = G(d.q)[i] * (rr * rr);
          acc[j] += qg;
          acc[NC + j] = __fmaf_rn(qg, 1.0f - rr, acc[NC + j]);
        }
      }
    }
    float h, l;
    block_sum_plain_then_df<2 * NC>(acc, h, l, scratch);
    store_partial(G(d.part), d.npart, blk, 2 * NC, h, l);
    // the partial sums are stored by lanes of wave 0 (2 NC < 64), which also takes the count
    static_assert(2 * NC <= 64, "partials stored by the first wave");
    if (threadIdx.x < 64) __threadfence();
    if (threadIdx.x == 0) is_last = atomicAdd(&stv[img].done, 1) == d.nchunk - 1;
    __syncthreads();
    if (is_last) {  // uniform over the block
      __threadfence();
      float hi[2 * NC], lo[2 * NC];
      // (at most 512 chunks: one batch of 8 per lane and value)
      reduce_partials<2 * NC, 8>(G(d.part), d.npart, d.nchunk, hi, lo, scratch);
      if (threadIdx.x == 0) {
        LamState st = (single && r == 0) ? sst : stv[img];
        float cand[NC];
        for (int j = 0; j < NC; ++j) cand[j] = st.cand[j];
        lam_absorb(st, NC, cand, hi, lo, hi + NC);
        const int fixed = lam_decide(st, r == rounds - 1);
        if (fixed) lam_commit(d, st, advance);
        st.done = 0;
        lam_publish(stv + img, st, fixed, r + 1, lq);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && atomicAdd(&lq->exits, 1) == (int)gridDim.x - 1) {
    __hip_atomic_store(&lq->next, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&lq->closed, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&lq->begun, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&lq->nopen, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&lq->exits, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ============================================================================ set-up kernels (one image)
template <class T, class TI, int E>
__global__ void __launch_bounds__(1024) k_row_fwd_plain(const TI *__restrict__ x, Layout lay, FftPlan pn,
                                                        const cpx<T> *__restrict__ tw, cpx<T> *__restrict__ S) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  row_fwd_body<T, E>(G(x), lay, pn, G(tw), G(S), blockIdx.x, reinterpret_cast<cpx<T> *>(smem_raw));
}

template <class T, int E>
__global__ void __launch_bounds__(1024) k_col_fwd_plain(cpx<T> *__restrict__ S, Layout lay, FftPlan pm,
                                                        const cpx<T> *__restrict__ tw) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T> *buf = reinterpret_cast<cpx<T> *>(smem_raw);
  const int n = lay.M * lay.C;
  GFD_AS1 cpx<T> *tile = G(S) + (size_t)blockIdx.x * lay.TS;
  col_fwd_load_fft<T, E>(tile, lay, pm, G(tw), buf);
  for (int e = threadIdx.x; e < n; e += blockDim.x) tile[e] = buf[e];
}

// Periodic embedding: entry (i, j) of the centred kh x kw PSF goes to ((i - kh/2) mod M,
// (j - kw/2) mod N).  With kh <= M and kw <= N the targets are distinct, so the scatter
// needs no atomics; the array is cleared first.
__global__ void k_fill_d(double *p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0.0;
}
__global__ void k_embed_psf(const float *__restrict__ h, int kh, int kw, int M, int N, double *__restrict__ hp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kh * kw) return;
  const int a = i / kw, b = i - a * kw;
  const int m = ((a - kh / 2) % M + M) % M, n = ((b - kw / 2) % N + N) % N;
  hp[(size_t)m * N + n] = (double)h[i];
}

// Constants of the solves in FP32, derived in FP64: H, Y (residual), conj(H) Y and |H|^2
// (solves and search).  |H|^2 uses the same FP32 expression as the residual pass.
__global__ void k_init_consts(const cd *__restrict__ Hd, const cd *__restrict__ Yd, size_t n, int Wh, int M, int C,
                              int TS, cf *__restrict__ H, cf *__restrict__ Y, cf *__restrict__ HY,
                              float *__restrict__ H2) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const size_t t = i / (size_t)TS, rem = i - t * TS;
    const int c = (int)(rem & (size_t)(C - 1));
    // bins past a tile's M x C block (padding) and columns at or beyond Wh hold zeros
    const bool valid = rem < (size_t)M * C && (int)(t * C) + c < Wh;
    const cd h = valid ? Hd[i] : cd{0.0, 0.0}, y = valid ? Yd[i] : cd{0.0, 0.0};
    const cf hf = {(float)h.re, (float)h.im};
    H[i] = hf;
    Y[i] = cf{(float)y.re, (float)y.im};
    HY[i] = cf{(float)(h.re * y.re + h.im * y.im), (float)(h.re * y.im - h.im * y.re)};
    H2[i] = abs2f(hf);
  }
}

// D2[m, k] = dM[m] + dN[k] with dM[m] = 4 sin^2(pi m / M), dN[k] = 4 sin^2(pi k / N): the
// symbol |F(d_x)|^2 + |F(d_y)|^2 of periodic forward differences (reading of Sec. 3.1).
__global__ void k_d2_tables(int M, int N, int Wh, float *dM, float *dN) {
  const double pi = 3.14159265358979323846;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < M + Wh; i += gridDim.x * blockDim.x) {
    if (i < M) {
      double s = sin(pi * i / M);
      dM[i] = (float)(4.0 * s * s);
    } else {
      int k = i - M;
      double s = sin(pi * k / N);
      dN[k] = (float)(4.0 * s * s);
    }
  }
}

// FP64 sums over y for Eq.(12): per-block sums of y and y^2, then of (y - mean)^2.
__global__ void k_ysums(const float *__restrict__ y, size_t n, double *__restrict__ part) {
  __shared__ double sh[2][256];
  double s1 = 0.0, s2 = 0.0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    double v = y[i];
    s1 += v;
    s2 += v * v;
  }
  sh[0][threadIdx.x] = s1;
  sh[1][threadIdx.x] = s2;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + o];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sh[0][0];
    part[2 * blockIdx.x + 1] = sh[1][0];
  }
}

__global__ void k_ycentred(const float *__restrict__ y, size_t n, const double *__restrict__ part, int nparts,
                           double *__restrict__ part2) {
  __shared__ double sh[256];
  __shared__ double mean;
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int p = 0; p < nparts; ++p) s += part[2 * p];
    mean = s / (double)n;
  }
  __syncthreads();
  double s = 0.0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    double dd = (double)y[i] - mean;
    s += dd * dd;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part2[blockIdx.x] = sh[0];
}

// rho of Eq.(12) (radicand clipped to [1e-12, 1]) unless fixed, target T = rho P sigma^2 over
// the n observed pixels, and the constants of the search state, whose Parseval factors use the
// ndom pixels of the transform domain (ndom = n unless the observation was padded).
__global__ void k_rho_final(const double *__restrict__ part, const double *__restrict__ part2, int nparts,
                            const float *__restrict__ h, int nh, size_t n, size_t ndom, double sigma2,
                            double rho_fixed, double *out2, LamState *st) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double sy2 = 0.0, sc = 0.0, h1 = 0.0;
  for (int p = 0; p < nparts; ++p) {
    sy2 += part[2 * p + 1];
    sc += part2[p];
  }
  for (int i = 0; i < nh; ++i) h1 += fabs((double)h[i]);
  const double P = (double)n;
  double rho = rho_fixed;
  if (!(rho_fixed > 0.0)) {
    double rad = 1.0 - (sc - P * sigma2) / (h1 * h1 * sy2);
    rad = fmin(fmax(rad, 1e-12), 1.0);
    rho = sqrt(rad);
  }
  const double T = rho * P * sigma2;
  out2[0] = rho;
  out2[1] = T;
  st->TP = (float)(T * (double)ndom);
  st->invP = (float)(1.0 / (double)ndom);
}

__global__ void k_fill_f(float *p, size_t n, float v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

// Fresh iteration state (keeps the image constants TP, invP and the scale count).
__global__ void k_state_reset(LamState *st) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  st->k = 0;
  st->phase = 0;
  st->flags = 0;
  st->flags_all = 0;
  st->rounds = 0;
  st->Einf = 0.0f;
  st->lam_star = 0.0f;
  st->lam = 0.0f;
  st->lam_prev = 0.0f;
  st->lam_prev2 = 0.0f;
  st->meanI = 0.0f;
  st->meanP = 0.0f;
  st->done = 0;
  st->round = -1;
  lam_first_candidates(*st);
}

__global__ void k_state_set_lam(LamState *st, float lam) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  st->lam = lam;
}

__global__ void k_state_set_nscale(LamState *st, int count, int ns) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) st[i].nscale = ns;
}

__global__ void k_copy_lam_star(const LamState *st, float *out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  out[0] = st->lam_star;
}

// ============================================================================ host side
static int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

static FastDiv mkdiv(int d) {
  FastDiv f;
  f.d = d;
  f.inv = 1.0f / (float)d;
  return f;
}

// Padding bins after every tile of a power-of-two-rich size (a multiple of 16, so that float4
// runs over the bins stay aligned in every tile).
constexpr int kTilePad = 64;

Layout make_layout(int M, int N, const Tuning &tune) {
  Layout L;
  L.M = M;
  L.N = N;
  L.Wh = N / 2 + 1;
  // tile width: the column pass keeps M x C complex values in LDS (<= 64 KiB)
  int C = 1;
  while (C < 16 && (size_t)M * (C * 2) * 8 <= 64 * 1024) C *= 2;
  while (C > 1 && C / 2 >= L.Wh) C /= 2;
  L.C = C;
  L.logC = ilog2(C);
  L.NT = (L.Wh + C - 1) / C;
  L.RP = L.NT * C;
  // tile stride: M * C bins, plus kTilePad where M * C is a multiple of 1024 (a tile of 16 KiB
  // or more of FP32 bins at a power-of-two-rich stride)
  L.TS = M * C + ((M * C) % 1024 == 0 ? kTilePad : 0);
  // (the folded passes also use 2 M complex values of the block's LDS, which C >= 2 provides)
  L.fold = (reg_plan_ok(M) && C >= 2 && N % 2 == 0 && (N / 2) % C == 0 && L.NT >= 2) ? 1 : 0;
  // rows per block in the LDS-resident row passes: aim at >= 128-byte segments, LDS <= 64 KiB
  int R = 2;
  while (R * C < 16 && (size_t)(R * 2) * (N + 1) * 8 <= 64 * 1024) R *= 2;
  // (a tuned value: even, and R rows of the inverse row pass within 64 KiB of LDS)
  if (tune.rows_lds >= 2 && tune.rows_lds % 2 == 0 && tune.rows_lds <= 64 &&
      (size_t)tune.rows_lds * (N + 1) * 8 <= 64 * 1024)
    R = tune.rows_lds;
  L.R = R;
  // register-resident row passes (power-of-two N): T = N / 16 threads per sequence, `seqs`
  // sequences per block (forward: pairs of rows; inverse: rows)
  L.Rf = L.Ri = 2;
  if (reg_plan_ok(N)) {
    const int T = N / 16, target = N >= 2048 ? 512 : 256;
    int seqs = target / T > 1 ? target / T : 1;
    while (seqs > 1 && seqs * reg_seq_lds(N) > 80 * 1024) seqs /= 2;
    int sf = seqs, si = seqs;
    if (tune.seq_fwd > 0 && reg_seqs_ok(N, tune.seq_fwd)) sf = tune.seq_fwd;
    if (tune.seq_inv > 0 && reg_seqs_ok(N, tune.seq_inv)) si = tune.seq_inv;
    L.Rf = 2 * sf;
    L.Ri = si;
    while (L.Rf > 2 && L.Rf / 2 > (M + 1) / 2) L.Rf /= 2;
    while (L.Ri > 1 && L.Ri > M) L.Ri /= 2;
  }
  L.Ndiv = mkdiv(N);
  L.RCdiv = mkdiv(R * C);
  L.RfCdiv = mkdiv(L.Rf * C);
  return L;
}

size_t reg_seq_lds(int N) { return (size_t)reg_row_pitch(N) * sizeof(cf); }

// A block of `seqs` register-resident sequences of length N fits: at most 1024 threads and
// 160 KiB of LDS, power-of-two count.
bool reg_seqs_ok(int N, int seqs) {
  return reg_plan_ok(N) && seqs >= 1 && (seqs & (seqs - 1)) == 0 && seqs * (N / 16) <= 1024 &&
         seqs * reg_seq_lds(N) <= 160 * 1024;
}

// Radix schedule of an LDS-resident transform of length L = 2^a 3^b 5^c: the power of two in
// radix-8 passes (radix 0 or 8; the remainder as one radix-4 or radix-2 pass, or two radix-4
// passes) or in radix-4 passes (radix 4; a leftover factor 2 as one radix-2 pass), then the 3s
// and 5s.  Fewer passes mean fewer LDS round trips; radix-4 butterflies need fewer registers.
FftPlan make_plan(int L, int radix) {
  FftPlan p = FftPlan{};
  p.L = L;
  int rad[kMaxPasses];
  int n = 0, rest = L, a = 0;
  while (rest % 2 == 0) { rest /= 2; ++a; }
  if (radix == 4) {
    if (a % 2) rad[n++] = 2;
    for (int i = 0; i < a / 2; ++i) rad[n++] = 4;
  } else {
    int n8 = a / 3, rem = a % 3;
    if (rem == 1 && n8 > 0) { n8 -= 1; rad[n++] = 4; rad[n++] = 4; }
    else if (rem == 1) rad[n++] = 2;
    else if (rem == 2) rad[n++] = 4;
    for (int i = 0; i < n8; ++i) rad[n++] = 8;
  }
  while (rest % 3 == 0) { rest /= 3; rad[n++] = 3; }
  while (rest % 5 == 0) { rest /= 5; rad[n++] = 5; }
  p.npass = n;
  int s = 1;
  for (int q = 0; q < n; ++q) {
    p.radix[q] = rad[q];
    p.s[q] = s;
    p.nbf[q] = L / rad[q];
    p.tstride[q] = L / (s * rad[q]);
    p.sdiv[q] = mkdiv(s);
    p.nbfdiv[q] = mkdiv(L / rad[q]);
    s *= rad[q];
  }
  return p;
}

// Chunks of an evaluation round: about 16384 bins each (a 512-thread block streams 128 KiB of q
// and |H|^2), at most 512.  Every chunk is one work-queue entry with its own atomics, waits and
// fences, so smaller chunks would spend a batch's rounds on entry overheads.
int lam_sweep_chunks(size_t nbins) {
  size_t want = (nbins + 16383) / 16384;
  if (want < 1) want = 1;
  if (want > 512) want = 512;
  return (int)want;
}

// Threads and elements per thread of a LDS-resident transform over `elems` elements.
static int pick_E(size_t elems, int &threads) {
  threads = 256;
  while ((size_t)threads * 16 < elems && threads < 1024) threads *= 2;
  size_t e = (elems + threads - 1) / threads;
  if (e <= 4) return 4;
  if (e <= 8) return 8;
  return 16;  // elems <= 16 * 1024 by construction of the layout
}

// Group images by a key and call `emit` for each group.
using GKey = std::tuple<int, int, int>;  // (register-resident?, threads or compile-time length, E)

// Length of the compile-time register-resident transform for a pass of length L whose
// sequences are interleaved LS apart in LDS (1 in the row passes, the tile width C in the
// column passes), given the interleave the kernel is compiled for; 0: the run-time transform.
static int fixed_len(int L, int LS, bool col) { return reg_plan_ok(L) && LS == (col ? col_ls(L) : 1) ? L : 0; }

// f(std::integral_constant<int, L>) for a compile-time length L (0: the run-time transform):
// picks the instantiation of a register-resident pass kernel.
template <class F>
static auto by_len(int L, F f) {
  switch (L) {
    case 4096: return f(std::integral_constant<int, 4096>{});
    case 2048: return f(std::integral_constant<int, 2048>{});
    case 1024: return f(std::integral_constant<int, 1024>{});
    case 512: return f(std::integral_constant<int, 512>{});
    case 256: return f(std::integral_constant<int, 256>{});
    default: return f(std::integral_constant<int, 0>{});
  }
}
// Largest images first within a launch: blocks are dealt in item order, so the longest work
// starts first and the small images fill the tail.
void sort_by_size(const ImgSet &set, std::vector<int> &imgs) {
  std::stable_sort(imgs.begin(), imgs.end(), [&](int a, int b) {
    return (size_t)set.imgs[a].L.M * set.imgs[a].L.N > (size_t)set.imgs[b].L.M * set.imgs[b].L.N;
  });
}

static void group_by(const ImgSet &set, const std::vector<int> &sel, const std::function<GKey(const Img &)> &key,
                     const std::function<void(const GKey &, const std::vector<int> &)> &emit) {
  std::map<GKey, std::vector<int>> g;
  for (int i : sel) g[key(set.imgs[i])].push_back(i);
  for (auto &kv : g) {
    sort_by_size(set, kv.second);
    emit(kv.first, kv.second);
  }
}

template <class K4, class K8, class K16>
static auto pickE(int E, K4 a, K8 b, K16 c) {
  return E == 4 ? a : E == 8 ? b : c;
}

void plan_row_fwd(Plan &p, ImgSet &set, const std::vector<int> &sel) {
  group_by(set, sel, [](const Img &d) {
    if (reg_plan_ok(d.L.N)) return GKey{1, fixed_len(d.L.N, 1, false), 0};
    int th; int E = pick_E((size_t)(d.L.R / 2) * d.L.N, th);
    return GKey{0, th, E};
  }, [&](const GKey &k, const std::vector<int> &imgs) {
    if (std::get<0>(k)) {
      int threads = 0; size_t lds = 0;
      for (int i : imgs) {
        const Img &d = set.imgs[i];
        threads = std::max(threads, (d.L.Rf / 2) * d.rn.T);
        lds = std::max(lds, (size_t)(d.L.Rf / 2) * reg_seq_lds(d.L.N));
      }
      // the compile-time transform's twiddle tables follow
      const int tw_off = (int)(lds / sizeof(cf));
      if (std::get<1>(k)) lds += 128 * sizeof(cf);
      ItemRange r = add_items(set, imgs, [](const Img &d) { return (d.L.M + d.L.Rf - 1) / d.L.Rf; });
      const auto kern = by_len(std::get<1>(k), [](auto L) { return k_row_fwd_r16<decltype(L)::value>; });
      p.steps.push_back(make_launch(&set, kern, r, threads, lds, tw_off));
    } else {
      const int threads = std::get<1>(k), E = std::get<2>(k);
      size_t lds = 0;
      for (int i : imgs) lds = std::max(lds, (size_t)(set.imgs[i].L.R / 2) * (set.imgs[i].L.N + 1) * sizeof(cf));
      ItemRange r = add_items(set, imgs, [](const Img &d) { return (d.L.M + d.L.R - 1) / d.L.R; });
      p.steps.push_back(make_launch(&set, pickE(E, k_row_fwd_g<4>, k_row_fwd_g<8>, k_row_fwd_g<16>), r, threads, lds));
    }
  });
}

void plan_col_fwd(Plan &p, ImgSet &set, const std::vector<int> &sel, bool resid) {
  group_by(set, sel, [](const Img &d) {
    if (reg_plan_ok(d.L.M)) return GKey{1, fixed_len(d.L.M, d.L.C, true), 0};
    int th; int E = pick_E((size_t)d.L.M * d.L.C, th);
    return GKey{0, th, E};
  }, [&](const GKey &k, const std::vector<int> &imgs) {
    // the register-resident residual pass folds the last tile into the block of tile 0
    const bool fold = std::get<0>(k) != 0 && resid;
    ItemRange r = add_items(set, imgs, [fold](const Img &d) { return fold ? d.L.col_blocks() : d.L.NT; });
    if (std::get<0>(k)) {
      int threads = 0; size_t lds = 0;
      for (int i : imgs) {
        const Img &d = set.imgs[i];
        threads = std::max(threads, d.L.C * d.rm.T);
        lds = std::max(lds, (size_t)d.L.C * (d.L.M + d.L.M / 16) * sizeof(cf));
      }
      const bool fx = std::get<1>(k) != 0;
      // the compile-time transform's twiddle tables follow
      const int tw_off = (int)(lds / sizeof(cf));
      if (fx) lds += 128 * sizeof(cf);
      const auto kern = resid ? by_len(std::get<1>(k), [](auto L) { return k_col_fwd_r16<true, decltype(L)::value>; })
                              : by_len(std::get<1>(k), [](auto L) { return k_col_fwd_r16<false, decltype(L)::value>; });
      p.steps.push_back(make_launch(&set, kern, r, threads, lds, tw_off));
    } else {
      const int threads = std::get<1>(k), E = std::get<2>(k);
      size_t lds = 0;
      for (int i : imgs) lds = std::max(lds, (size_t)set.imgs[i].L.M * set.imgs[i].L.C * sizeof(cf));
      if (resid)
        p.steps.push_back(make_launch(&set, pickE(E, k_col_fwd_g<4, true>, k_col_fwd_g<8, true>, k_col_fwd_g<16, true>),
                                      r, threads, lds));
      else
        p.steps.push_back(make_launch(
            &set, pickE(E, k_col_fwd_g<4, false>, k_col_fwd_g<8, false>, k_col_fwd_g<16, false>), r, threads, lds));
    }
  });
}

void plan_lambda(Plan &p, ImgSet &set, const std::vector<int> &sel, int rounds, bool advance) {
  // one launch for the whole search after the residual pass: blocks take the images' starts,
  // then the open images' (round, chunk) entries from the set's queue, so the grid need not
  // cover the chunks
  const ItemRange one = add_one_per_image(set, sel);
  size_t chunks = 0;
  for (int i : sel) chunks += (size_t)set.imgs[i].nchunk;
  const int adv = advance ? 1 : 0;
  ImgSet *setp = &set;
  p.steps.push_back([=](hipStream_t s) -> hipError_t {
    if (one.n == 0) return hipSuccess;
    const unsigned grid = (unsigned)std::min<size_t>(std::max(chunks, one.n), 256);
    hipLaunchKernelGGL(k_lam_rounds, dim3(grid), dim3(512), 0, s, (const Img *)setp->dev,
                       (const Item *)(setp->items_dev + one.off), (int)one.n, setp->st_base, setp->lamq, rounds, adv);
    return hipGetLastError();
  });
}

void plan_col_inv(Plan &p, ImgSet &set, const std::vector<int> &sel) {
  group_by(set, sel, [](const Img &d) {
    if (reg_plan_ok(d.L.M)) return GKey{1, fixed_len(d.L.M, d.L.C, true), 0};
    int th; int E = pick_E((size_t)d.L.M * d.L.C, th);
    return GKey{0, th, E};
  }, [&](const GKey &k, const std::vector<int> &imgs) {
    const bool reg = std::get<0>(k) != 0;  // the register-resident pass folds the last tile
    ItemRange r = add_items(set, imgs, [reg](const Img &d) { return reg ? d.L.col_blocks() : d.L.NT; });
    if (std::get<0>(k)) {
      int threads = 0; size_t lds = 0;
      for (int i : imgs) {
        const Img &d = set.imgs[i];
        threads = std::max(threads, d.L.C * d.rm.T);
        lds = std::max(lds, (size_t)d.L.C * (d.L.M + d.L.M / 16) * sizeof(cf));
      }
      const auto kern = by_len(std::get<1>(k), [](auto L) { return k_col_inv_r16<decltype(L)::value>; });
      p.steps.push_back(make_launch(&set, kern, r, threads, lds));
    } else {
      const int threads = std::get<1>(k), E = std::get<2>(k);
      size_t lds = 0;
      for (int i : imgs) lds = std::max(lds, (size_t)set.imgs[i].L.M * set.imgs[i].L.C * sizeof(cf));
      p.steps.push_back(make_launch(&set, pickE(E, k_col_inv_g<4>, k_col_inv_g<8>, k_col_inv_g<16>), r, threads, lds));
    }
  });
}

void plan_row_inv(Plan &p, ImgSet &set, const std::vector<int> &sel) {
  group_by(set, sel, [](const Img &d) {
    if (reg_plan_ok(d.L.N)) return GKey{1, fixed_len(d.L.N, 1, false), 0};
    int th; int E = pick_E((size_t)d.L.R * d.L.N, th);
    return GKey{0, th, E};
  }, [&](const GKey &k, const std::vector<int> &imgs) {
    if (std::get<0>(k)) {
      int threads = 0; size_t lds = 0;
      for (int i : imgs) {
        const Img &d = set.imgs[i];
        threads = std::max(threads, d.L.Ri * d.rn.T);
        // the transform's exchange area, which first holds the staged 16-byte words of the rows
        lds = std::max(lds, (size_t)d.L.Ri * reg_seq_lds(d.L.N));
        lds = std::max(lds, (size_t)d.L.Ri * (d.L.RP + 8) * 16);
      }
      // the compile-time transform's twiddle tables follow
      const int tw_off = (int)(lds / sizeof(cf));
      if (std::get<1>(k)) lds += 128 * sizeof(cf);
      ItemRange r = add_items(set, imgs, [](const Img &d) { return (d.L.M + d.L.Ri - 1) / d.L.Ri; });
      const auto kern = by_len(std::get<1>(k), [](auto L) { return k_row_inv_r16<decltype(L)::value>; });
      p.steps.push_back(make_launch(&set, kern, r, threads, lds, tw_off));
    } else {
      const int threads = std::get<1>(k), E = std::get<2>(k);
      size_t lds = 0;
      for (int i : imgs) lds = std::max(lds, (size_t)set.imgs[i].L.R * (set.imgs[i].L.N + 1) * sizeof(cf));
      ItemRange r = add_items(set, imgs, [](const Img &d) { return (d.L.M + d.L.R - 1) / d.L.R; });
      p.steps.push_back(make_launch(&set, pickE(E, k_row_inv_g<4>, k_row_inv_g<8>, k_row_inv_g<16>), r, threads, lds));
    }
  });
}

hipError_t finalize_items(ImgSet &set) {
  if (set.arena) {
    void *p = nullptr;
    hipError_t e = set.arena->take(std::max<size_t>(set.items_host.size(), 1) * sizeof(Item), &p);
    if (e != hipSuccess) return e;
    set.items_dev = (Item *)p;
    if (set.arena->dry || set.items_host.empty()) return hipSuccess;
    return hipMemcpy(set.items_dev, set.items_host.data(), set.items_host.size() * sizeof(Item), hipMemcpyHostToDevice);
  }
  if (set.items_dev) {
    hipError_t e = hipFree(set.items_dev);
    set.items_dev = nullptr;
    if (e != hipSuccess) return e;
  }
  size_t n = std::max<size_t>(set.items_host.size(), 1);
  hipError_t e = hipMalloc((void **)&set.items_dev, n * sizeof(Item));
  if (e != hipSuccess) return e;
  if (!set.items_host.empty())
    e = hipMemcpy(set.items_dev, set.items_host.data(), set.items_host.size() * sizeof(Item), hipMemcpyHostToDevice);
  return e;
}

// ---------------------------------------------------------------- set-up launchers (one image)
template <class T, class TI>
static hipError_t row_fwd_plain(const TI *x, const Layout &L, const FftPlan &pn, const cpx<T> *tw, cpx<T> *S,
                                hipStream_t st) {
  int threads;
  int E = pick_E((size_t)(L.R / 2) * L.N, threads);
  size_t lds = (size_t)(L.R / 2) * (L.N + 1) * sizeof(cpx<T>);
  int blocks = (L.M + L.R - 1) / L.R;
  auto kern = pickE(E, k_row_fwd_plain<T, TI, 4>, k_row_fwd_plain<T, TI, 8>, k_row_fwd_plain<T, TI, 16>);
  hipError_t e = set_lds(kern, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(threads), lds, st, x, L, pn, tw, S);
  return hipGetLastError();
}

hipError_t launch_row_fwd_d(const double *x, const Layout &L, const FftPlan &pn, const cd *twN, cd *S,
                            hipStream_t st) {
  return row_fwd_plain<double, double>(x, L, pn, twN, S, st);
}
hipError_t launch_row_fwd_fd(const float *x, const Layout &L, const FftPlan &pn, const cd *twN, cd *S,
                             hipStream_t st) {
  return row_fwd_plain<double, float>(x, L, pn, twN, S, st);
}

hipError_t launch_col_fwd_d(cd *S, const Layout &L, const FftPlan &pm, const cd *twM, hipStream_t st) {
  int threads;
  int E = pick_E((size_t)L.M * L.C, threads);
  size_t lds = (size_t)L.M * L.C * sizeof(cd);
  auto kern = pickE(E, k_col_fwd_plain<double, 4>, k_col_fwd_plain<double, 8>, k_col_fwd_plain<double, 16>);
  hipError_t e = set_lds(kern, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(L.NT), dim3(threads), lds, st, S, L, pm, twM);
  return hipGetLastError();
}

hipError_t launch_embed_psf(const float *h, int kh, int kw, int M, int N, double *hp, hipStream_t st) {
  size_t P = (size_t)M * N;
  int blocks = (int)((P + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_d, dim3(blocks), dim3(256), 0, st, hp, P);
  hipLaunchKernelGGL(k_embed_psf, dim3((kh * kw + 255) / 256), dim3(256), 0, st, h, kh, kw, M, N, hp);
  return hipGetLastError();
}

hipError_t launch_init_consts(const cd *Hd, const cd *Yd, const Layout &L, cf *H, cf *Y, cf *HY, float *H2,
                              hipStream_t st) {
  size_t n = L.bins();
  int blocks = (int)((n + 255) / 256);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_init_consts, dim3(blocks), dim3(256), 0, st, Hd, Yd, n, L.Wh, L.M, L.C, L.TS, H, Y, HY, H2);
  return hipGetLastError();
}

hipError_t launch_d2_tables(int M, int N, int Wh, float *dM, float *dN, hipStream_t st) {
  hipLaunchKernelGGL(k_d2_tables, dim3(16), dim3(256), 0, st, M, N, Wh, dM, dN);
  return hipGetLastError();
}

hipError_t launch_rho_target(const float *y, int M, int N, size_t ndom, const float *h, int kh, int kw,
                             double sigma2, double rho_fixed, double *work, double *out2, LamState *st,
                             hipStream_t s) {
  size_t n = (size_t)M * N;
  const int nb = 256;
  hipLaunchKernelGGL(k_ysums, dim3(nb), dim3(256), 0, s, y, n, work);
  hipLaunchKernelGGL(k_ycentred, dim3(nb), dim3(256), 0, s, y, n, work, nb, work + 2 * nb);
  hipLaunchKernelGGL(k_rho_final, dim3(1), dim3(64), 0, s, work, work + 2 * nb, nb, h, kh * kw, n, ndom, sigma2,
                     rho_fixed, out2, st);
  return hipGetLastError();
}

// The observation (or an estimate) y, M x N, in the top-left corner of an Mp x Np image whose
// periodic extension is continuous: columns N.. of each row ramp linearly from its last value
// towards its first (t / (Np - N + 1) of the way at column N - 1 + t), then rows M.. ramp the
// same way between rows M - 1 and 0 of the widened image.  FP64 arithmetic, one rounding.
__global__ void k_pad_ramp(const float *__restrict__ y, int M, int N, float *__restrict__ out, int Mp, int Np) {
  const size_t total = (size_t)Mp * Np;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const int m = (int)(i / Np), n = (int)(i - (size_t)m * Np);
    auto row = [&](int r) -> double {
      const float *yr = y + (size_t)r * N;
      if (n < N) return (double)yr[n];
      const double a = yr[N - 1], b = yr[0];
      return a + (b - a) * (double)(n - N + 1) / (double)(Np - N + 1);
    };
    double v;
    if (m < M) {
      v = row(m);
    } else {
      const double a = row(M - 1), b = row(0);
      v = a + (b - a) * (double)(m - M + 1) / (double)(Mp - M + 1);
    }
    out[i] = (float)v;
  }
}

hipError_t launch_pad_ramp(const float *y, int M, int N, float *out, int Mp, int Np, hipStream_t st) {
  const size_t n = (size_t)Mp * Np;
  int blocks = (int)((n + 255) / 256);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_pad_ramp, dim3(blocks), dim3(256), 0, st, y, M, N, out, Mp, Np);
  return hipGetLastError();
}

hipError_t launch_fill_f(float *p, size_t n, float v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  int blocks = (int)((n + 255) / 256);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_fill_f, dim3(blocks), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_state_reset(LamState *st, hipStream_t s) {
  hipLaunchKernelGGL(k_state_reset, dim3(1), dim3(64), 0, s, st);
  return hipGetLastError();
}

hipError_t launch_state_set_lam(LamState *st, float lam, hipStream_t s) {
  hipLaunchKernelGGL(k_state_set_lam, dim3(1), dim3(64), 0, s, st, lam);
  return hipGetLastError();
}

hipError_t launch_state_set_nscale(LamState *st, int count, int ns, hipStream_t s) {
  hipLaunchKernelGGL(k_state_set_nscale, dim3((count + 255) / 256), dim3(256), 0, s, st, count, ns);
  return hipGetLastError();
}

hipError_t launch_copy_lam_star(const LamState *st, float *out, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_lam_star, dim3(1), dim3(64), 0, s, st, out);
  return hipGetLastError();
}

}  // namespace gfd
