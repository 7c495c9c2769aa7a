// Spectral part of the iteration on gfx950: row / column FFT passes over a tile-major half
// spectrum, the residual and lambda reductions (Sec. 3.2, Eqs.(10)-(11)), the two Fourier
// solves (Sec. 3.1, Eqs.(8)-(9)) and the per-image set-up.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "fft_reg.h"
#include "gfd_internal.h"

namespace gfd {

// ============================================================================ helpers

template <class T>
__device__ __forceinline__ T zero_of() { return (T)0; }

// Sum NV (hi, lo) accumulators of `nparts` block partials with every thread of the block;
// deterministic order.  Result in thread 0.
template <int NV>
__device__ void reduce_partials(const float *__restrict__ partials, int nparts, float (&hi)[NV], float (&lo)[NV],
                                float *scratch) {
#pragma unroll
  for (int v = 0; v < NV; ++v) hi[v] = lo[v] = 0.0f;
  for (int p = threadIdx.x; p < nparts; p += blockDim.x) {
    const float *src = partials + (size_t)p * kLamAcc * 2;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      df_add(hi[v], lo[v], src[2 * v], src[2 * v + 1]);
    }
  }
  block_reduce_df<NV>(hi, lo, scratch);
}

// Plain FP32 butterfly over the wave, then compensated across waves; thread 0 gets the sum.
template <int NV>
__device__ void block_sum_plain_then_df(float (&acc)[NV], float (&hi)[NV], float (&lo)[NV], float *scratch) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] += __shfl_xor(acc[v], off, 64);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) scratch[wid * NV + v] = acc[v];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int v = 0; v < NV; ++v) {
      float h = 0.0f, l = 0.0f;
      for (int w = 0; w < nw; ++w) df_add(h, l, scratch[w * NV + v], 0.0f);
      hi[v] = h;
      lo[v] = l;
    }
  }
  __syncthreads();
}

// Commit the lambda of this iteration (called by one thread once the search is finished).
__device__ void lam_commit(LamState *st, const LamBuffers &lb) {
  float ls = st->lam_star;
  float lam = ls;
  if (!isinf(ls)) {
    float sc = (lb.scales != nullptr && st->k < st->nscale) ? lb.scales[st->k] : 1.0f;
    lam = sc * ls;
    if (!(st->flags & kFlagNoRoot)) {
      st->lam_prev2 = st->lam_prev;
      st->lam_prev = ls;
    }
  }
  st->lam = lam;
  st->flags_all |= (unsigned)st->flags;
  if (lb.lam_hist != nullptr && st->k < lb.hist_cap) {
    lb.lam_hist[st->k] = lam;
    lb.flag_hist[st->k] = st->flags;
  }
}

// ============================================================================ row pass, forward
// Block handles rows [r0, r0 + R): rows are paired into complex sequences z = x_a + i x_b,
// transformed, and separated into the two half spectra X_a[k] = (Z[k] + conj Z[N-k]) / 2,
// X_b[k] = (Z[k] - conj Z[N-k]) / 2i, written tile-major.
template <class T, class TI, int E>
__global__ void __launch_bounds__(1024) k_row_fwd(const TI *__restrict__ x, Layout lay, FftPlan pn,
                                                  const cpx<T> *__restrict__ tw, cpx<T> *__restrict__ S) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T> *buf = reinterpret_cast<cpx<T> *>(smem_raw);
  const int M = lay.M, N = lay.N, R = lay.R, LP = N + 1;
  const int npair = R >> 1;
  const int r0 = xcd_remap(blockIdx.x, gridDim.x) * R;  // neighbouring row blocks share an XCD's L2
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
    S[((size_t)t * M + m) * C + c] = X;
  }
}

// ============================================================================ column pass, forward
template <class T, int E>
__global__ void __launch_bounds__(1024) k_col_fwd(cpx<T> *__restrict__ S, Layout lay, FftPlan pm,
                                                  const cpx<T> *__restrict__ tw) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T> *buf = reinterpret_cast<cpx<T> *>(smem_raw);
  const int n = lay.M * lay.C;
  cpx<T> *tile = S + (size_t)blockIdx.x * n;
  for (int e = threadIdx.x; e < n; e += blockDim.x) buf[e] = tile[e];
  __syncthreads();
  lds_fft<T, E, -1, true>(buf, lay.C, lay.logC, lay.C, 1, pm, tw);
  for (int e = threadIdx.x; e < n; e += blockDim.x) tile[e] = buf[e];
}

// Column pass fused with the residual R = H U_E - Y of Eq.(10), the Hermitian-weighted
// q = w |R|^2 (w = 1 on columns 0 and N/2, else 2), Einf = sum q / P, and the first lambda
// candidates of the search.  Each block writes its compensated partial sums; k_lam_begin
// finishes them.
template <int E>
__global__ void __launch_bounds__(1024) k_col_fwd_resid(cf *__restrict__ S, float *__restrict__ q,
                                                        const cf *__restrict__ H, const cf *__restrict__ Y,
                                                        Layout lay, FftPlan pm, const cf *__restrict__ tw,
                                                        LamBuffers lb) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cf *buf = reinterpret_cast<cf *>(smem_raw);
  __shared__ float scratch[2 * kLamAcc * 16];
  LamState *st = lb.st;
  const int n = lay.M * lay.C;
  const size_t off = (size_t)blockIdx.x * n;
  cf *tile = S + off;
  for (int e = threadIdx.x; e < n; e += blockDim.x) buf[e] = tile[e];
  __syncthreads();
  lds_fft<float, E, -1, true>(buf, lay.C, lay.logC, lay.C, 1, pm, tw);

  constexpr int NC = kLamFirstCand;
  float mu[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) mu[j] = st->mu[j];
  const float mu_floor = 1.0f / kLamFloor;
  float acc[2 + 2 * NC];
#pragma unroll
  for (int v = 0; v < 2 + 2 * NC; ++v) acc[v] = 0.0f;
  const int N = lay.N, Wh = lay.Wh, C = lay.C;
  const int kbase = blockIdx.x * C;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const cf U = buf[e];
    tile[e] = U;
    const int k = kbase + (e & (C - 1));
    float qq = 0.0f, t2 = 0.0f;
    if (k < Wh) {
      const cf h = H[off + e], y = Y[off + e];
      const cf r = cmul(h, U) - y;
      const float wgt = (k == 0 || 2 * k == N) ? 1.0f : 2.0f;
      qq = wgt * abs2f(r);
      t2 = abs2f(h);
    }
    q[off + e] = qq;
    acc[0] += qq;
    {
      float r = __builtin_amdgcn_rcpf(__fmaf_rn(t2, mu_floor, 1.0f));
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
  float hi[2 + 2 * NC], lo[2 + 2 * NC];
  block_sum_plain_then_df<2 + 2 * NC>(acc, hi, lo, scratch);
  if (threadIdx.x == 0) {
    float *dst = lb.partials + (size_t)blockIdx.x * kLamAcc * 2;
    for (int v = 0; v < 2 + 2 * NC; ++v) {
      dst[2 * v] = hi[v];
      dst[2 * v + 1] = lo[v];
    }
  }
}

// ============================================================================ lambda sweep
// One evaluation round: per-block sums over the bins of q g_j and q g_j (1 - r_j) for the
// current candidates (k_lam_round finishes them).
template <int NC>
__global__ void __launch_bounds__(256) k_lam_sweep(const float *__restrict__ q, const float *__restrict__ H2,
                                                   size_t nbins, LamBuffers lb) {
  __shared__ float scratch[2 * kLamAcc * 4];
  LamState *st = lb.st;
  if (st->phase != 0) return;  // lambda already fixed for this iteration
  float mu[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) mu[j] = st->mu[j];
  float acc[2 * NC];
#pragma unroll
  for (int v = 0; v < 2 * NC; ++v) acc[v] = 0.0f;
  const size_t n4 = nbins / 4;
  const float4 *q4 = reinterpret_cast<const float4 *>(q);
  const float4 *h4 = reinterpret_cast<const float4 *>(H2);
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n4; i += (size_t)gridDim.x * blockDim.x) {
    const float4 qa = q4[i], ta = h4[i];
    const float qs[4] = {qa.x, qa.y, qa.z, qa.w}, ts[4] = {ta.x, ta.y, ta.z, ta.w};
#pragma unroll
    for (int u = 0; u < 4; ++u) {
#pragma unroll
      for (int j = 0; j < NC; ++j) {
        const float r = __builtin_amdgcn_rcpf(__fmaf_rn(ts[u], mu[j], 1.0f));
        const float qg = qs[u] * (r * r);
        acc[j] += qg;
        acc[NC + j] = __fmaf_rn(qg, 1.0f - r, acc[NC + j]);
      }
    }
  }
  if (blockIdx.x == 0) {  // tail that does not fill a float4
    for (size_t i = n4 * 4 + threadIdx.x; i < nbins; i += blockDim.x) {
#pragma unroll
      for (int j = 0; j < NC; ++j) {
        const float r = __builtin_amdgcn_rcpf(__fmaf_rn(H2[i], mu[j], 1.0f));
        const float qg = q[i] * (r * r);
        acc[j] += qg;
        acc[NC + j] = __fmaf_rn(qg, 1.0f - r, acc[NC + j]);
      }
    }
  }
  float hi[2 * NC], lo[2 * NC];
  block_sum_plain_then_df<2 * NC>(acc, hi, lo, scratch);
  if (threadIdx.x == 0) {
    float *dst = lb.partials + (size_t)blockIdx.x * kLamAcc * 2;
    for (int v = 0; v < 2 * NC; ++v) {
      dst[2 * v] = hi[v];
      dst[2 * v + 1] = lo[v];
    }
  }
}

// ============================================================================ lambda decisions
// One block finishes the partial sums of the residual pass (round 0) or of a sweep and runs the
// search state machine; deterministic order.
__global__ void __launch_bounds__(256) k_lam_begin(LamBuffers lb, int nparts) {
  __shared__ float scratch[2 * kLamAcc * 4];
  constexpr int NC = kLamFirstCand;
  float hi[2 + 2 * NC], lo[2 + 2 * NC];
  reduce_partials<2 + 2 * NC>(lb.partials, nparts, hi, lo, scratch);
  if (threadIdx.x == 0) {
    LamState *st = lb.st;
    st->phase = 0;
    st->flags = 0;
    float cand[NC];
    for (int j = 0; j < NC; ++j) cand[j] = st->cand[j];
    if (lam_begin(*st, hi[0], lo[0], hi[1], lo[1], NC, cand, hi + 2, lo + 2, hi + 2 + NC)) lam_commit(st, lb);
  }
}

__global__ void __launch_bounds__(256) k_lam_round(LamBuffers lb, int nparts, int last) {
  __shared__ float scratch[2 * kLamAcc * 4];
  constexpr int NC = kLamMaxCand;
  if (lb.st->phase != 0) return;
  float hi[2 * NC], lo[2 * NC];
  reduce_partials<2 * NC>(lb.partials, nparts, hi, lo, scratch);
  if (threadIdx.x == 0) {
    LamState *st = lb.st;
    float cand[NC];
    for (int j = 0; j < NC; ++j) cand[j] = st->cand[j];
    lam_absorb(*st, NC, cand, hi, lo, hi + NC);
    if (lam_decide(*st, last != 0)) lam_commit(st, lb);
  }
}

// ============================================================================ solves + column inverse
// F(u_p) = (conj(H) Y + lam F(u_E)) / (|H|^2 + lam)                         (Eq. 9)
// F(u_I) = (conj(H) Y + lam D2 F(u_E)) / (|H|^2 + lam D2), D2 = |F(grad)|^2 (Eq. 8)
// written with mu = 1/lam when lam >= 1 so that nothing overflows for large lam; lam = +inf
// copies F(u_E) to both.  The 1/P of the inverse transform is applied here.  The U_I spectrum
// waits in registers while U_p is transformed in LDS.
template <int E>
__global__ void __launch_bounds__(1024) k_col_inv(const cf *__restrict__ UE, const cf *__restrict__ HY,
                                                  const float *__restrict__ H2, const float *__restrict__ dM,
                                                  const float *__restrict__ dN, Layout lay, FftPlan pm,
                                                  const cf *__restrict__ tw, LamState *st,
                                                  cf *__restrict__ SI, cf *__restrict__ SP) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cf *buf = reinterpret_cast<cf *>(smem_raw);
  const int n = lay.M * lay.C, C = lay.C, Wh = lay.Wh;
  const size_t off = (size_t)blockIdx.x * n;
  const float lam = st->lam, invP = st->invP;
  const bool inf_branch = isinf(lam);
  const bool big = lam >= 1.0f;
  const float mu = big ? 1.0f / lam : 0.0f;
  const int kbase = blockIdx.x * C;
  cf ui[E];
#pragma unroll
  for (int u = 0; u < E; ++u) {
    const int e = threadIdx.x + u * blockDim.x;
    if (e < n) {
      const int k = kbase + (e & (C - 1)), m = e >> lay.logC;
      cf Up = {0.0f, 0.0f}, Ui = {0.0f, 0.0f};
      if (k < Wh) {
        const cf U = UE[off + e];
        if (inf_branch) {
          Up = cscale(U, invP);
          Ui = Up;
        } else {
          const cf hy = HY[off + e];
          const float t2 = H2[off + e];
          const float d2 = dM[m] + dN[k];
          if (big) {
            const float ip = invP * __builtin_amdgcn_rcpf(__fmaf_rn(mu, t2, 1.0f));
            const float ii = invP * __builtin_amdgcn_rcpf(__fmaf_rn(mu, t2, d2));
            Up = cf{(__fmaf_rn(mu, hy.re, U.re)) * ip, (__fmaf_rn(mu, hy.im, U.im)) * ip};
            Ui = cf{(__fmaf_rn(mu, hy.re, d2 * U.re)) * ii, (__fmaf_rn(mu, hy.im, d2 * U.im)) * ii};
          } else {
            const float ip = invP * __builtin_amdgcn_rcpf(t2 + lam);
            const float ld = lam * d2;
            const float ii = invP * __builtin_amdgcn_rcpf(t2 + ld);
            Up = cf{__fmaf_rn(lam, U.re, hy.re) * ip, __fmaf_rn(lam, U.im, hy.im) * ip};
            Ui = cf{__fmaf_rn(ld, U.re, hy.re) * ii, __fmaf_rn(ld, U.im, hy.im) * ii};
          }
        }
        if (k == 0 && m == 0) {  // zero frequency: the means of u_p and u_I
          st->meanP = Up.re;
          st->meanI = Ui.re;
        }
      }
      buf[e] = Up;
      ui[u] = Ui;
    }
  }
  __syncthreads();
  lds_fft<float, E, +1, true>(buf, C, lay.logC, C, 1, pm, tw);
  for (int e = threadIdx.x; e < n; e += blockDim.x) SP[off + e] = buf[e];
  __syncthreads();
#pragma unroll
  for (int u = 0; u < E; ++u) {
    const int e = threadIdx.x + u * blockDim.x;
    if (e < n) buf[e] = ui[u];
  }
  __syncthreads();
  lds_fft<float, E, +1, true>(buf, C, lay.logC, C, 1, pm, tw);
  for (int e = threadIdx.x; e < n; e += blockDim.x) SI[off + e] = buf[e];
}

// ============================================================================ row pass, inverse
// Row m of the two half spectra A (of u_I) and B (of u_p) are combined into the full
// spectrum Z = A + iB (with Z[N-k] = conj A[k] + i conj B[k]); its inverse transform is
// u_I + i u_p.  Columns 0 and N/2 of a real row's spectrum are real: their imaginary parts
// (rounding residue) are dropped.
template <int E>
__global__ void __launch_bounds__(1024) k_row_inv(const cf *__restrict__ SI, const cf *__restrict__ SP,
                                                  Layout lay, FftPlan pn, const cf *__restrict__ tw,
                                                  float *__restrict__ uI, float *__restrict__ uP) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cf *buf = reinterpret_cast<cf *>(smem_raw);
  const int M = lay.M, N = lay.N, R = lay.R, C = lay.C, Wh = lay.Wh, LP = N + 1;
  const int r0 = xcd_remap(blockIdx.x, gridDim.x) * R;  // neighbouring row blocks share an XCD's L2
  const int per_t = R * C, total = lay.NT * per_t;
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    const int t = fdiv(e, lay.RCdiv), rem = e - t * per_t;
    const int rho = rem >> lay.logC, c = rem & (C - 1);
    const int m = r0 + rho, k = t * C + c;
    if (m >= M || k >= Wh) continue;
    const size_t g = ((size_t)t * M + m) * C + c;
    cf A = SI[g], B = SP[g];
    if (k == 0 || 2 * k == N) {
      A.im = 0.0f;
      B.im = 0.0f;
    }
    cf *z = buf + rho * LP;
    z[k] = cf{A.re - B.im, A.im + B.re};
    if (k > 0 && N - k >= Wh) z[N - k] = cf{A.re + B.im, B.re - A.im};
  }
  __syncthreads();
  lds_fft<float, E, +1, false>(buf, R, 0, 1, LP, pn, tw);
  for (int e = threadIdx.x; e < R * N; e += blockDim.x) {
    const int rho = fdiv(e, lay.Ndiv), nn = e - rho * N;
    const int m = r0 + rho;
    if (m >= M) continue;
    const cf z = buf[rho * LP + nn];
    uI[(size_t)m * N + nn] = z.re;
    uP[(size_t)m * N + nn] = z.im;
  }
}


// ============================================================================ power-of-two lengths
// The same passes with the register-resident radix-16 transform of fft_reg.h: two LDS
// exchanges per transform instead of one per radix pass, and the first / last passes read and
// write global memory directly.

// Row pass, forward: block = npair sequences x T threads.
__global__ void __launch_bounds__(512) k_row_fwd_r16(const float *__restrict__ x, Layout lay, RegPlan rp,
                                                      const cf *__restrict__ tw, cf *__restrict__ S) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cf *lds = reinterpret_cast<cf *>(smem_raw);
  const int M = lay.M, N = lay.N, R = lay.Rf, T = rp.T;
  const int LP = N + (N >> 4);
  const int seq = threadIdx.x / T, t = threadIdx.x - seq * T;
  const int r0 = xcd_remap(blockIdx.x, gridDim.x) * R;
  const int ra = r0 + 2 * seq, rb = ra + 1;
  cf v[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int n = t + T * m;
    v[m] = cf{ra < M ? x[(size_t)ra * N + n] : 0.0f, rb < M ? x[(size_t)rb * N + n] : 0.0f};
  }
  cf *my = lds + seq * LP;
  reg_fft<-1>(v, t, rp, my, 1, tw);
#pragma unroll
  for (int m = 0; m < 16; ++m) my[lds_pad(t + T * m)] = v[m];
  __syncthreads();
  const int C = lay.C, per_t = R * C, Wh = lay.Wh;
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
    S[((size_t)tt * M + m) * C + c] = X;
  }
}

// Column pass, forward (optionally fused with the residual and the first lambda candidates,
// as k_col_fwd_resid): block = C columns x T threads, column c = tid % C.
template <bool RESID>
__global__ void __launch_bounds__(512) k_col_fwd_r16(cf *__restrict__ S, float *__restrict__ q,
                                                      const cf *__restrict__ H, const cf *__restrict__ Y, Layout lay,
                                                      RegPlan rp, const cf *__restrict__ tw, LamBuffers lb) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cf *lds = reinterpret_cast<cf *>(smem_raw);
  __shared__ float scratch[kLamAcc * 16];
  const int C = lay.C, T = rp.T;
  const int c = threadIdx.x & (C - 1), t = threadIdx.x >> lay.logC;
  const size_t off = (size_t)blockIdx.x * lay.M * C;
  cf *tile = S + off;
  cf v[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) v[m] = tile[(t + T * m) * C + c];
  reg_fft<-1>(v, t, rp, lds + c, C, tw);
  if (!RESID) {
#pragma unroll
    for (int m = 0; m < 16; ++m) tile[(t + T * m) * C + c] = v[m];
    return;
  }
  LamState *st = lb.st;
  constexpr int NC = kLamFirstCand;
  float mu[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) mu[j] = st->mu[j];
  const float mu_floor = 1.0f / kLamFloor;
  float acc[2 + 2 * NC];
#pragma unroll
  for (int a = 0; a < 2 + 2 * NC; ++a) acc[a] = 0.0f;
  const int k = blockIdx.x * C + c;
  const bool valid = k < lay.Wh;
  const float wgt = (k == 0 || 2 * k == lay.N) ? 1.0f : 2.0f;
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int e = (t + T * m) * C + c;
    tile[e] = v[m];
    float qq = 0.0f, t2 = 0.0f;
    if (valid) {
      const cf h = H[off + e], y = Y[off + e];
      const cf r = cmul(h, v[m]) - y;
      qq = wgt * abs2f(r);
      t2 = abs2f(h);
    }
    q[off + e] = qq;
    acc[0] += qq;
    {
      const float r = __builtin_amdgcn_rcpf(__fmaf_rn(t2, mu_floor, 1.0f));
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
  float hi[2 + 2 * NC], lo[2 + 2 * NC];
  block_sum_plain_then_df<2 + 2 * NC>(acc, hi, lo, scratch);
  if (threadIdx.x == 0) {
    float *dst = lb.partials + (size_t)blockIdx.x * kLamAcc * 2;
    for (int a = 0; a < 2 + 2 * NC; ++a) {
      dst[2 * a] = hi[a];
      dst[2 * a + 1] = lo[a];
    }
  }
}

// Solves (Eqs. 8-9) and column inverse of both spectra; U_I waits in registers.
__global__ void __launch_bounds__(512) k_col_inv_r16(const cf *__restrict__ UE, const cf *__restrict__ HY,
                                                      const float *__restrict__ H2, const float *__restrict__ dM,
                                                      const float *__restrict__ dN, Layout lay, RegPlan rp,
                                                      const cf *__restrict__ tw, LamState *st, cf *__restrict__ SI,
                                                      cf *__restrict__ SP) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cf *lds = reinterpret_cast<cf *>(smem_raw);
  const int C = lay.C, T = rp.T;
  const int c = threadIdx.x & (C - 1), t = threadIdx.x >> lay.logC;
  const size_t off = (size_t)blockIdx.x * lay.M * C;
  const float lam = st->lam, invP = st->invP;
  const bool inf_branch = isinf(lam);
  const bool big = lam >= 1.0f;
  const float mu = big ? 1.0f / lam : 0.0f;
  const int k = blockIdx.x * C + c;
  const bool valid = k < lay.Wh;
  const float dk = valid ? dN[k] : 0.0f;
  cf vp[16], vi[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int row = t + T * m;
    const int e = row * C + c;
    cf Up = {0.0f, 0.0f}, Ui = {0.0f, 0.0f};
    if (valid) {
      const cf U = UE[off + e];
      if (inf_branch) {
        Up = cscale(U, invP);
        Ui = Up;
      } else {
        const cf hy = HY[off + e];
        const float t2 = H2[off + e];
        const float d2 = dM[row] + dk;
        if (big) {
          const float ip = invP * __builtin_amdgcn_rcpf(__fmaf_rn(mu, t2, 1.0f));
          const float ii = invP * __builtin_amdgcn_rcpf(__fmaf_rn(mu, t2, d2));
          Up = cf{(__fmaf_rn(mu, hy.re, U.re)) * ip, (__fmaf_rn(mu, hy.im, U.im)) * ip};
          Ui = cf{(__fmaf_rn(mu, hy.re, d2 * U.re)) * ii, (__fmaf_rn(mu, hy.im, d2 * U.im)) * ii};
        } else {
          const float ip = invP * __builtin_amdgcn_rcpf(t2 + lam);
          const float ld = lam * d2;
          const float ii = invP * __builtin_amdgcn_rcpf(t2 + ld);
          Up = cf{__fmaf_rn(lam, U.re, hy.re) * ip, __fmaf_rn(lam, U.im, hy.im) * ip};
          Ui = cf{__fmaf_rn(ld, U.re, hy.re) * ii, __fmaf_rn(ld, U.im, hy.im) * ii};
        }
      }
      if (k == 0 && row == 0) {
        st->meanP = Up.re;
        st->meanI = Ui.re;
      }
    }
    vp[m] = Up;
    vi[m] = Ui;
  }
  reg_fft<+1>(vp, t, rp, lds + c, C, tw);
#pragma unroll
  for (int m = 0; m < 16; ++m) SP[off + (t + T * m) * C + c] = vp[m];
  reg_fft<+1>(vi, t, rp, lds + c, C, tw);
#pragma unroll
  for (int m = 0; m < 16; ++m) SI[off + (t + T * m) * C + c] = vi[m];
}

// Row pass, inverse: block = Ri rows x T threads; the Hermitian completion is gathered
// straight from the tile-major spectra.
__global__ void __launch_bounds__(512) k_row_inv_r16(const cf *__restrict__ SI, const cf *__restrict__ SP,
                                                      Layout lay, RegPlan rp, const cf *__restrict__ tw,
                                                      float *__restrict__ uI, float *__restrict__ uP) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cf *lds = reinterpret_cast<cf *>(smem_raw);
  const int M = lay.M, N = lay.N, C = lay.C, Wh = lay.Wh, T = rp.T;
  const int LP = N + (N >> 4);
  const int seq = threadIdx.x / T, t = threadIdx.x - seq * T;
  const int m0 = xcd_remap(blockIdx.x, gridDim.x) * lay.Ri;
  const int row = m0 + seq;
  const int rowc = row < M ? row : M - 1;  // rows past the end compute a copy, never stored
  cf v[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int n = t + T * m;
    const bool direct = n < Wh;
    const int kk = direct ? n : N - n;
    const size_t g = ((size_t)(kk >> lay.logC) * M + rowc) * C + (kk & (C - 1));
    cf A = SI[g], B = SP[g];
    if (kk == 0 || 2 * kk == N) {
      A.im = 0.0f;
      B.im = 0.0f;
    }
    v[m] = direct ? cf{A.re - B.im, A.im + B.re} : cf{A.re + B.im, B.re - A.im};
  }
  reg_fft<+1>(v, t, rp, lds + seq * LP, 1, tw);
  if (row < M) {
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const size_t g = (size_t)row * N + t + T * m;
      uI[g] = v[m].re;
      uP[g] = v[m].im;
    }
  }
}

// ============================================================================ init kernels
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
                              int logC, cf *__restrict__ H, cf *__restrict__ Y, cf *__restrict__ HY,
                              float *__restrict__ H2) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const size_t t = i / ((size_t)M * C);
    const int c = (int)(i & (size_t)(C - 1));
    const bool valid = (int)(t * C) + c < Wh;
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

// FP64 sums over y for Eq.(12): stage 1 per-block partial sums of y and y^2.
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

// Stage 2: centred sum of squares sum (y - mean)^2 (second pass, per block).
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
    double d = (double)y[i] - mean;
    s += d * d;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part2[blockIdx.x] = sh[0];
}

// Stage 3: rho of Eq.(12) (radicand clipped to [1e-12, 1]) unless fixed, target
// T = rho P sigma^2, and the constants of the search state.
__global__ void k_rho_final(const double *__restrict__ part, const double *__restrict__ part2, int nparts,
                            const float *__restrict__ h, int nh, size_t n, double sigma2, double rho_fixed,
                            double *out2, LamState *st) {
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
  st->TP = (float)(T * P);
  st->invP = (float)(1.0 / P);
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
  lam_first_candidates(*st);
}

__global__ void k_state_set_lam(LamState *st, float lam) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  st->lam = lam;
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

Layout make_layout(int M, int N) {
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
  // rows per block in the row passes: aim at >= 128-byte segments, keep LDS <= 64 KiB
  int R = 2;
  while (R * C < 16 && (size_t)(R * 2) * (N + 1) * 8 <= 64 * 1024) R *= 2;
  L.R = R;
  // register-resident row passes (power-of-two N): T = N / 16 threads per sequence
  L.Rf = L.Ri = 2;
  if (reg_plan_ok(N)) {
    const int T = N / 16, target = N >= 2048 ? 512 : 256;
    const size_t lds_seq = (size_t)(N + N / 16) * sizeof(cf);
    int seqs = target / T > 1 ? target / T : 1;
    while (seqs > 1 && seqs * lds_seq > 80 * 1024) seqs /= 2;
    L.Rf = 2 * seqs;
    L.Ri = seqs;
    if (const char *e = getenv("GFD_TUNE_RF")) L.Rf = atoi(e);
    if (const char *e = getenv("GFD_TUNE_RI")) L.Ri = atoi(e);
    while (L.Rf > 2 && L.Rf / 2 > (M + 1) / 2) L.Rf /= 2;
    while (L.Ri > 1 && L.Ri > M) L.Ri /= 2;
  }
  L.Ndiv = mkdiv(N);
  L.RCdiv = mkdiv(R * C);
  L.RfCdiv = mkdiv(L.Rf * C);
  return L;
}

FftPlan make_plan(int L) {
  FftPlan p;
  p = FftPlan{};
  p.L = L;
  int rad[kMaxPasses];
  int n = 0, rest = L, a = 0;
  while (rest % 2 == 0) { rest /= 2; ++a; }
  int n8 = a / 3, rem = a % 3;
  if (rem == 1 && n8 > 0) { n8 -= 1; rad[n++] = 4; rad[n++] = 4; }
  else if (rem == 1) rad[n++] = 2;
  else if (rem == 2) rad[n++] = 4;
  for (int i = 0; i < n8; ++i) rad[n++] = 8;
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

// Elements per thread for a block of `threads` threads over `elems` elements.
static int pick_E(size_t elems, int &threads) {
  threads = 256;
  while ((size_t)threads * 16 < elems && threads < 1024) threads *= 2;
  size_t e = (elems + threads - 1) / threads;
  if (e <= 4) return 4;
  if (e <= 8) return 8;
  return 16;  // callers keep elems <= 16 * 1024
}

#define GFD_DISPATCH_E(E_, ...)                  \
  switch (E_) {                                  \
    case 4: { constexpr int EE = 4; __VA_ARGS__; } break;   \
    case 8: { constexpr int EE = 8; __VA_ARGS__; } break;   \
    default: { constexpr int EE = 16; __VA_ARGS__; } break; \
  }

template <class T, class TI>
static hipError_t row_fwd_any(const TI *x, const Layout &L, const FftPlan &pn, const cpx<T> *tw, cpx<T> *S,
                              hipStream_t st) {
  int threads;
  int E = pick_E((size_t)(L.R / 2) * L.N, threads);
  size_t lds = (size_t)(L.R / 2) * (L.N + 1) * sizeof(cpx<T>);
  int blocks = (L.M + L.R - 1) / L.R;
  GFD_DISPATCH_E(E, {
    auto kern = k_row_fwd<T, TI, EE>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(threads), lds, st, x, L, pn, tw, S);
  });
  return hipGetLastError();
}

template <class K>
static hipError_t set_lds(K kern, size_t lds) {
  return hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

hipError_t launch_row_fwd(const float *x, const Layout &L, const FftPlan &pn, const cf *twN, cf *S, hipStream_t st) {
  if (reg_plan_ok(L.N)) {
    const RegPlan rp = make_reg_plan(L.N);
    const size_t lds = (size_t)(L.Rf / 2) * (L.N + L.N / 16) * sizeof(cf);
    hipError_t e = set_lds(k_row_fwd_r16, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_row_fwd_r16, dim3((L.M + L.Rf - 1) / L.Rf), dim3((L.Rf / 2) * rp.T), lds, st, x, L, rp, twN,
                       S);
    return hipGetLastError();
  }
  return row_fwd_any<float, float>(x, L, pn, twN, S, st);
}
hipError_t launch_row_fwd_d(const double *x, const Layout &L, const FftPlan &pn, const cd *twN, cd *S,
                            hipStream_t st) {
  return row_fwd_any<double, double>(x, L, pn, twN, S, st);
}
hipError_t launch_row_fwd_fd(const float *x, const Layout &L, const FftPlan &pn, const cd *twN, cd *S,
                             hipStream_t st) {
  return row_fwd_any<double, float>(x, L, pn, twN, S, st);
}

template <class T>
static hipError_t col_fwd_any(cpx<T> *S, const Layout &L, const FftPlan &pm, const cpx<T> *tw, hipStream_t st) {
  int threads;
  int E = pick_E((size_t)L.M * L.C, threads);
  size_t lds = (size_t)L.M * L.C * sizeof(cpx<T>);
  GFD_DISPATCH_E(E, {
    auto kern = k_col_fwd<T, EE>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(L.NT), dim3(threads), lds, st, S, L, pm, tw);
  });
  return hipGetLastError();
}
hipError_t launch_col_fwd_d(cd *S, const Layout &L, const FftPlan &pm, const cd *twM, hipStream_t st) {
  return col_fwd_any<double>(S, L, pm, twM, st);
}
static size_t col_r16_lds(const Layout &L) { return (size_t)L.C * (L.M + L.M / 16) * sizeof(cf); }

hipError_t launch_col_fwd_f(cf *S, const Layout &L, const FftPlan &pm, const cf *twM, hipStream_t st) {
  if (reg_plan_ok(L.M)) {
    const RegPlan rp = make_reg_plan(L.M);
    const size_t lds = col_r16_lds(L);
    hipError_t e = set_lds(k_col_fwd_r16<false>, lds);
    if (e != hipSuccess) return e;
    LamBuffers none = {};
    hipLaunchKernelGGL(k_col_fwd_r16<false>, dim3(L.NT), dim3(L.C * rp.T), lds, st, S, nullptr, nullptr, nullptr, L, rp,
                       twM, none);
    return hipGetLastError();
  }
  return col_fwd_any<float>(S, L, pm, twM, st);
}

hipError_t launch_col_fwd_resid(cf *S, float *q, const cf *H, const cf *Y, const Layout &L, const FftPlan &pm,
                                const cf *twM, const LamBuffers &lb, hipStream_t st) {
  if (reg_plan_ok(L.M)) {
    const RegPlan rp = make_reg_plan(L.M);
    const size_t lds = col_r16_lds(L);
    hipError_t e = set_lds(k_col_fwd_r16<true>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_col_fwd_r16<true>, dim3(L.NT), dim3(L.C * rp.T), lds, st, S, q, H, Y, L, rp, twM, lb);
    hipLaunchKernelGGL(k_lam_begin, dim3(1), dim3(256), 0, st, lb, L.NT);
    return hipGetLastError();
  }
  int threads;
  int E = pick_E((size_t)L.M * L.C, threads);
  size_t lds = (size_t)L.M * L.C * sizeof(cf);
  GFD_DISPATCH_E(E, {
    auto kern = k_col_fwd_resid<EE>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(L.NT), dim3(threads), lds, st, S, q, H, Y, L, pm, twM, lb);
  });
  hipLaunchKernelGGL(k_lam_begin, dim3(1), dim3(256), 0, st, lb, L.NT);
  return hipGetLastError();
}

int lam_sweep_blocks(size_t nbins) {
  size_t want = (nbins / 4 + 255) / 256;
  if (want < 1) want = 1;
  if (want > 512) want = 512;
  return (int)want;
}

hipError_t launch_lam_sweep(const float *q, const float *H2, size_t nbins, const LamBuffers &lb, int last,
                            hipStream_t st) {
  const int nb = lam_sweep_blocks(nbins);
  hipLaunchKernelGGL(k_lam_sweep<kLamMaxCand>, dim3(nb), dim3(256), 0, st, q, H2, nbins, lb);
  hipLaunchKernelGGL(k_lam_round, dim3(1), dim3(256), 0, st, lb, nb, last);
  return hipGetLastError();
}

hipError_t launch_col_inv(const cf *UE, const cf *HY, const float *H2, const float *dM, const float *dN,
                          const Layout &L, const FftPlan &pm, const cf *twM, const LamBuffers &lb, cf *SI, cf *SP,
                          hipStream_t st) {
  if (reg_plan_ok(L.M)) {
    const RegPlan rp = make_reg_plan(L.M);
    const size_t lds = col_r16_lds(L);
    hipError_t e = set_lds(k_col_inv_r16, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_col_inv_r16, dim3(L.NT), dim3(L.C * rp.T), lds, st, UE, HY, H2, dM, dN, L, rp, twM, lb.st, SI,
                       SP);
    return hipGetLastError();
  }
  int threads;
  int E = pick_E((size_t)L.M * L.C, threads);
  size_t lds = (size_t)L.M * L.C * sizeof(cf);
  GFD_DISPATCH_E(E, {
    auto kern = k_col_inv<EE>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(L.NT), dim3(threads), lds, st, UE, HY, H2, dM, dN, L, pm, twM, lb.st, SI, SP);
  });
  return hipGetLastError();
}

hipError_t launch_row_inv(const cf *SI, const cf *SP, const Layout &L, const FftPlan &pn, const cf *twN, float *uI,
                          float *uP, hipStream_t st) {
  if (reg_plan_ok(L.N)) {
    const RegPlan rp = make_reg_plan(L.N);
    const size_t lds = (size_t)L.Ri * (L.N + L.N / 16) * sizeof(cf);
    hipError_t e = set_lds(k_row_inv_r16, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_row_inv_r16, dim3((L.M + L.Ri - 1) / L.Ri), dim3(L.Ri * rp.T), lds, st, SI, SP, L, rp, twN, uI,
                       uP);
    return hipGetLastError();
  }
  int threads;
  int E = pick_E((size_t)L.R * L.N, threads);
  size_t lds = (size_t)L.R * (L.N + 1) * sizeof(cf);
  int blocks = (L.M + L.R - 1) / L.R;
  GFD_DISPATCH_E(E, {
    auto kern = k_row_inv<EE>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(threads), lds, st, SI, SP, L, pn, twN, uI, uP);
  });
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
  hipLaunchKernelGGL(k_init_consts, dim3(blocks), dim3(256), 0, st, Hd, Yd, n, L.Wh, L.M, L.C, L.logC, H, Y, HY, H2);
  return hipGetLastError();
}

hipError_t launch_d2_tables(int M, int N, int Wh, float *dM, float *dN, hipStream_t st) {
  hipLaunchKernelGGL(k_d2_tables, dim3(16), dim3(256), 0, st, M, N, Wh, dM, dN);
  return hipGetLastError();
}

hipError_t launch_rho_target(const float *y, int M, int N, const float *h, int kh, int kw, double sigma2,
                             double rho_fixed, double *work, double *out2, LamState *st, hipStream_t s) {
  size_t n = (size_t)M * N;
  const int nb = 256;
  hipLaunchKernelGGL(k_ysums, dim3(nb), dim3(256), 0, s, y, n, work);
  hipLaunchKernelGGL(k_ycentred, dim3(nb), dim3(256), 0, s, y, n, work, nb, work + 2 * nb);
  hipLaunchKernelGGL(k_rho_final, dim3(1), dim3(64), 0, s, work, work + 2 * nb, nb, h, kh * kw, n, sigma2, rho_fixed,
                     out2, st);
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

hipError_t launch_copy_lam_star(const LamState *st, float *out, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_lam_star, dim3(1), dim3(64), 0, s, st, out);
  return hipGetLastError();
}

}  // namespace gfd
