// Reverse mode of one iteration on gfx950: the adjoint of the guided filter (Sec. 2,
// Eqs.(3)-(5)), of the two Fourier solves (Eqs.(8)-(9)) with lambda tied to the pre-estimate
// by the discrepancy equation (Eq.(11)), and of the transforms.
//
// Guided filter.  With mu = B(I), pbar = B(p), v = B(I^2) - mu^2, c = B(I p) - mu pbar,
// a = c / (v + eps), b = pbar - a mu and u = B(a) I + B(b), and B its own transpose (centred
// odd periodic windows), the gradient g_u of u gives
//   g_pbar = B(g_u), g_a = B(g_u I) - B(g_u) mu, g_mu = -B(g_u) a,
//   g_c = g_a / (v + eps), g_v = -g_a a / (v + eps), d eps += sum g_v,
//   g_mu -= g_c pbar + 2 mu g_v, g_pbar -= g_c mu,
//   g_I = g_u B(a) + B(g_mu) + p B(g_c) + 2 I B(g_v),  g_p = B(g_pbar) + I B(g_c).
// Three streaming box passes compute it (k_box_stage with three epilogues), in the same
// mean-centred variables as the forward filter (the filter commutes with constant shifts, so
// the gradient is the same); the first one's results (a, mu, pbar, v + eps) come from the
// replayed iteration's own filter wherever the strip kernel runs it, so that pass runs only for
// windows that take the separable passes.  With windows clipped to the image, B = D^-1 S (S the clipped
// window sum, symmetric; D the counts) and the box sums that carry gradients backwards are
// B^T = S D^-1: their fields are divided by the count of the input pixel's window before they
// are summed, and their sums are used as they are.
//
// Solves.  For lambda = s lambda*, R = H U_E - Y, dp = |H|^2 + lambda, dI = |H|^2 + lambda D2:
//   G_UE = (lambda / dp) G_p + (lambda D2 / dI) G_I  with  G_x = F(g_x) / P,
//   g_lambda = Re sum conj(G_p) conj(H) R / dp^2 + Re sum conj(G_I) D2 conj(H) R / dI^2,
//   g_s = g_lambda lambda*, and from f(lambda*, U_E) = T (Eq.(11)):
//   G_UE += kappa g conj(H) R,  kappa = -(2 / P) g_lambda s / f'(lambda*),
//   g = (lambda* / (|H|^2 + lambda*))^2,  f' = (1/P) sum |R|^2 2 lambda* |H|^2 / (|H|^2 + lambda*)^3,
// and g_uE = Re(P F^-1(G_UE)), the unnormalised inverse transform.  Sums over the full
// spectrum are taken over the half spectrum with Hermitian weights.  lambda = +inf passes
// g_uE = g_I + g_p; a lambda* clamped at its floor is a constant (kappa = 0).
#include <algorithm>
#include <map>

#include "box_sum.h"
#include "gfd_internal.h"
#include "wide_box.h"

namespace gfd {

// ============================================================================ box passes
// Each stage loads NR raw values per pixel (load) and derives its NF summed fields from them
// (fields).  Its epilogue receives, for the output pixel, the raw values (from the register ring)
// and NE more values loaded a round ahead (eload).
// kT marks the fields whose sums are transposed means (gradients flowing back through B).
struct BoxStage1 {  // window means of I, p, I^2, I p  ->  a, mu, pbar, v + eps
  static constexpr int NF = 4, NR = 2, NE = 1;
  static constexpr int kWideRows = 2;  // rows per round of barriers at r >= 7
  static constexpr unsigned kT = 0u;
  static constexpr bool kEps = false;
  __device__ static void load(const Img &d, size_t g, float (&r)[NR]) {
    r[0] = G(d.uI)[g];
    r[1] = G(d.uP)[g];
  }
  __device__ static void eload(const Img &, size_t, float (&e)[NE]) { e[0] = 0.0f; }
  __device__ static void fields(const float (&r)[NR], float cI, float cP, float (&v)[NF]) {
    const float I = __fsub_rn(r[0], cI), p = __fsub_rn(r[1], cP);
    v[0] = I;
    v[1] = p;
    v[2] = I * I;
    v[3] = I * p;
  }
  __device__ static void emit(const Img &d, size_t g, const float (&B)[NF], const float (&)[NR],
                              const float (&)[NE], float, float, float &) {
    const float mu = B[0], pb = B[1];
    const float var = fmaxf(__fmaf_rn(-mu, mu, B[2]), 0.0f);
    const float cov = __fmaf_rn(-mu, pb, B[3]);
    const float ve = var + d.eps;
    G(d.ga)[g] = cov / ve;
    G(d.gmu)[g] = mu;
    G(d.gpb)[g] = pb;
    G(d.gve)[g] = ve;
  }
};

struct BoxStage2 {  // window means of a, g_u I, g_u  ->  g_mu, g_pbar, g_v, g_c, g_u B(a)
  static constexpr int NF = 3, NR = 3, NE = 3;
  static constexpr int kWideRows = 4;
  static constexpr unsigned kT = 6u;  // B^T(g_u I), B^T(g_u)
  static constexpr bool kEps = true;
  __device__ static void load(const Img &d, size_t g, float (&r)[NR]) {
    r[0] = G(d.ga)[g];
    r[1] = G(d.gu)[g];
    r[2] = G(d.uI)[g];
  }
  __device__ static void eload(const Img &d, size_t g, float (&e)[NE]) {
    e[0] = G(d.gmu)[g];
    e[1] = G(d.gpb)[g];
    e[2] = G(d.gve)[g];
  }
  __device__ static void fields(const float (&r)[NR], float cI, float, float (&v)[NF]) {
    v[0] = r[0];
    v[1] = r[1] * __fsub_rn(r[2], cI);
    v[2] = r[1];
  }
  // mu, pbar and v + eps of the output pixel are read (a round ahead) before this epilogue
  // replaces them; no other pixel reads them.
  __device__ static void emit(const Img &d, size_t g, const float (&B)[NF], const float (&r)[NR],
                              const float (&e)[NE], float, float, float &eacc) {
    const float A = B[0], Ga = B[1], Gb = B[2];
    const float a = r[0], gu = r[1], mu = e[0], pb = e[1], ve = e[2];
    float g_pbar = Gb;
    const float g_a = __fmaf_rn(-Gb, mu, Ga);
    float g_mu = -Gb * a;
    const float g_c = g_a / ve;
    const float g_v = -g_c * a;
    eacc += g_v;
    g_mu = g_mu - g_c * pb - 2.0f * mu * g_v;
    g_pbar = __fmaf_rn(-g_c, mu, g_pbar);
    G(d.gmu)[g] = g_mu;
    G(d.gpb)[g] = g_pbar;
    G(d.gve)[g] = g_v;
    G(d.gc)[g] = g_c;
    G(d.gd)[g] = gu * A;
  }
};

struct BoxStage3 {  // window means of g_mu, g_c, g_v, g_pbar  ->  g_I, g_p
  static constexpr int NF = 4, NR = 4, NE = 3;
  static constexpr int kWideRows = 2;
  static constexpr unsigned kT = 15u;  // all four are transposed means
  static constexpr bool kEps = false;
  __device__ static void load(const Img &d, size_t g, float (&r)[NR]) {
    r[0] = G(d.gmu)[g];
    r[1] = G(d.gc)[g];
    r[2] = G(d.gve)[g];
    r[3] = G(d.gpb)[g];
  }
  __device__ static void eload(const Img &d, size_t g, float (&e)[NE]) {
    e[0] = G(d.uI)[g];
    e[1] = G(d.uP)[g];
    e[2] = G(d.gd)[g];
  }
  __device__ static void fields(const float (&r)[NR], float, float, float (&v)[NF]) {
#pragma unroll
    for (int f = 0; f < NF; ++f) v[f] = r[f];
  }
  __device__ static void emit(const Img &d, size_t g, const float (&B)[NF], const float (&)[NR],
                              const float (&e)[NE], float cI, float cP, float &) {
    const float I = __fsub_rn(e[0], cI), p = __fsub_rn(e[1], cP);
    G(d.gI)[g] = e[2] + B[0] + p * B[1] + 2.0f * I * B[2];
    G(d.gP)[g] = __fmaf_rn(I, B[1], B[3]);
  }
};

// One periodic w x w box pass over a strip of bxTX columns and bxTY rows per block: every
// thread owns a column of the strip extended by r on both sides, keeps compensated vertical
// running sums of the stage's NF fields and the block forms the horizontal window sums in
// LDS; the stage's epilogue consumes the window means of each output pixel.  Images whose
// lambda was +inf skip nothing here (the filter is applied on that branch too).  With CLIP,
// pixels outside the image enter the sums as zeros and the means are normalised by counts.
template <int R, class Op, bool CLIP>
__global__ void __launch_bounds__(kGfThreads) k_box_stage(const Img *__restrict__ D, const Item *__restrict__ W,
                                                          int nitems) {
  // rows per round of barriers: Op::kWideRows for the widest periodic radii (measured at w = 17,
  // 4096^2: four rows for the three-field stage, two for the four-field stages, which then lose
  // more occupancy to registers than they save in barriers; the clipped variant's longer body is
  // not unrolled over four rows), two otherwise
  constexpr int NF = Op::NF, Wn = 2 * R + 1, RB = R >= 7 && !CLIP ? Op::kWideRows : kGfRB;
  constexpr int VP = hs_pitch<R>();
  __shared__ __align__(16) float vbuf[RB * NF * VP];
  __shared__ __align__(16) float hbuf[RB * NF * kHsOut];
  __shared__ float red[kGfThreads / 64];
  const float inv_w2 = 1.0f / (float)(Wn * Wn);
  for (int ii = blockIdx.x; ii < nitems; ii += gridDim.x) {
    const Item wi = W[ii];
    if (wi.blk < 0) continue;
    const Img &d = D[wi.img];
    const int M = d.L.M, N = d.L.N, TX = d.bxTX, TY = d.bxTY, nby = d.bxNBY;
    const int bx = wi.blk / nby, by = wi.blk - bx * nby;
    const int x0 = bx * TX, y0 = by * TY;
    const int j = threadIdx.x, used = TX + 2 * R;
    const bool active = j < used;
    const int gx = wrap(x0 - R + j, N);
    const int nrows = TY + 2 * R, ybase = y0 - R;  // stream row it is image row ybase + it
    const float cI = d.st->meanI, cP = d.st->meanP;
    const int xcol = x0 - R + j;
    const bool colin = !CLIP || (xcol >= 0 && xcol < N);
    const int ncol = CLIP && colin ? clip_count<R>(xcol, N) : 1;
    // CLIP: factor of the fields of stream row `row` (0 outside the image; the reciprocal count
    // of the pixel's window for transposed fields)
    auto in_scale = [&](int row, int f) -> float {
      const int y = ybase + row;
      if (!(colin && y >= 0 && y < M)) return 0.0f;
      return ((Op::kT >> f) & 1u) ? __builtin_amdgcn_rcpf((float)(clip_count<R>(y, M) * ncol)) : 1.0f;
    };
    hs_zero_pads<R>(vbuf, RB * NF);  // ordered before the first reads by the first barrier
    Kahan s[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) s[f] = Kahan{0.0f, 0.0f};
    float eacc = 0.0f;
    constexpr int NR = Op::NR, NE = Op::NE;
    // Register ring of the raw values of the last Wn stream rows (slot it % Wn; the row loop is
    // unrolled over RB * Wn rows so that slots are compile-time indices): rows leaving the
    // windows are never loaded twice.  Loads run one round ahead: each round consumes the values
    // loaded during the previous round before it issues the next loads.  The epilogue operands
    // of the output row (stream row it - r) come from the ring and from NE loads, also issued a
    // round ahead.
    float ring[Wn][NR];
#pragma unroll
    for (int k = 0; k < Wn; ++k)
#pragma unroll
      for (int x = 0; x < NR; ++x) ring[k][x] = 0.0f;
    float nr[RB][NR], ne[RB][NE];
    // Rows are fetched in stream order: the wrapped image row of the next fetch is carried from
    // one fetch to the next (no division per row); stream rows past the end repeat the last.
    int f_it = 0, f_row = wrap(ybase, M);
    auto fetch_next = [&](float (&rn)[NR], float (&en)[NE]) {
      Op::load(d, (size_t)f_row * N + gx, rn);
      // epilogue row: image row ybase + it - R, clamped into the strip's output rows
      const int ye = min(max(ybase + f_it - R, y0), min(y0 + TY, M) - 1);
      const int xe = min(x0 - R + j, N - 1);
      Op::eload(d, (size_t)ye * N + max(xe, 0), en);
      if (f_it < nrows - 1) {
        ++f_it;
        if (++f_row == M) f_row = 0;
      }
    };
#pragma unroll
    for (int q = 0; q < RB; ++q) fetch_next(nr[q], ne[q]);
    for (int base0 = 0; base0 < nrows; base0 += RB * Wn) {
#pragma unroll
      for (int rr = 0; rr < Wn; ++rr) {
        const int base = base0 + RB * rr;
        if (base >= nrows) break;  // uniform
        float er[RB][NR], ee[RB][NE];
#pragma unroll
        for (int q = 0; q < RB; ++q) {
          const int it = base + q;
          const int sl = (RB * rr + q) % Wn, so = (RB * rr + q + Wn - R) % Wn;
          float vn[NF], vo[NF];
          Op::fields(nr[q], cI, cP, vn);
          Op::fields(ring[sl], cI, cP, vo);  // stream row it - Wn (zeros while it < Wn)
          if (CLIP) {
#pragma unroll
            for (int f = 0; f < NF; ++f) {
              vn[f] *= in_scale(it, f);
              vo[f] *= in_scale(it - Wn, f);
            }
          }
#pragma unroll
          for (int x = 0; x < NR; ++x) ring[sl][x] = nr[q][x];
#pragma unroll
          for (int x = 0; x < NR; ++x) er[q][x] = ring[so][x];  // the output row's raw values
#pragma unroll
          for (int x = 0; x < NE; ++x) ee[q][x] = ne[q][x];
          float *vb = vbuf + q * NF * VP + hs_col(j + R);
          if (active && it < nrows) {
#pragma unroll
            for (int f = 0; f < NF; ++f) {
              kahan_slide(s[f], vn[f], it >= Wn ? vo[f] : 0.0f);
              vb[f * VP] = s[f].s;
            }
          } else {
#pragma unroll
            for (int f = 0; f < NF; ++f) vb[f * VP] = 0.0f;
          }
        }
#pragma unroll
        for (int q = 0; q < RB; ++q) fetch_next(nr[q], ne[q]);  // stream rows base + RB + q
        __syncthreads();
        if (base + RB - 1 < Wn - 1) continue;  // no complete window in this round (uniform)
        for (int t = j; t < RB * NF * (kGfThreads / kGfRun); t += kGfThreads) hsum_task<R>(vbuf, hbuf, t);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < RB; ++q) {
          const int it = base + q;
          const int y = ybase + it - R, x = x0 - R + j;
          if (it < nrows && it >= 2 * R && j >= R && j < TX + R && x < N && y < M && y < y0 + TY) {
            float B[NF];
            float nrm = inv_w2;
            if (CLIP) nrm = __builtin_amdgcn_rcpf((float)(clip_count<R>(y, M) * ncol));
#pragma unroll
            for (int f = 0; f < NF; ++f)
              B[f] = hbuf[(q * NF + f) * kHsOut + hs_col(j)] * (CLIP && ((Op::kT >> f) & 1u) ? 1.0f : nrm);
            Op::emit(d, (size_t)y * N + x, B, er[q], ee[q], cI, cP, eacc);
          }
        }
        // the next round's first barrier orders these hbuf reads before hbuf is rewritten
      }
    }
    if (Op::kEps) {
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) eacc += __shfl_xor(eacc, off, 64);
      __syncthreads();
      if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = eacc;
      __syncthreads();
      if (threadIdx.x == 0) {
        float h = 0.0f, l = 0.0f;
        for (int w = 0; w < kGfThreads / 64; ++w) df_add(h, l, red[w], 0.0f);
        G(d.geps_part)[wi.blk] = h + l;
      }
    }
    __syncthreads();
  }
}

// The same three stages for windows wider than the strip kernel holds (r > kGfRmax), as
// separable box stages on the image's descriptor; the eps-gradient partials are per image row.
template <class S>
struct WideAdj {
  static constexpr int NF = S::NF, NR = S::NR, NE = S::NE;
  static constexpr unsigned kT = S::kT;
  static constexpr bool kEps = S::kEps;
  __device__ static void load(const WideArgs &a, size_t g, float (&r)[NR]) { S::load(*a.d, g, r); }
  __device__ static void eload(const WideArgs &a, size_t g, float (&e)[NE]) { S::eload(*a.d, g, e); }
  __device__ static void fields(const float (&r)[NR], const float (&c)[4], float (&v)[NF]) {
    S::fields(r, c[0], c[1], v);
  }
  __device__ static void emit(const WideArgs &a, size_t g, const float (&B)[NF], const float (&r)[NR],
                              const float (&e)[NE], const float (&c)[4], float &eacc) {
    S::emit(*a.d, g, B, r, e, c[0], c[1], eacc);
  }
};

static hipError_t launch_box_wide(const ImgSet &set, int i, int stage, hipStream_t s) {
  const Img &d = set.imgs[i];
  WideArgs a = {};
  a.d = set.dev + i;
  a.V = d.wV;
  a.eps_part = d.geps_part;
  a.cen[0] = state_field(d.st, offsetof(LamState, meanI));
  a.cen[1] = state_field(d.st, offsetof(LamState, meanP));
  a.M = d.L.M;
  a.N = d.L.N;
  a.r = (d.w - 1) / 2;
  a.clip = d.clip;
  a.eps = d.eps;
  if (stage == 1) return wide_stage<WideAdj<BoxStage1>>(a, s);
  if (stage == 2) return wide_stage<WideAdj<BoxStage2>>(a, s);
  return wide_stage<WideAdj<BoxStage3>>(a, s);
}

// ============================================================================ lambda of the replayed iteration
// The forward's lambda history drives the recomputation: lambda, lambda* and the flags of
// iteration k.
__global__ void k_lam_replay(const Img *__restrict__ D, const Item *__restrict__ W, int nitems, int k) {
  for (int ii = blockIdx.x; ii < nitems; ii += gridDim.x) {
    const Item wi = W[ii];
    if (wi.blk < 0 || threadIdx.x != 0) continue;
    const Img &d = D[wi.img];
    const float lam = d.lam_hist[k];
    d.st->lam = lam;
    d.st->lam_star = d.lam_star_hist[k];
    d.st->flags = d.flag_hist[k];
    if (d.ad != nullptr) d.ad->skip = isinf(lam) ? 1 : 0;
  }
}

// Points the replay descriptors of every image at segment position j, so that the replay of an
// iteration writes u_I, u_p and U_E there (and its filter the first box pass's results, where it
// runs) and its adjoint reads them there (no copies).  dir > 0 also saves the centring constants
// the replay has just computed, dir < 0 restores them.
__global__ void k_bwd_bind(Img *__restrict__ D, int count, const BwdSlot *__restrict__ slots, int nslot, int j,
                           int dir) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const BwdSlot sl = slots[(size_t)i * nslot + j];
  Img &d = D[i];
  d.uI = sl.uI;
  d.uP = sl.uP;
  d.S1 = sl.S1;
  d.ga = sl.ga;
  d.gmu = sl.gmu;
  d.gpb = sl.gpb;
  d.gve = sl.gve;
  if (dir > 0) {
    sl.means[0] = d.st->meanI;
    sl.means[1] = d.st->meanP;
  } else if (dir < 0) {
    d.st->meanI = sl.means[0];
    d.st->meanP = sl.means[1];
  }
}

// ============================================================================ spectral adjoint
// Per bin of one tile: G = (lambda / dp) G_p + (lambda D2 / dI) G_I and the partial sums of
// g_lambda and of P f'(lambda*).
__global__ void __launch_bounds__(256) k_adj_spec(const Img *__restrict__ D, const Item *__restrict__ W, int nitems) {
  __shared__ float red[4 * 4];
  for (int ii = blockIdx.x; ii < nitems; ii += gridDim.x) {
    const Item wi = W[ii];
    if (wi.blk < 0) continue;
    const Img &d = D[wi.img];
    if (d.ad->skip) continue;
    const Layout &lay = d.L;
    const int C = lay.C, n = lay.M * C;
    const size_t off = (size_t)wi.blk * lay.TS;
    const float lam = d.st->lam, ls = d.st->lam_star, invP = d.st->invP;
    float gl = 0.0f, fp = 0.0f;
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
      const int k = wi.blk * C + (e & (C - 1)), m = e >> lay.logC;
      cf Gt = {0.0f, 0.0f};
      if (k < lay.Wh) {
        const cf U = G(d.S1)[off + e], h = G(d.H)[off + e], yv = G(d.Y)[off + e];
        const float t2 = G(d.H2)[off + e], d2 = G(d.dM)[m] + G(d.dN)[k];
        const cf Rr = cmul(h, U) - yv;
        const cf HR = cmulc(Rr, h);  // conj(H) R
        const cf gi = cscale(G(d.SgI)[off + e], invP), gp = cscale(G(d.SgP)[off + e], invP);
        const float dp = t2 + lam, dI = __fmaf_rn(lam, d2, t2);
        const float mp = lam / dp, mI = lam * d2 / dI;
        Gt = cf{mp * gp.re + mI * gi.re, mp * gp.im + mI * gi.im};
        if (t2 > 0.0f) {
          const float wk = (k == 0 || 2 * k == lay.N) ? 1.0f : 2.0f;
          const float rp = 1.0f / dp, ri = 1.0f / dI;
          gl += wk * ((gp.re * HR.re + gp.im * HR.im) * rp * rp + d2 * (gi.re * HR.re + gi.im * HR.im) * ri * ri);
          const float rs = 1.0f / (t2 + ls);
          fp += wk * abs2f(Rr) * 2.0f * ls * t2 * rs * rs * rs;
        }
      }
      G(d.G)[off + e] = Gt;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      gl += __shfl_xor(gl, o, 64);
      fp += __shfl_xor(fp, o, 64);
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
      red[(threadIdx.x >> 6) * 2] = gl;
      red[(threadIdx.x >> 6) * 2 + 1] = fp;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
      float h = 0.0f, l = 0.0f;
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) df_add(h, l, red[w * 2 + threadIdx.x], 0.0f);
      G(d.part)[(size_t)(2 * threadIdx.x) * d.npart + wi.blk] = h;
      G(d.part)[(size_t)(2 * threadIdx.x + 1) * d.npart + wi.blk] = l;
    }
    __syncthreads();
  }
}

// One block per image: g_lambda, f', the scale gradient, kappa and the eps gradient of
// iteration k.
__global__ void __launch_bounds__(256) k_adj_fin(const Img *__restrict__ D, const Item *__restrict__ W, int nitems,
                                                 int k) {
  __shared__ float scratch[2 * 3 * 4];
  for (int ii = blockIdx.x; ii < nitems; ii += gridDim.x) {
    const Item wi = W[ii];
    if (wi.blk < 0) continue;
    const Img &d = D[wi.img];
    const bool skip = d.ad->skip != 0;
    const int nstrip = (d.L.N + d.bxTX - 1) / d.bxTX * d.bxNBY;
    float hi[3] = {0.0f, 0.0f, 0.0f}, lo[3] = {0.0f, 0.0f, 0.0f};
    if (!skip) {
      for (int p = threadIdx.x; p < d.L.NT; p += blockDim.x) {
        df_add(hi[0], lo[0], G(d.part)[p], G(d.part)[(size_t)d.npart + p]);
        df_add(hi[1], lo[1], G(d.part)[(size_t)2 * d.npart + p], G(d.part)[(size_t)3 * d.npart + p]);
      }
    }
    for (int p = threadIdx.x; p < nstrip; p += blockDim.x) df_add(hi[2], lo[2], G(d.geps_part)[p], 0.0f);
    block_reduce_df<3>(hi, lo, scratch);
    if (threadIdx.x == 0) {
      const LamState *st = d.st;
      d.geps_hist[k] = hi[2] + lo[2];
      if (skip) {
        d.gs_hist[k] = 0.0f;
        d.ad->kappa = 0.0f;
      } else {
        const float glam = hi[0] + lo[0];
        const float fprime = (hi[1] + lo[1]) * st->invP;
        const float s = (d.scales != nullptr && k < st->nscale) ? d.scales[k] : 1.0f;
        d.gs_hist[k] = glam * st->lam_star;
        d.ad->kappa = (st->flags & kFlagNoRoot) || !(fprime > 0.0f) ? 0.0f : -2.0f * st->invP * glam * s / fprime;
      }
    }
    __syncthreads();
  }
}

// Column pass of the adjoint spectrum: G + kappa g conj(H) R, then the unnormalised inverse
// column transform, written row-major to SI (free again once the replayed solves were
// transformed) for the row pass.
__device__ __forceinline__ cf adj_total(const Img &d, size_t i, int k, float kappa, float ls) {
  const cf h = G(d.H)[i];
  const cf Rr = cmul(h, G(d.S1)[i]) - G(d.Y)[i];
  const cf HR = cmulc(Rr, h);
  const float t2 = G(d.H2)[i];
  const float r = ls / (t2 + ls);
  const float c = kappa * r * r;
  const cf g0 = G(d.G)[i];
  return cf{__fmaf_rn(c, HR.re, g0.re), __fmaf_rn(c, HR.im, g0.im)};
}

// LF != 0: the compile-time transform of length M = LF (tiles of col_ls(LF) columns: every
// thread of the block holds a sequence).
template <int LF>
__global__ void __launch_bounds__(512) k_adjcol_r16(const Img *__restrict__ D, const Item *__restrict__ W,
                                                    int nitems) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cf *lds = reinterpret_cast<cf *>(smem_raw);
  for (int ii = blockIdx.x; ii < nitems; ii += gridDim.x) {
    const Item wi = W[ii];
    if (wi.blk < 0) continue;
    const Img &d = D[wi.img];
    if (d.ad->skip) continue;
    const Layout &lay = d.L;
    const int C = lay.C, T = d.rm.T;
    const int c = threadIdx.x & (C - 1), t = threadIdx.x >> lay.logC;
    const bool active = t < T;
    const size_t off = (size_t)wi.blk * lay.TS;
    const int k = wi.blk * C + c;
    const bool valid = active && k < lay.Wh;
    const float kappa = d.ad->kappa, ls = d.st->lam_star;
    cf v[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) v[m] = valid ? adj_total(d, off + (t + T * m) * C + c, k, kappa, ls) : cf{0.0f, 0.0f};
    if constexpr (LF != 0) reg_fft_c<LF, +1, col_ls(LF), false>(v, t, active, lds + c, TwTable{G(d.twB)});
    else reg_fft<+1>(v, t, active, d.rm, lds + c, C, G(d.twM));
    if (active) {
#pragma unroll
      for (int m = 0; m < 16; ++m)
        reinterpret_cast<GFD_AS1 float4 *>(G(d.SIP))[off + (size_t)(t + T * m) * C + c] = make_float4(v[m].re, v[m].im, 0.0f, 0.0f);
    }
    __syncthreads();
  }
}

template <int E>
__global__ void __launch_bounds__(1024) k_adjcol_g(const Img *__restrict__ D, const Item *__restrict__ W, int nitems) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cf *buf = reinterpret_cast<cf *>(smem_raw);
  for (int ii = blockIdx.x; ii < nitems; ii += gridDim.x) {
    const Item wi = W[ii];
    if (wi.blk < 0) continue;
    const Img &d = D[wi.img];
    if (d.ad->skip) continue;
    const Layout &lay = d.L;
    const int C = lay.C, n = lay.M * C;
    const size_t off = (size_t)wi.blk * lay.TS;
    const float kappa = d.ad->kappa, ls = d.st->lam_star;
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
      const int k = wi.blk * C + (e & (C - 1));
      buf[e] = k < lay.Wh ? adj_total(d, off + e, k, kappa, ls) : cf{0.0f, 0.0f};
    }
    __syncthreads();
    lds_fft<float, E, +1, true>(buf, C, lay.logC, C, 1, d.pm, G(d.twM));
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
      reinterpret_cast<GFD_AS1 float4 *>(G(d.SIP))[off + e] = make_float4(buf[e].re, buf[e].im, 0.0f, 0.0f);
    }
    __syncthreads();
  }
}

// lambda = +inf on this iteration: the solves were the identity, g_uE = g_I + g_p.
__global__ void __launch_bounds__(256) k_adj_inf(const Img *__restrict__ D, const Item *__restrict__ W, int nitems) {
  for (int ii = blockIdx.x; ii < nitems; ii += gridDim.x) {
    const Item wi = W[ii];
    if (wi.blk < 0) continue;
    const Img &d = D[wi.img];
    if (!d.ad->skip) continue;
    const size_t P = (size_t)d.L.M * d.L.N;
    const size_t i0 = (size_t)wi.blk * 4096;
    for (size_t i = i0 + threadIdx.x; i < i0 + 4096 && i < P; i += blockDim.x) G(d.gu)[i] = G(d.gI)[i] + G(d.gP)[i];
  }
}

// Sum of the per-iteration eps gradients (FP64) and the scale gradients of every image, for
// iterations k0 .. k0 + K - 1.
__global__ void k_adj_out(const Img *__restrict__ D, const Item *__restrict__ W, int nitems, int K, int k0,
                          float *geps_out, float *gs_out) {
  for (int ii = blockIdx.x; ii < nitems; ii += gridDim.x) {
    const Item wi = W[ii];
    if (wi.blk < 0) continue;
    const Img &d = D[wi.img];
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int k = 0; k < K; ++k) s += (double)d.geps_hist[k0 + k];
      if (geps_out != nullptr) geps_out[wi.img] = (float)s;
    }
    if (gs_out != nullptr)
      for (int k = threadIdx.x; k < K; k += blockDim.x) gs_out[(size_t)wi.img * K + k] = d.gs_hist[k0 + k];
  }
}

// ============================================================================ host side
void adj_geometry(Img &d) {
  const int R = (d.w - 1) / 2;
  if (R > kGfRmax) {  // separable passes: one eps-gradient partial per image row
    d.bxTX = d.L.N;
    d.bxTY = 1;
    d.bxNBY = d.L.M;
    return;
  }
  d.bxTX = std::min(kGfThreads - 2 * R, d.L.N);
  d.bxTY = std::min(64, d.L.M);
  d.bxNBY = (d.L.M + d.bxTY - 1) / d.bxTY;
}

int adj_strips(const Img &d) { return (d.L.N + d.bxTX - 1) / d.bxTX * d.bxNBY; }

#define GFD_R_CASES(X) \
  X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8)

void plan_box_stage(Plan &p, ImgSet &set, const std::vector<int> &sel, int stage) {
  std::map<int, std::vector<int>> byR;  // key 2 r + clip
  for (int i : sel) byR[(set.imgs[i].w - 1) + (set.imgs[i].clip ? 1 : 0)].push_back(i);
  for (auto &kv : byR) {
    if (kv.first / 2 > kGfRmax) {
      ImgSet *setp = &set;
      for (int i : kv.second)
        p.steps.push_back([setp, i, stage](hipStream_t s) { return launch_box_wide(*setp, i, stage, s); });
      continue;
    }
    ItemRange r = add_items(set, kv.second, [](const Img &d) { return adj_strips(d); });
    const int R = kv.first / 2;
    const bool clip = (kv.first & 1) != 0;
#define GFD_BOX_ONE(RR, OP) \
  p.steps.push_back(make_launch(&set, clip ? k_box_stage<RR, OP, true> : k_box_stage<RR, OP, false>, r, kGfThreads, 0))
#define GFD_BOX_CASE(RR)                      \
  if (R == RR) {                              \
    if (stage == 1) GFD_BOX_ONE(RR, BoxStage1); \
    if (stage == 2) GFD_BOX_ONE(RR, BoxStage2); \
    if (stage == 3) GFD_BOX_ONE(RR, BoxStage3); \
  }
    GFD_R_CASES(GFD_BOX_CASE)
#undef GFD_BOX_CASE
#undef GFD_BOX_ONE
  }
}

void plan_adj_spec(Plan &p, ImgSet &set, const std::vector<int> &sel) {
  ItemRange r = add_items(set, sel, [](const Img &d) { return d.L.NT; });
  p.steps.push_back(make_launch(&set, k_adj_spec, r, 256, 0));
}

static int adj_pick_E(size_t elems, int &threads) {
  threads = 256;
  while ((size_t)threads * 16 < elems && threads < 1024) threads *= 2;
  const size_t e = (elems + threads - 1) / threads;
  return e <= 4 ? 4 : e <= 8 ? 8 : 16;
}

void plan_adj_col(Plan &p, ImgSet &set, const std::vector<int> &sel) {
  std::map<std::pair<int, int>, std::vector<int>> groups;  // (threads, E); threads = 0: register-resident
                                                           // (E = M: the compile-time transform)
  for (int i : sel) {
    const Img &d = set.imgs[i];
    if (reg_plan_ok(d.L.M)) {
      groups[{0, d.L.C == col_ls(d.L.M) ? d.L.M : 0}].push_back(i);
    } else {
      int th;
      const int E = adj_pick_E((size_t)d.L.M * d.L.C, th);
      groups[{th, E}].push_back(i);
    }
  }
  for (auto &kv : groups) {
    ItemRange r = add_items(set, kv.second, [](const Img &d) { return d.L.NT; });
    int threads = kv.first.first;
    const int E = kv.first.second;
    size_t lds = 0;
    if (kv.first.first == 0) {
      for (int i : kv.second) {
        const Img &d = set.imgs[i];
        threads = std::max(threads, d.L.C * d.rm.T);
        lds = std::max(lds, (size_t)d.L.C * (d.L.M + d.L.M / 16) * sizeof(cf));
      }
      auto kern = k_adjcol_r16<0>;
      switch (E) {
        case 4096: kern = k_adjcol_r16<4096>; break;
        case 2048: kern = k_adjcol_r16<2048>; break;
        case 1024: kern = k_adjcol_r16<1024>; break;
        case 512: kern = k_adjcol_r16<512>; break;
        case 256: kern = k_adjcol_r16<256>; break;
        default: break;
      }
      p.steps.push_back(make_launch(&set, kern, r, threads, lds));
    } else {
      for (int i : kv.second) lds = std::max(lds, (size_t)set.imgs[i].L.M * set.imgs[i].L.C * sizeof(cf));
      p.steps.push_back(make_launch(&set, E == 4 ? k_adjcol_g<4> : E == 8 ? k_adjcol_g<8> : k_adjcol_g<16>, r,
                                    threads, lds));
    }
  }
}

void plan_adj_inf(Plan &p, ImgSet &set, const std::vector<int> &sel) {
  ItemRange r = add_items(set, sel, [](const Img &d) { return (int)(((size_t)d.L.M * d.L.N + 4095) / 4096); });
  p.steps.push_back(make_launch(&set, k_adj_inf, r, 256, 0));
}

ItemRange plan_one_per_image(ImgSet &set, const std::vector<int> &sel) {
  return add_one_per_image(set, sel);
}

hipError_t launch_lam_replay(ImgSet &set, ItemRange one, int k, hipStream_t s) {
  return make_launch(&set, k_lam_replay, one, 64, 0, k)(s);
}

hipError_t launch_bwd_bind(ImgSet &set, const BwdSlot *slots, int nslot, int j, int dir, hipStream_t s) {
  const int n = (int)set.imgs.size();
  hipLaunchKernelGGL(k_bwd_bind, dim3((n + 63) / 64), dim3(64), 0, s, set.dev, n, slots, nslot, j, dir);
  return hipGetLastError();
}

hipError_t launch_adj_fin(ImgSet &set, ItemRange one, int k, hipStream_t s) {
  return make_launch(&set, k_adj_fin, one, 256, 0, k)(s);
}

hipError_t launch_adj_out(ImgSet &set, ItemRange one, int K, int k0, float *geps, float *gs, hipStream_t s) {
  return make_launch(&set, k_adj_out, one, 256, 0, K, k0, geps, gs)(s);
}

}  // namespace gfd
