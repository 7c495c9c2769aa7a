// Guided filter u = guidfilter(u_I, u_p, w, eps) on gfx950 (Sec. 2, Eqs.(3)-(5)).
//
// One block owns a strip of TX output columns and TY output rows and streams down its rows,
// RB rows per round of barriers.  Every thread owns one column of the strip extended by 2r on
// each side (r = (w-1)/2):
//   stage 1: vertical running sums over the last w rows of I, p, I*I, I*p (FP32, summed afresh
//            from the register ring once every w rows and slid by one row in between, so that
//            rounding errors never accumulate over more than w slides), then horizontal sliding
//            sums across the block's columns (LDS) -> w x w window sums -> a_k, b_k
//            (Eqs.(3)-(4)) for one row of windows;
//   stage 2: the same two-direction sums over a and b -> abar, bbar (Eq.(5)), then
//            u = abar * I + bbar.
// The inputs of the last w rows and the coefficients of the last w rows of windows stay in
// per-thread register rings, so nothing is loaded twice.  Windows wrap periodically in both
// directions.  Inputs are shifted by constants
// (the image means when known) before products are formed; the filter commutes with such
// shifts (u shifts by the input's constant).  The radius is a template parameter so that the
// horizontal sums unroll into back-to-back LDS reads.
//
// With CLIP, windows are clipped to the image instead of wrapping: pixels outside the image
// enter the sums as zeros, every mean divides by the number of the window's pixels inside the
// image, and windows centred outside the image contribute no coefficients.
//
// Windows wider than the register rings hold (r > kGfRmax) run as two separable box stages
// (wide_box.h): window means of I, p, I^2, I p -> a, b; window means of a, b -> u.
#include <map>

#include "box_sum.h"
#include "gfd_internal.h"
#include "wide_box.h"

namespace gfd {

// Rows per round of barriers of the filter's streaming strip.  Four for the two widest radii
// (measured at w = 17): one barrier per row, and the second-stage horizontal sums of a round
// occupy every thread; the doubled LDS (about 50 KB) allows three blocks per CU, and with them
// up to 168 VGPRs (at 128, with two rows per round, r = 7 spilled).  Two for the other radii,
// whose registers allow four to six blocks per CU.
template <int R>
constexpr int gf_rows() { return R >= 7 ? 4 : 2; }

// Waves per SIMD the LDS of one strip allows: the occupancy the register allocator aims for.
template <int R>
constexpr int gf_waves() { return gf_rows<R>() == 4 ? 3 : 4; }

// LDS of one strip: RB rows x 4 fields of padded vertical sums and of horizontal sums.
template <int R>
struct GfLds {
  float vbuf[gf_rows<R>() * 4 * hs_pitch<R>()];
  float hbuf[gf_rows<R>() * 4 * kHsOut];
};

// Planes that keep the first stage's results for the reverse mode (Eqs.(3)-(4)): a, the window
// means of I and p, and var + eps, per pixel, in the same mean-centred variables.
struct GfSave {
  float *a, *mu, *pb, *ve;
};

// One strip (logical block lb of an nbx x nby grid of strips, nby strips per column).  FULL:
// the strip uses every thread (TX = kGfThreads - 4R, images at least that wide), so no thread
// needs the selects that zero the sums of columns past a narrow strip.  SAVE: the first stage's
// results of the windows centred on the strip's output pixels also go to `sv` (every pixel of
// the image is an output pixel of exactly one strip).
template <int R, bool CLIP, bool FULL, bool SAVE>
__device__ __forceinline__ void gf_strip(const GFD_AS1 float *__restrict__ uI, const GFD_AS1 float *__restrict__ uP,
                                         GFD_AS1 float *__restrict__ u, int M, int N, float eps, int TX, int TY, int nby,
                                         int lb, float cI, float cP, const GfSave &sv, GfLds<R> &sh) {
  // No contraction of separate multiplies and additions into fused ones: every fused operation
  // is written out, so the arithmetic is the same in every instantiation (with and without SAVE,
  // whatever the compiler's choices), and the reverse mode's replays reproduce the forward
  // filter bit for bit.
#pragma clang fp contract(off)
  constexpr int W = 2 * R + 1;
  constexpr int RB = gf_rows<R>();
  constexpr int VP = hs_pitch<R>();  // padded row of vertical sums
  float *__restrict__ vbuf = sh.vbuf;
  float *__restrict__ hbuf = sh.hbuf;
  hs_zero_pads<R>(vbuf, RB * 4);  // ordered before the first reads by the first barrier
  const float inv_w2 = 1.0f / (float)(W * W);
  const int bx = lb / nby, by = lb - bx * nby;
  const int x0 = bx * TX, y0 = by * TY;
  const int j = gf_col(threadIdx.x);  // the strip column this thread owns
  const int used = TX + 4 * R;
  const bool active = FULL || j < used;
  const int gx = wrap(x0 - 2 * R + j, N);
  // Stream rows it = 0 .. nrows-1 run down the strip's rows (and the 2R halo rows on each side)
  // in strips with even `by` and up in the others: neighbouring strips then read the 4R halo rows
  // they share at the same time (both at their starts, or both at their ends), so the second
  // read finds them in L2.  The windows are symmetric, so only the order of the sums changes.
  const int nrows = TY + 4 * R;
  const int dir = (by & 1) ? -1 : 1;
  const int ybase = dir > 0 ? y0 - 2 * R : y0 + TY - 1 + 2 * R;  // image row of stream row 0
  auto yrow = [&](int it) { return ybase + dir * it; };
  // CLIP: whether this thread's column lies in the image, and the reciprocal column count of
  // the windows centred on it (stage-1 coefficients and stage-2 outputs share the column)
  const int xcol = x0 - 2 * R + j;
  const bool colin = !CLIP || (xcol >= 0 && xcol < N);
  const int ncol = CLIP && colin ? clip_count<R>(xcol, N) : 1;
  const int cj = hs_col(j + R), hj = hs_col(j);  // this column in the rows of vertical / horizontal sums

  // Each thread keeps, in registers, the mean-centred I and p of the last RS >= W stream rows of
  // its column (slot it % RS) and the coefficients (a, b) of the last RS rows of windows centred
  // on it (slot it2 % RS), so rows leaving the windows and the guide value of the output row
  // (stream row it - 2r, still in the ring) are never loaded or recomputed.  RS is W rounded up
  // to a multiple of RB: the row loop is unrolled over RS rows (RS / RB rounds), which makes
  // every ring slot a compile-time index with a short unrolled body (RB W rows with RS = W had
  // the register allocator shuffle the rings).  Loads run one round ahead: a round first
  // consumes the rows loaded during the previous round, then issues the next loads, and only
  // then does its LDS work.
  // Rows are fetched in stream order; the wrapped image row of the next fetch is carried from
  // one fetch to the next (a step of one row and a compare, no division per row), and stream
  // rows past the end repeat the last row.
  int f_it = 0, f_row = wrap(ybase, M);
  auto fetch_next = [&](float &I, float &p) {
    const uint32_t g = (uint32_t)f_row * (uint32_t)N + (uint32_t)gx;
    I = E(uI, g);
    p = E(uP, g);
    if (f_it < nrows - 1) {
      ++f_it;
      f_row += dir;
      if (f_row == M) f_row = 0;
      if (f_row < 0) f_row = M - 1;
    }
  };
  constexpr int RS = (W + RB - 1) / RB * RB;
  float sI = 0.0f, sP = 0.0f, sII = 0.0f, sIP = 0.0f, sA = 0.0f, sB = 0.0f;
  float rI[RS], rP[RS], rA[RS], rB[RS];  // slots not yet written hold zeros (rows before the stream)
#pragma unroll
  for (int k = 0; k < RS; ++k) rI[k] = rP[k] = rA[k] = rB[k] = 0.0f;
  float nI[RB], nP[RB];
#pragma unroll
  for (int q = 0; q < RB; ++q) fetch_next(nI[q], nP[q]);  // stream rows 0 .. RB - 1
  for (int base0 = 0; base0 < nrows; base0 += RS) {
#pragma unroll
    for (int r = 0; r < RS / RB; ++r) {
      const int base = base0 + RB * r;
      if (base >= nrows) break;  // uniform
      float Ig[RB];
      // ---- stage 1, vertical
#pragma unroll
      for (int q = 0; q < RB; ++q) {
        // slots (base0 is a multiple of RS): this row, the row leaving the window (it - W) and
        // the guide of this round's output row (it - 2r)
        const int s = RB * r + q, so = (RB * r + q - W + RS) % RS, sg = (RB * r + q - 2 * R + RS) % RS;
        float I = __fsub_rn(nI[q], cI), p = __fsub_rn(nP[q], cP);
        if (CLIP) {
          const int y = yrow(base + q);
          if (!(colin && y >= 0 && y < M)) I = p = 0.0f;  // outside the image: no contribution
        }
        const float Io = rI[so], po = rP[so];  // stream row it - W (zero while it < W)
        rI[s] = I;
        rP[s] = p;
        Ig[q] = rI[sg];
        float *vb = vbuf + q * 4 * VP + cj;
        // Threads past the strip's columns (narrow images) run the same arithmetic on their
        // clamped, finite inputs and store zeros: a select per value, no divergent branch.
        if (base + q < nrows) {  // uniform
          if (s == RS - 1) {  // slots RS - W .. RS - 1 hold the window's W rows: sum them afresh
            sI = sP = sII = sIP = 0.0f;
#pragma unroll
            for (int k = RS - W; k < RS; ++k) {
              sI = __fadd_rn(sI, rI[k]);
              sP = __fadd_rn(sP, rP[k]);
              sII = __fmaf_rn(rI[k], rI[k], sII);
              sIP = __fmaf_rn(rI[k], rP[k], sIP);
            }
          } else {
            // I^2 - Io^2 = (I - Io)(I + Io) and I p - Io po = (I - Io) p + Io (p - po): the
            // differences of the first two sums feed the other two (eight operations, not twelve)
            const float dI = __fsub_rn(I, Io), dP = __fsub_rn(p, po);
            sI = __fadd_rn(sI, dI);
            sP = __fadd_rn(sP, dP);
            sII = __fmaf_rn(dI, __fadd_rn(I, Io), sII);
            sIP = __fmaf_rn(dI, p, __fmaf_rn(Io, dP, sIP));
          }
          vb[0] = active ? sI : 0.0f;
          vb[VP] = active ? sP : 0.0f;
          vb[2 * VP] = active ? sII : 0.0f;
          vb[3 * VP] = active ? sIP : 0.0f;
        } else {
          vb[0] = vb[VP] = vb[2 * VP] = vb[3 * VP] = 0.0f;
        }
      }
#pragma unroll
      for (int q = 0; q < RB; ++q) fetch_next(nI[q], nP[q]);  // stream rows base + RB + q
      __syncthreads();
      if (base + RB - 1 < W - 1) continue;  // no complete window in this round (uniform)
      // ---- stage 1, horizontal: RB rows x 4 quantities
#pragma unroll
      for (int t = threadIdx.x; t < RB * 4 * (kGfThreads / kGfRun); t += kGfThreads) hsum_task<R>(vbuf, hbuf, t);
      __syncthreads();
      // ---- a, b (Eqs. 3-4) and stage 2, vertical
#pragma unroll
      for (int q = 0; q < RB; ++q) {
        const int it = base + q;
        const int it2 = it - (W - 1);  // row index of (a, b) in the stage-2 stream
        float *vb = vbuf + q * 2 * VP + cj;
        const bool cvalid = j >= R && j < used - R;  // columns with coefficients (selects below)
        if (it < nrows && it2 >= 0) {  // uniform
          const float *hb = hbuf + q * 4 * kHsOut + hj;
          float nrm = inv_w2;
          bool cin = true;
          if (CLIP) {  // window centred at image row yrow(it - R), column xcol
            const int yc = yrow(it - R);
            cin = colin && yc >= 0 && yc < M;
            nrm = cin ? __builtin_amdgcn_rcpf((float)(clip_count<R>(yc, M) * ncol)) : 0.0f;
          }
          const float mu = hb[0] * nrm;
          const float pb = hb[kHsOut] * nrm;
          const float var = fmaxf(__fmaf_rn(-mu, mu, hb[2 * kHsOut] * nrm), 0.0f);
          const float cov = __fmaf_rn(-mu, pb, hb[3 * kHsOut] * nrm);
          const float ve = var + eps;
          const float rv = __builtin_amdgcn_rcpf(ve);  // hardware reciprocal, 1 ulp
          float a = cov * rv;
          float b = __fmaf_rn(-a, mu, pb);
          if (CLIP && !cin) a = b = 0.0f;  // windows centred outside the image do not exist
          if (SAVE) {  // window centred at image row yrow(it - R), column x0 - 2R + j
            const int yc = yrow(it - R), xc = x0 - 2 * R + j;
            if (j >= 2 * R && j < TX + 2 * R && xc < N && yc >= y0 && yc < y0 + TY && yc < M) {
              const uint32_t g = (uint32_t)yc * (uint32_t)N + (uint32_t)xc;
              E(G(sv.a), g) = a;
              E(G(sv.mu), g) = mu;
              E(G(sv.pb), g) = pb;
              E(G(sv.ve), g) = ve;
            }
          }
          // slots of it2 and of it2 - W (zero while it2 < W)
          const int slot = (RB * r + q - (W - 1) + RS) % RS, slo = (RB * r + q - (W - 1) - W + 2 * RS) % RS;
          const float ao = rA[slo], bo = rB[slo];
          rA[slot] = a;
          rB[slot] = b;
          if (slot == RS - 1) {  // slots RS - W .. RS - 1: rows it2 - W + 1 .. it2 of coefficients
            sA = sB = 0.0f;
#pragma unroll
            for (int k = RS - W; k < RS; ++k) {
              sA = __fadd_rn(sA, rA[k]);
              sB = __fadd_rn(sB, rB[k]);
            }
          } else {
            // a - ao as one fused operation, cov rv - ao
            sA = __fadd_rn(sA, (CLIP && !cin) ? -ao : __fmaf_rn(cov, rv, -ao));
            slide(sB, b, bo);
          }
          // Columns without coefficients still enter the first window of a sliding run before
          // they are subtracted again: they hold zeros, never a stale (large) stage-1 sum.
          vb[0] = cvalid ? sA : 0.0f;
          vb[VP] = cvalid ? sB : 0.0f;
        } else {
          vb[0] = 0.0f;
          vb[VP] = 0.0f;
        }
      }
      __syncthreads();
      if (base + RB - 1 < 4 * R) continue;  // no complete stage-2 window yet (uniform)
      // ---- stage 2, horizontal: RB rows x 2 quantities
#pragma unroll
      for (int t = threadIdx.x; t < RB * 2 * (kGfThreads / kGfRun); t += kGfThreads) hsum_task<R>(vbuf, hbuf, t);
      __syncthreads();
      // ---- output rows
#pragma unroll
      for (int q = 0; q < RB; ++q) {
        const int it = base + q;
        const int yo = yrow(it - 2 * R);  // output row
        const int xo = x0 - 2 * R + j;      // output column
        if (it < nrows && it >= 4 * R && j >= 2 * R && j < TX + 2 * R && xo < N && yo < M && yo < y0 + TY) {
          const float *hb = hbuf + q * 2 * kHsOut + hj;
          const float nrm = CLIP ? __builtin_amdgcn_rcpf((float)(clip_count<R>(yo, M) * ncol)) : inv_w2;
          const float abar = hb[0] * nrm, bbar = hb[kHsOut] * nrm;
          E(u, (uint32_t)yo * (uint32_t)N + (uint32_t)xo) = __fadd_rn(__fmaf_rn(abar, Ig[q], bbar), cP);
        }
      }
      // the next round's first barrier orders these hbuf reads before hbuf is rewritten
    }
  }
}

// Inside the iteration: one launch filters every image of the group (images of one radius).
// SAVE (the reverse mode's replays): the first stage's results go to the image's ga, gmu, gpb
// and gve planes as well.
template <int R, bool CLIP, bool SAVE = false>
__global__ void __launch_bounds__(kGfThreads) __attribute__((amdgpu_waves_per_eu(gf_waves<R>()))) k_gf_g(const Img *__restrict__ D, const Item *__restrict__ W,
                                                     int nitems) {
  __shared__ __align__(16) GfLds<R> sh;
  for (int ii = blockIdx.x; ii < nitems; ii += gridDim.x) {
    const Item wi = W[ii];
    if (wi.blk < 0) continue;
    const Img &d = D[wi.img];
    const float cI = d.st->meanI, cP = d.st->meanP;
    const GfSave sv = {d.ga, d.gmu, d.gpb, d.gve};
    if (d.gfTX + 4 * R == kGfThreads)
      gf_strip<R, CLIP, true, SAVE>(G(d.uI), G(d.uP), G(d.uE), d.L.M, d.L.N, d.eps, d.gfTX, d.gfTY, d.gfNBY, wi.blk, cI,
                                    cP, sv, sh);
    else
      gf_strip<R, CLIP, false, SAVE>(G(d.uI), G(d.uP), G(d.uE), d.L.M, d.L.N, d.eps, d.gfTX, d.gfTY, d.gfNBY, wi.blk, cI,
                                     cP, sv, sh);
    __syncthreads();
  }
}

// Stand-alone filter: the offsets are the first pixels of the inputs.
template <int R, bool CLIP>
__global__ void __launch_bounds__(kGfThreads) __attribute__((amdgpu_waves_per_eu(gf_waves<R>()))) k_gf_plain(const float *__restrict__ uI, const float *__restrict__ uP,
                                                         float *__restrict__ u, int M, int N, float eps, int TX,
                                                         int TY, int nby) {
  __shared__ __align__(16) GfLds<R> sh;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const GfSave none = {};
  if (TX + 4 * R == kGfThreads)
    gf_strip<R, CLIP, true, false>(G(uI), G(uP), G(u), M, N, eps, TX, TY, nby, lb, uI[0], uP[0], none, sh);
  else gf_strip<R, CLIP, false, false>(G(uI), G(uP), G(u), M, N, eps, TX, TY, nby, lb, uI[0], uP[0], none, sh);
}

bool guided_filter_supported(int w) { return w >= 1 && (w % 2) == 1; }
bool gf_wide(int w) { return (w - 1) / 2 > kGfRmax; }

// ---------------------------------------------------------------- windows of any width
// The two stages of the filter as separable box stages, in the same mean-centred variables as
// the strip kernel (src = {u_I, u_p}, dst = {a, b}, cen = {centre of u_I, centre of u_p}).
struct WideGf1 {  // window means of I, p, I^2, I p  ->  a, b (Eqs. 3-4)
  static constexpr int NF = 4, NR = 2, NE = 1;
  static constexpr unsigned kT = 0u;
  static constexpr bool kEps = false;
  __device__ static void load(const WideArgs &a, size_t g, float (&r)[NR]) {
    r[0] = a.src[0][g];
    r[1] = a.src[1][g];
  }
  __device__ static void eload(const WideArgs &, size_t, float (&e)[NE]) { e[0] = 0.0f; }
  __device__ static void fields(const float (&r)[NR], const float (&c)[4], float (&v)[NF]) {
    const float I = __fsub_rn(r[0], c[0]), p = __fsub_rn(r[1], c[1]);
    v[0] = I;
    v[1] = p;
    v[2] = I * I;
    v[3] = I * p;
  }
  __device__ static void emit(const WideArgs &a, size_t g, const float (&B)[NF], const float (&)[NR],
                              const float (&)[NE], const float (&)[4], float &) {
    const float mu = B[0], pb = B[1];
    const float var = fmaxf(__fmaf_rn(-mu, mu, B[2]), 0.0f);
    const float cov = __fmaf_rn(-mu, pb, B[3]);
    const float A = cov * __builtin_amdgcn_rcpf(var + a.eps);
    a.dst[0][g] = A;
    a.dst[1][g] = __fmaf_rn(-A, mu, pb);
  }
};

struct WideGf2 {  // window means of a, b  ->  u = abar I + bbar (Eq. 5)
  static constexpr int NF = 2, NR = 2, NE = 1;
  static constexpr unsigned kT = 0u;
  static constexpr bool kEps = false;
  __device__ static void load(const WideArgs &a, size_t g, float (&r)[NR]) {
    r[0] = a.dst[0][g];
    r[1] = a.dst[1][g];
  }
  __device__ static void eload(const WideArgs &a, size_t g, float (&e)[NE]) { e[0] = a.src[0][g]; }
  __device__ static void fields(const float (&r)[NR], const float (&)[4], float (&v)[NF]) {
    v[0] = r[0];
    v[1] = r[1];
  }
  __device__ static void emit(const WideArgs &a, size_t g, const float (&B)[NF], const float (&)[NR],
                              const float (&e)[NE], const float (&c)[4], float &) {
    a.out[g] = __fadd_rn(__fmaf_rn(B[0], __fsub_rn(e[0], c[0]), B[1]), c[1]);
  }
};

static hipError_t launch_gf_wide(const WideArgs &a, hipStream_t s) {
  hipError_t e = wide_stage<WideGf1>(a, s);
  return e == hipSuccess ? wide_stage<WideGf2>(a, s) : e;
}

// The filter of image i of a descriptor set as separable passes, centred like the strip kernel
// (the image means kept in its lambda state); guide, input and output come from the set's
// device table when the kernels run.
static WideArgs gf_wide_args(const ImgSet &set, int i) {
  const Img &d = set.imgs[i];
  WideArgs a = {};
  a.d = set.dev + i;
  a.table = 1;
  a.dst[0] = d.wa;
  a.dst[1] = d.wb;
  a.V = d.wV;
  a.cen[0] = state_field(d.st, offsetof(LamState, meanI));
  a.cen[1] = state_field(d.st, offsetof(LamState, meanP));
  a.M = d.L.M;
  a.N = d.L.N;
  a.r = (d.w - 1) / 2;
  a.clip = d.clip;
  a.eps = d.eps;
  return a;
}

static void gf_tiles(int M, int N, int R, int ty, int &TX, int &TY, int &nbx, int &nby) {
  TX = kGfThreads - 4 * R;
  if (TX > N) TX = N;
  TY = ty > 0 ? ty : 64;
  if (TY > M) TY = M;
  nbx = (N + TX - 1) / TX;
  nby = (M + TY - 1) / TY;
}

void gf_geometry(Img &d, int ty) {
  if (gf_wide(d.w)) {  // separable passes: no strips
    d.gfTX = d.L.N;
    d.gfTY = d.L.M;
    d.gfNBY = 1;
    return;
  }
  int nbx;
  gf_tiles(d.L.M, d.L.N, (d.w - 1) / 2, ty, d.gfTX, d.gfTY, nbx, d.gfNBY);
}


#define GFD_R_SWITCH(r, X)                                                                                  \
  switch (r) {                                                                                              \
    case 0: X(0); break;                                                                                    \
    case 1: X(1); break;                                                                                    \
    case 2: X(2); break;                                                                                    \
    case 3: X(3); break;                                                                                    \
    case 4: X(4); break;                                                                                    \
    case 5: X(5); break;                                                                                    \
    case 6: X(6); break;                                                                                    \
    case 7: X(7); break;                                                                                    \
    case 8: X(8); break;                                                                                    \
    default: break;                                                                                         \
  }

// The lowest strip height (a multiple of 8, at least 32) whose strips of one image all fit on
// the device at once (one wave of resident blocks); 0 if none does.  Taller strips re-read
// fewer halo rows; more strips than resident blocks leave a second, mostly idle wave.
int gf_fill_height(const Img &d) {
  const int r = (d.w - 1) / 2;
  if (gf_wide(d.w)) return 0;
  int dev = 0, ncu = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  hipError_t e = hipErrorInvalidValue;
#define GFD_OCC(RR)                                                                                   \
  {                                                                                                   \
    auto kern = d.clip ? k_gf_g<RR, true> : k_gf_g<RR, false>;                                        \
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void *)kern, kGfThreads, 0);        \
  }
  GFD_R_SWITCH(r, GFD_OCC)
#undef GFD_OCC
  if (e != hipSuccess || per < 1) return 0;
  const long slots = (long)per * ncu;
  const int TX = kGfThreads - 4 * r, nbx = (d.L.N + TX - 1) / TX;
  for (int ty = 32; ty <= d.L.M; ty += 8)
    if ((long)nbx * ((d.L.M + ty - 1) / ty) <= slots) return ty;
  return 0;
}

void plan_guided_filter(Plan &p, ImgSet &set, const std::vector<int> &sel, bool save) {
  std::map<int, std::vector<int>> byR;  // key 2 r + clip
  for (int i : sel) byR[(set.imgs[i].w - 1) + (set.imgs[i].clip ? 1 : 0)].push_back(i);
  for (auto &kv : byR) {
    sort_by_size(set, kv.second);
    if (kv.first / 2 > kGfRmax) {  // one stream-ordered sequence of separable passes per image
      ImgSet *setp = &set;
      for (int i : kv.second)
        p.steps.push_back([setp, i](hipStream_t s) { return launch_gf_wide(gf_wide_args(*setp, i), s); });
      continue;
    }
    const size_t off = set.items_host.size();
    for (int i : kv.second) {
      const Img &d = set.imgs[i];
      append_items(set, i, (d.L.N + d.gfTX - 1) / d.gfTX * d.gfNBY);
    }
    const size_t n = set.items_host.size() - off;
    const int r = kv.first / 2;
    const bool clip = (kv.first & 1) != 0;
    const ItemRange range{off, n};
#define GFD_PLAN_GF(RR)                                                                              \
  p.steps.push_back(make_launch(&set,                                                                \
                                save ? (clip ? k_gf_g<RR, true, true> : k_gf_g<RR, false, true>)     \
                                     : (clip ? k_gf_g<RR, true, false> : k_gf_g<RR, false, false>),  \
                                range, kGfThreads, 0))
    GFD_R_SWITCH(r, GFD_PLAN_GF)
#undef GFD_PLAN_GF
  }
}

hipError_t launch_guided_filter_plain(const float *uI, const float *uP, float *u, int M, int N, int w, float eps,
                                      bool clip, hipStream_t s) {
  const int r = (w - 1) / 2;
  if (!guided_filter_supported(w)) return hipErrorInvalidValue;
  if (gf_wide(w)) {
    // separable passes: 4 planes of window sums and a, b (and the row prefixes of rows wider
    // than kWideMaxN), stream-ordered temporaries
    const size_t P = (size_t)M * N;
    const size_t npre = N > kWideMaxN ? (size_t)M * (N + 1) : 0;
    float *tmp = nullptr;
    hipError_t e = hipMallocAsync((void **)&tmp, 6 * P * sizeof(float) + npre * sizeof(double), s);
    if (e != hipSuccess) return e;
    WideArgs a = {};
    a.pre = npre ? reinterpret_cast<double *>(tmp + 6 * P) : nullptr;
    a.src[0] = uI;
    a.src[1] = uP;
    a.V = tmp;
    a.dst[0] = tmp + 4 * P;
    a.dst[1] = tmp + 5 * P;
    a.out = u;
    a.cen[0] = uI;  // the first pixels, like the strip kernel
    a.cen[1] = uP;
    a.M = M;
    a.N = N;
    a.r = r;
    a.clip = clip ? 1 : 0;
    a.eps = eps;
    e = launch_gf_wide(a, s);
    const hipError_t ef = hipFreeAsync(tmp, s);
    return e != hipSuccess ? e : ef;
  }
  int TX, TY, nbx, nby;
  gf_tiles(M, N, r, 0, TX, TY, nbx, nby);
#define GFD_LAUNCH_GFP(RR)                                                                          \
  {                                                                                                 \
    auto kern = clip ? k_gf_plain<RR, true> : k_gf_plain<RR, false>;                                \
    hipLaunchKernelGGL(kern, dim3(nbx * nby), dim3(kGfThreads), 0, s, uI, uP, u, M, N, eps, TX, TY, nby); \
  }
  GFD_R_SWITCH(r, GFD_LAUNCH_GFP)
#undef GFD_LAUNCH_GFP
  return hipGetLastError();
}

}  // namespace gfd
