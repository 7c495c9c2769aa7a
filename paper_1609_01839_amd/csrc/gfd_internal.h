// Internal interface between the C ABI layer and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include <functional>
#include <vector>

#include "fft_lds.h"
#include "fft_reg.h"
#include "lam_search.h"

namespace gfd {

// Geometry of one image and of its half spectrum.
// The half spectrum (columns k = 0 .. N/2 of the row transforms) is stored tile-major: tile t
// holds columns [t*C, t*C + C) for all M rows as a contiguous M x C block, element (m, c) of
// tile t at t * TS + m * C + c.  Columns at or beyond Wh are zero padding.  Tiles start TS >=
// M * C bins apart: where M * C has a large power-of-two factor, a few bins of padding after
// every tile keep the row passes' accesses (a few rows of every tile) from falling on the same
// HBM channels.  Padding bins are never written by the passes and hold zeros.
struct Layout {
  int M, N;
  int Wh;         // N / 2 + 1
  int C, logC;    // tile width (power of two)
  int NT;         // number of tiles = ceil(Wh / C)
  int RP;         // columns of all tiles, NT * C
  int TS;         // bins between the starts of consecutive tiles (>= M * C)
  int R;          // image rows per block in the LDS-resident row passes (even)
  int Rf, Ri;     // rows per block of the register-resident row passes (forward even, inverse)
  FastDiv Ndiv;   // division by N
  FastDiv RCdiv;  // division by R * C
  FastDiv RfCdiv; // division by Rf * C
  // 1: the register-resident residual pass and column inverse fold column N/2 (alone in the
  // last tile) into the block of tile 0 as the imaginary part of column 0, so they launch
  // NT - 1 blocks (the forward pass without the residual launches NT)
  int fold;
  __host__ __device__ int col_blocks() const { return NT - fold; }
  __host__ __device__ size_t bins() const { return (size_t)NT * TS; }
  // tile-major position of bin (m, k): tile k / C, row m, column k % C
  __host__ __device__ size_t tpos(int m, int k) const {
    return (size_t)(k >> logC) * TS + (size_t)m * C + (k & (C - 1));
  }
};

// Launch-shape choices that do not change results (the autotuner's knobs); 0 = default.
struct Tuning {
  int gf_ty = 0;     // rows per guided-filter strip
  int seq_fwd = 0;   // row pairs per block of the register-resident forward row pass
  int seq_inv = 0;   // rows per block of the register-resident inverse row pass
  int rows_lds = 0;  // image rows per block of the LDS-resident (mixed-radix) row passes
  int radix = 0;     // radix schedule of the LDS-resident transforms: 0 (or 8) radix-8 passes, 4 radix-4 passes
};
constexpr int kTuningKnobs = 5;

// LDS pitch (complex slots) of one sequence of the register-resident row passes: the
// transform's padded exchange area plus 8 slots, so that the same position of two sequences
// falls in opposite halves of the LDS banks (the forward pass's split reads both rows of a
// pair, one from each of two sequences, in one access).
__host__ __device__ inline int reg_row_pitch(int N) { return N + N / 16 + 8; }

Layout make_layout(int M, int N, const Tuning &tune = Tuning{});
size_t reg_seq_lds(int N);
bool reg_seqs_ok(int N, int seqs);
FftPlan make_plan(int L, int radix = 0);

constexpr int kLamAccFirst = 2 + 2 * kLamFirstCand;  // Einf, floor, f and slope per candidate
constexpr int kLamAccSweep = 2 * kLamMaxCand;
constexpr int kLamAcc = kLamAccFirst > kLamAccSweep ? kLamAccFirst : kLamAccSweep;

// Everything a kernel needs to know about one image.  Kernels receive a device table of these
// plus a list of work items (image, block); one launch serves every image of a batch.
struct Img {
  Layout L;
  FftPlan pm, pn;        // LDS-resident plans (any 2^a 3^b 5^c length)
  RegPlan rm, rn;        // register-resident plans (power-of-two lengths)
  const cf *twM, *twN;   // twiddles exp(-2 pi i n / L)
  const cf *twB;         // power-of-two M in [256, 4096]: the column transforms' twiddles by
                         // butterfly (kRegTwRows rows of 16, TwTable), null otherwise
  const cf *H, *Y, *HY;  // F(h), F(y), conj(F(h)) F(y), tile-major
  const float *H2;       // |F(h)|^2, tile-major
  const float *dM, *dN;  // |F(grad)|^2 = dM[m] + dN[k]
  float *uE, *uI, *uP;   // images (u_E is also the filter's output)
  float *q;              // Hermitian-weighted |R|^2, tile-major
  cf *S1;                // spectra: row transforms, then U_E
  cf *SIP;               // the two solves after the column inverse, tile-major like S1 and
                         // interleaved: bin (m, k) of tile t = k / C, column c = k % C holds
                         // U_I at SIP[2 e] and U_p at SIP[2 e + 1], e = t TS + m C + c
  float *part;           // partial sums, [2 * kLamAcc][npart]
  int npart;             // stride of `part` (>= NT and >= nchunk)
  int nchunk;            // blocks of a lambda evaluation round
  LamState *st;
  float *lam_hist;
  int *flag_hist;
  const float *scales;
  int hist_cap;
  int w;
  float eps;
  int gfTX, gfTY, gfNBY;  // guided-filter strip geometry
  int clip;               // 1: filter windows clipped to the image (count-normalised means)
  float *lam_star_hist;   // lambda* of each iteration (before the scale)
  // reverse mode (set only in the backward descriptor sets; null otherwise)
  float *ga, *gmu, *gpb, *gve;  // stage 1 of the filter's adjoint: a, mean I, mean p, var + eps
  float *gc, *gd;               // d/dc and the direct term g_u * mean(a)
  float *gu;                    // incoming gradient with respect to the filter output
  float *gI, *gP;               // outgoing gradients with respect to u_I and u_p
  float *geps_part;             // per-strip partial sums of the eps gradient
  cf *SgI, *SgP;                // half spectra of gI and gP
  cf *G;                        // adjoint spectrum with respect to F(u_E)
  struct AdjState *ad;
  float *geps_hist, *gs_hist;   // per-iteration eps gradient and scale gradient
  int bxTX, bxTY, bxNBY;        // strip geometry of the adjoint's box passes
  // windows wider than the strip kernels hold (r > kGfRmax): the separable passes' window sums
  // (4 planes) and the coefficients a, b between the filter's two stages; null otherwise
  float *wV, *wa, *wb;
};

// Per-image scalars of one reverse-mode iteration.
struct AdjState {
  float kappa;  // coefficient of the implicit-lambda term
  int skip;     // 1: lambda = +inf on this iteration (no spectral adjoint)
};

struct Item {
  int img, blk;  // blk < 0: padding item (no work)
};

// A sequence of launches (one per image group and pass) enqueued on a stream.
using Launch = std::function<hipError_t(hipStream_t)>;
struct Plan {
  std::vector<Launch> steps;
  hipError_t enqueue(hipStream_t s) const {
    for (const auto &f : steps) {
      hipError_t e = f(s);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
};

// Device memory carved out of one caller-owned region instead of hipMalloc (the allocation-free
// entry point): 256-byte aligned, bumped, never freed.  A dry arena (base = null) only counts
// the bytes, and copies into it are skipped.
struct Arena {
  unsigned char *base = nullptr;
  size_t cap = 0, off = 0;
  bool dry = false;
  hipError_t take(size_t bytes, void **p) {
    const size_t o = (off + 255) & ~(size_t)255;
    if (o > cap || bytes > cap - o) return hipErrorOutOfMemory;
    *p = base + o;
    off = o + bytes;
    return hipSuccess;
  }
};

// Host-side view of a set of images for building launch plans.  `dev` is the device copy of
// `imgs`; work lists are appended to items_host and uploaded once by finalize_items().  With
// `arena` set, both device tables are carved from it.
struct ImgSet {
  std::vector<Img> imgs;
  LamState *st_base = nullptr;  // states of the images, imgs[i].st == st_base + i
  Img *dev = nullptr;
  std::vector<Item> items_host;
  Item *items_dev = nullptr;
  Arena *arena = nullptr;
  LamQueue *lamq = nullptr;  // work queue of the lambda rounds (zeroed when allocated)
};

template <class K>
inline hipError_t set_lds(K kern, size_t lds) {
  return hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

// Append the work items of one image (blocks 0 .. nblk-1), padded to a multiple of 8 and
// permuted so that every 8th item (one XCD's share: the hardware deals blocks to the 8 XCDs
// in turn) covers a contiguous run of blocks, which then share that XCD's L2.
inline void append_items(ImgSet &set, int img, int nblk, int first = 0) {
  const int nx = 8;
  const int padded = (nblk + nx - 1) / nx * nx;
  const int per = padded / nx;
  for (int i = 0; i < padded; ++i) {
    const int xcd = i % nx, local = i / nx;
    const int blk = xcd * per + local;
    set.items_host.push_back(Item{img, blk < nblk ? first + blk : -1});
  }
}

struct ItemRange {
  size_t off, n;
};

inline ItemRange add_items(ImgSet &set, const std::vector<int> &imgs, const std::function<int(const Img &)> &nblk) {
  ItemRange r{set.items_host.size(), 0};
  for (int i : imgs) append_items(set, i, nblk(set.imgs[i]));
  r.n = set.items_host.size() - r.off;
  return r;
}

// One block per image, without padding (kernels with a single block per image).
inline ItemRange add_one_per_image(ImgSet &set, const std::vector<int> &imgs) {
  ItemRange r{set.items_host.size(), 0};
  for (int i : imgs) set.items_host.push_back(Item{i, 0});
  r.n = set.items_host.size() - r.off;
  return r;
}

// One launch over an item range (grid = number of items, one item per block).  The set's
// tables are read when the launch is enqueued, so it may be built before finalize_items().
template <class K, class... A>
inline Launch make_launch(ImgSet *setp, K kern, ItemRange r, int threads, size_t lds, A... extra) {
  return [=](hipStream_t s) -> hipError_t {
    if (r.n == 0) return hipSuccess;
    if (lds > 48 * 1024) {
      hipError_t e = set_lds(kern, lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)r.n), dim3(threads), lds, s, (const Img *)setp->dev,
                       (const Item *)(setp->items_dev + r.off), (int)r.n, extra...);
    return hipGetLastError();
  };
}

// Plan builders.  `sel` picks images of the set; launches reference set.dev and offsets into
// set.items_dev, so finalize_items() must run before a plan is enqueued.
void plan_row_fwd(Plan &p, ImgSet &set, const std::vector<int> &sel);
void plan_col_fwd(Plan &p, ImgSet &set, const std::vector<int> &sel, bool resid);
void plan_lambda(Plan &p, ImgSet &set, const std::vector<int> &sel, int rounds, bool advance);
void plan_col_inv(Plan &p, ImgSet &set, const std::vector<int> &sel);
void plan_row_inv(Plan &p, ImgSet &set, const std::vector<int> &sel);
// save: the reverse mode's replays, whose filter also writes the first stage's results (a, the
// means of I and p, var + eps) to the images' ga, gmu, gpb and gve planes (strip kernels only;
// windows that run as separable passes write none)
void plan_guided_filter(Plan &p, ImgSet &set, const std::vector<int> &sel, bool save = false);
hipError_t finalize_items(ImgSet &set);
void sort_by_size(const ImgSet &set, std::vector<int> &imgs);
void gf_geometry(Img &d, int ty = 0);
int gf_fill_height(const Img &d);
bool guided_filter_supported(int w);
bool gf_wide(int w);  // the window runs as separable passes (wider than the strip kernels hold)

// Reverse mode (kernels_adj.hip).
void adj_geometry(Img &d);
int adj_strips(const Img &d);
void plan_box_stage(Plan &p, ImgSet &set, const std::vector<int> &sel, int stage);
void plan_adj_spec(Plan &p, ImgSet &set, const std::vector<int> &sel);
void plan_adj_col(Plan &p, ImgSet &set, const std::vector<int> &sel);
void plan_adj_inf(Plan &p, ImgSet &set, const std::vector<int> &sel);
ItemRange plan_one_per_image(ImgSet &set, const std::vector<int> &sel);
hipError_t launch_lam_replay(ImgSet &set, ItemRange one, int k, hipStream_t s);
// Buffers of one segment position of the reverse mode, per image: what the adjoint of an
// iteration reads from its replayed forward pass (u_I, u_p, U_E and the two centring constants).
struct BwdSlot {
  float *uI, *uP, *means;
  cf *S1;
  float *ga, *gmu, *gpb, *gve;  // the first box pass's results for this iteration
};
hipError_t launch_bwd_bind(ImgSet &set, const BwdSlot *slots, int nslot, int j, int dir, hipStream_t s);
hipError_t launch_adj_fin(ImgSet &set, ItemRange one, int k, hipStream_t s);
hipError_t launch_adj_out(ImgSet &set, ItemRange one, int K, int k0, float *geps, float *gs, hipStream_t s);

// Stand-alone guided filter on caller-provided images (context-free).
hipError_t launch_guided_filter_plain(const float *uI, const float *uP, float *u, int M, int N, int w, float eps,
                                      bool clip, hipStream_t s);
hipError_t launch_guided_filter_color(const float *I3, const float *up, float *u, int M, int N, int w, float eps,
                                      hipStream_t s);

// Per-image set-up (FP64 transforms of h and y, constants, rho and the target).
hipError_t launch_embed_psf(const float *h, int kh, int kw, int M, int N, double *hp, hipStream_t st);
hipError_t launch_row_fwd_d(const double *x, const Layout &L, const FftPlan &pn, const cd *twN, cd *S,
                            hipStream_t st);
hipError_t launch_row_fwd_fd(const float *x, const Layout &L, const FftPlan &pn, const cd *twN, cd *S,
                             hipStream_t st);
hipError_t launch_col_fwd_d(cd *S, const Layout &L, const FftPlan &pm, const cd *twM, hipStream_t st);
hipError_t launch_init_consts(const cd *Hd, const cd *Yd, const Layout &L, cf *H, cf *Y, cf *HY, float *H2,
                              hipStream_t st);
hipError_t launch_d2_tables(int M, int N, int Wh, float *dM, float *dN, hipStream_t st);
hipError_t launch_rho_target(const float *y, int M, int N, size_t ndom, const float *h, int kh, int kw,
                             double sigma2, double rho_fixed, double *work, double *out2, LamState *st,
                             hipStream_t s);
hipError_t launch_pad_ramp(const float *y, int M, int N, float *out, int Mp, int Np, hipStream_t st);
hipError_t launch_fill_f(float *p, size_t n, float v, hipStream_t st);
hipError_t launch_state_reset(LamState *st, hipStream_t s);
hipError_t launch_state_set_lam(LamState *st, float lam, hipStream_t s);
hipError_t launch_copy_lam_star(const LamState *st, float *out, hipStream_t s);
hipError_t launch_state_set_nscale(LamState *st, int count, int ns, hipStream_t s);
int lam_sweep_chunks(size_t nbins);

}  // namespace gfd
