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
// The half spectrum (columns k = 0 .. N/2 of the row transforms) is stored tile-major:
// tile t holds columns [t*C, t*C + C) for all M rows as a contiguous M x C block, element
// (m, c) of tile t at ((t * M) + m) * C + c.  Columns at or beyond Wh are zero padding.
struct Layout {
  int M, N;
  int Wh;         // N / 2 + 1
  int C, logC;    // tile width (power of two)
  int NT;         // number of tiles = ceil(Wh / C)
  int R;          // image rows per block in the LDS-resident row passes (even)
  int Rf, Ri;     // rows per block of the register-resident row passes (forward even, inverse)
  FastDiv Ndiv;   // division by N
  FastDiv RCdiv;  // division by R * C
  FastDiv RfCdiv; // division by Rf * C
  __host__ __device__ size_t bins() const { return (size_t)NT * M * C; }
};

Layout make_layout(int M, int N);
FftPlan make_plan(int L);

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
  const cf *H, *Y, *HY;  // F(h), F(y), conj(F(h)) F(y), tile-major
  const float *H2;       // |F(h)|^2, tile-major
  const float *dM, *dN;  // |F(grad)|^2 = dM[m] + dN[k]
  float *uE, *uI, *uP;   // images (u_E is also the filter's output)
  float *q;              // Hermitian-weighted |R|^2, tile-major
  cf *S1, *SI, *SP;      // spectra: row transforms / U_E, and the two solves
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

// Host-side view of a set of images for building launch plans.  `dev` is the device copy of
// `imgs`; work lists are appended to items_host and uploaded once by finalize_items().
struct ImgSet {
  std::vector<Img> imgs;
  LamState *st_base = nullptr;  // states of the images, imgs[i].st == st_base + i
  Img *dev = nullptr;
  std::vector<Item> items_host;
  Item *items_dev = nullptr;
};

// Plan builders.  `sel` picks images of the set; launches reference set.dev and offsets into
// set.items_dev, so finalize_items() must run before a plan is enqueued.
void plan_row_fwd(Plan &p, ImgSet &set, const std::vector<int> &sel);
void plan_col_fwd(Plan &p, ImgSet &set, const std::vector<int> &sel, bool resid);
void plan_lambda(Plan &p, ImgSet &set, const std::vector<int> &sel, int rounds);
void plan_col_inv(Plan &p, ImgSet &set, const std::vector<int> &sel);
void plan_row_inv(Plan &p, ImgSet &set, const std::vector<int> &sel);
void plan_guided_filter(Plan &p, ImgSet &set, const std::vector<int> &sel, bool close_iteration);
hipError_t finalize_items(ImgSet &set);
void gf_geometry(Img &d);
bool guided_filter_supported(int w);

// Stand-alone guided filter on caller-provided images (context-free).
hipError_t launch_guided_filter_plain(const float *uI, const float *uP, float *u, int M, int N, int w, float eps,
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
hipError_t launch_rho_target(const float *y, int M, int N, const float *h, int kh, int kw, double sigma2,
                             double rho_fixed, double *work, double *out2, LamState *st, hipStream_t st_);
hipError_t launch_fill_f(float *p, size_t n, float v, hipStream_t st);
hipError_t launch_state_reset(LamState *st, hipStream_t s);
hipError_t launch_state_set_lam(LamState *st, float lam, hipStream_t s);
hipError_t launch_copy_lam_star(const LamState *st, float *out, hipStream_t s);
int lam_sweep_chunks(size_t nbins);

}  // namespace gfd
