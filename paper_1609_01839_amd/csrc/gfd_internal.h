// Internal interface between the C ABI layer and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include "fft_lds.h"
#include "lam_search.h"

namespace gfd {

// Geometry of one image and of its half spectrum.
// The half spectrum (columns k = 0 .. N/2 of the row transforms) is stored tile-major:
// tile t holds columns [t*C, t*C + C) for all M rows as a contiguous M x C block, element
// (m, c) of tile t at ((t * M) + m) * C + c.  Columns at or beyond Wh are zero padding.
struct Layout {
  int M, N;
  int Wh;        // N / 2 + 1
  int C, logC;   // tile width (power of two)
  int NT;        // number of tiles = ceil(Wh / C)
  int R;         // image rows per block in the LDS-resident row passes (even)
  int Rf, Ri;    // rows per block of the register-resident row passes (forward even, inverse)
  FastDiv Ndiv;  // division by N
  FastDiv RCdiv; // division by R * C
  FastDiv RfCdiv;// division by Rf * C
  size_t bins() const { return (size_t)NT * M * C; }
};

Layout make_layout(int M, int N);
FftPlan make_plan(int L);

// Results of the residual pass: per-block partial sums and the bookkeeping to finish them.
struct LamBuffers {
  LamState *st;          // device
  float *partials;       // device, [blocks][kLamAcc][2]
  float *lam_hist;       // device, per iteration lambda (scale * lambda_star, +inf on the branch)
  int *flag_hist;        // device, per iteration flags
  const float *scales;   // device, nscale entries (may be null)
  int hist_cap;          // capacity of the history arrays
};
constexpr int kLamAccFirst = 2 + 2 * kLamFirstCand;  // Einf, floor, f and slope per candidate
constexpr int kLamAccSweep = 2 * kLamMaxCand;
constexpr int kLamAcc = kLamAccFirst > kLamAccSweep ? kLamAccFirst : kLamAccSweep;

// ---------------------------------------------------------------- launchers (kernels_*.hip)
// Row pass, forward real-to-half-complex: x (M x N real) -> S (tile-major half spectrum).
hipError_t launch_row_fwd(const float *x, const Layout &L, const FftPlan &pn, const cf *twN, cf *S,
                          hipStream_t st);
hipError_t launch_row_fwd_d(const double *x, const Layout &L, const FftPlan &pn, const cd *twN, cd *S,
                            hipStream_t st);
hipError_t launch_row_fwd_fd(const float *x, const Layout &L, const FftPlan &pn, const cd *twN, cd *S,
                             hipStream_t st);
// Column pass, forward, in place (transform only).
hipError_t launch_col_fwd_d(cd *S, const Layout &L, const FftPlan &pm, const cd *twM, hipStream_t st);
hipError_t launch_col_fwd_f(cf *S, const Layout &L, const FftPlan &pm, const cf *twM, hipStream_t st);
// Column pass, forward, in place, fused with R = H U_E - Y, q = w |R|^2 and the first lambda
// candidates; the last block starts the lambda search.
hipError_t launch_col_fwd_resid(cf *S, float *q, const cf *H, const cf *Y, const Layout &L,
                                const FftPlan &pm, const cf *twM, const LamBuffers &lb, hipStream_t st);
// One evaluation round of the lambda search over (q, |H|^2).
hipError_t launch_lam_sweep(const float *q, const float *H2, size_t nbins, const LamBuffers &lb, int last,
                            hipStream_t st);
// Spectral solves (Eqs. 8-9) with lambda from the state, then column inverse of both spectra.
hipError_t launch_col_inv(const cf *UE, const cf *HY, const float *H2, const float *dM, const float *dN,
                          const Layout &L, const FftPlan &pm, const cf *twM, const LamBuffers &lb,
                          cf *SI, cf *SP, hipStream_t st);
// Row pass, inverse: two half spectra -> two real images.
hipError_t launch_row_inv(const cf *SI, const cf *SP, const Layout &L, const FftPlan &pn, const cf *twN,
                          float *uI, float *uP, hipStream_t st);
// Guided filter; cI / cP point at the offsets subtracted before forming products.  With a
// state, the kernel also closes the iteration (counter, first lambda candidates of the next).
hipError_t launch_guided_filter(const float *uI, const float *uP, float *u, int M, int N, int w, float eps,
                                const float *cI, const float *cP, LamState *st, hipStream_t s);
bool guided_filter_supported(int w);

// Init helpers
hipError_t launch_embed_psf(const float *h, int kh, int kw, int M, int N, double *hp, hipStream_t st);
hipError_t launch_init_consts(const cd *Hd, const cd *Yd, const Layout &L, cf *H, cf *Y, cf *HY, float *H2,
                              hipStream_t st);
hipError_t launch_d2_tables(int M, int N, int Wh, float *dM, float *dN, hipStream_t st);
// rho of Eq.(12) and the target; writes doubles {rho, T} to out2 and fills the state constants.
hipError_t launch_rho_target(const float *y, int M, int N, const float *h, int kh, int kw, double sigma2,
                             double rho_fixed, double *work, double *out2, LamState *st, hipStream_t st_);
hipError_t launch_fill_f(float *p, size_t n, float v, hipStream_t st);
hipError_t launch_state_reset(LamState *st, hipStream_t s);

}  // namespace gfd
