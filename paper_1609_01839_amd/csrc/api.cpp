// C ABI of the library: argument checks, context lifetime, per-image set-up, the iteration
// (eager or as a replayed HIP graph) and the stand-alone entry points.  See gfdeconv.h.
#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "../../include/gfdeconv.h"
#include "gfd_internal.h"

namespace gfd {
hipError_t launch_state_set_lam(LamState *st, float lam, hipStream_t s);
hipError_t launch_copy_lam_star(const LamState *st, float *out, hipStream_t s);
}  // namespace gfd

using namespace gfd;

static const uint64_t kMagic = 0x6766646563763031ull;  // "gfdecv01"
static const int kSweeps = 3;      // lambda evaluation rounds per iteration after the first (graph)
static const int kSweepsFull = 10; // rounds of a stand-alone search (cold start allowed)

struct gfd_ctx {
  uint64_t magic;
  int device;
  int M, N, w;
  float eps;
  double sigma2, rho, T;
  Layout lay;
  FftPlan pm, pn;
  cf *twM, *twN;
  cf *H, *Y, *HY;
  float *H2, *dM, *dN;
  float *uE, *uI, *uP, *q;
  cf *S1, *SI, *SP;
  LamState *st, *st_aux;
  float *partials;
  float *lam_hist, *lam_hist_aux;
  int *flag_hist, *flag_hist_aux;
  float *scales;
  double *rho_out;
  int hist_cap;
  int iters;
  int use_graph;
  hipGraphExec_t gexec;
  hipStream_t cap_stream;
};

static thread_local std::string g_err;
static std::mutex g_live_mu;
static std::set<gfd_ctx *> g_live;

static gfd_status fail(gfd_status code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(call)                                                                           \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess) return fail(GFD_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

static bool size_ok(int n) {
  if (n < 2 || n > 4096) return false;
  for (int p : {2, 3, 5})
    while (n % p == 0) n /= p;
  return n == 1;
}

static bool live(gfd_ctx *c) {
  std::lock_guard<std::mutex> g(g_live_mu);
  return c != nullptr && g_live.count(c) && c->magic == kMagic;
}

static void free_ctx(gfd_ctx *c) {
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  void *ptrs[] = {c->twM, c->twN, c->H, c->Y, c->HY, c->H2, c->dM, c->dN, c->uE, c->uI, c->uP, c->q, c->S1, c->SI,
                  c->SP, c->st, c->st_aux, c->partials, c->lam_hist, c->lam_hist_aux, c->flag_hist,
                  c->flag_hist_aux, c->scales, c->rho_out};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  c->magic = 0;
  delete c;
}

template <class T>
static hipError_t dalloc(T **p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  return hipMalloc((void **)p, count * sizeof(T));
}

static std::vector<double> twiddles(int L) {
  std::vector<double> t(2 * (size_t)L);
  const double pi = 3.14159265358979323846;
  for (int n = 0; n < L; ++n) {
    t[2 * n] = cos(2.0 * pi * n / L);
    t[2 * n + 1] = -sin(2.0 * pi * n / L);
  }
  return t;
}

static LamBuffers lam_buffers(gfd_ctx *c, bool aux) {
  LamBuffers lb;
  lb.st = aux ? c->st_aux : c->st;
  lb.partials = c->partials;
  lb.lam_hist = aux ? c->lam_hist_aux : c->lam_hist;
  lb.flag_hist = aux ? c->flag_hist_aux : c->flag_hist;
  lb.scales = aux ? nullptr : c->scales;
  lb.hist_cap = aux ? 1 : c->hist_cap;
  return lb;
}

// The work of one iteration, Steps 1-3 of Sec. 3.1.
static hipError_t enqueue_iteration(gfd_ctx *c, hipStream_t s) {
  const Layout &L = c->lay;
  LamBuffers lb = lam_buffers(c, false);
  hipError_t e;
  if ((e = launch_row_fwd(c->uE, L, c->pn, c->twN, c->S1, s)) != hipSuccess) return e;
  if ((e = launch_col_fwd_resid(c->S1, c->q, c->H, c->Y, L, c->pm, c->twM, lb, s)) != hipSuccess) return e;
  for (int k = 0; k < kSweeps; ++k)
    if ((e = launch_lam_sweep(c->q, c->H2, L.bins(), lb, k == kSweeps - 1, s)) != hipSuccess) return e;
  if ((e = launch_col_inv(c->S1, c->HY, c->H2, c->dM, c->dN, L, c->pm, c->twM, lb, c->SI, c->SP, s)) != hipSuccess)
    return e;
  if ((e = launch_row_inv(c->SI, c->SP, L, c->pn, c->twN, c->uI, c->uP, s)) != hipSuccess) return e;
  return launch_guided_filter(c->uI, c->uP, c->uE, c->M, c->N, c->w, c->eps, &c->st->meanI, &c->st->meanP,
                              c->st, s);
}

// The same launches as enqueue_iteration with an event recorded after each pass.
static hipError_t enqueue_iteration_timed(gfd_ctx *c, hipStream_t s, hipEvent_t *ev) {
  const Layout &L = c->lay;
  LamBuffers lb = lam_buffers(c, false);
  hipError_t e;
  if ((e = hipEventRecord(ev[0], s)) != hipSuccess) return e;
  if ((e = launch_row_fwd(c->uE, L, c->pn, c->twN, c->S1, s)) != hipSuccess) return e;
  if ((e = hipEventRecord(ev[1], s)) != hipSuccess) return e;
  if ((e = launch_col_fwd_resid(c->S1, c->q, c->H, c->Y, L, c->pm, c->twM, lb, s)) != hipSuccess) return e;
  if ((e = hipEventRecord(ev[2], s)) != hipSuccess) return e;
  for (int k = 0; k < kSweeps; ++k)
    if ((e = launch_lam_sweep(c->q, c->H2, L.bins(), lb, k == kSweeps - 1, s)) != hipSuccess) return e;
  if ((e = hipEventRecord(ev[3], s)) != hipSuccess) return e;
  if ((e = launch_col_inv(c->S1, c->HY, c->H2, c->dM, c->dN, L, c->pm, c->twM, lb, c->SI, c->SP, s)) != hipSuccess)
    return e;
  if ((e = hipEventRecord(ev[4], s)) != hipSuccess) return e;
  if ((e = launch_row_inv(c->SI, c->SP, L, c->pn, c->twN, c->uI, c->uP, s)) != hipSuccess) return e;
  if ((e = hipEventRecord(ev[5], s)) != hipSuccess) return e;
  if ((e = launch_guided_filter(c->uI, c->uP, c->uE, c->M, c->N, c->w, c->eps, &c->st->meanI, &c->st->meanP,
                                c->st, s)) != hipSuccess)
    return e;
  return hipEventRecord(ev[6], s);
}

// Lambda search for the current estimate outside the graph, with enough rounds for a cold start;
// leaves lambda_star as the warm start of the next iteration (the iteration count is unchanged).
static hipError_t enqueue_warm_start(gfd_ctx *c, hipStream_t s) {
  const Layout &L = c->lay;
  LamBuffers lb = lam_buffers(c, false);
  hipError_t e;
  if ((e = launch_row_fwd(c->uE, L, c->pn, c->twN, c->S1, s)) != hipSuccess) return e;
  if ((e = launch_col_fwd_resid(c->S1, c->q, c->H, c->Y, L, c->pm, c->twM, lb, s)) != hipSuccess) return e;
  for (int k = 0; k < kSweepsFull; ++k)
    if ((e = launch_lam_sweep(c->q, c->H2, L.bins(), lb, k == kSweepsFull - 1, s)) != hipSuccess) return e;
  return hipSuccess;
}

static gfd_status capture_graph(gfd_ctx *c) {
  if (!c->cap_stream) HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
  hipError_t e = enqueue_iteration(c, c->cap_stream);
  hipError_t e2 = hipStreamEndCapture(c->cap_stream, &g);
  if (e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return fail(GFD_ERR_HIP, "capturing the iteration failed: %s", hipGetErrorString(e));
  }
  if (e2 != hipSuccess) return fail(GFD_ERR_HIP, "hipStreamEndCapture failed: %s", hipGetErrorString(e2));
  e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    c->gexec = nullptr;
    return fail(GFD_ERR_HIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
  }
  return GFD_OK;
}

extern "C" {

const char *gfd_last_error(void) { return g_err.c_str(); }

gfd_status deconv_init(gfd_ctx **out, const float *y, int M, int N, const float *h, int kh, int kw, double sigma2,
                       int w, float eps, double rho, void *stream) {
  g_err.clear();
  if (!out) return fail(GFD_ERR_ARG, "out is NULL");
  if (!y || !h) return fail(GFD_ERR_ARG, "y and h must be device pointers");
  if (!size_ok(M) || !size_ok(N))
    return fail(GFD_ERR_SIZE, "M=%d, N=%d: each must be 2^a 3^b 5^c in [2, 4096]", M, N);
  if (kh < 1 || kw < 1 || kh % 2 == 0 || kw % 2 == 0 || kh > M || kw > N)
    return fail(GFD_ERR_SIZE, "PSF %dx%d: sides must be odd and at most the image sides", kh, kw);
  if (!(sigma2 >= 0.0) || !isfinite(sigma2)) return fail(GFD_ERR_ARG, "sigma2 must be finite and >= 0");
  if (w < 1 || w % 2 == 0 || w > M || w > N) return fail(GFD_ERR_ARG, "w=%d must be odd, 1 <= w <= min(M, N)", w);
  if (!(eps > 0.0f) || !isfinite(eps)) return fail(GFD_ERR_ARG, "eps must be finite and > 0");
  if (!(rho <= 1.0) || !isfinite(rho)) return fail(GFD_ERR_ARG, "rho must be <= 1 (<= 0 selects Eq.(12))");
  if (!guided_filter_supported(w)) return fail(GFD_ERR_UNIMPLEMENTED, "w=%d: windows wider than 17 are not built", w);
  hipStream_t s = (hipStream_t)stream;
  // the PSF sum decides solvability at the zero frequency: read the (small) PSF first
  std::vector<float> hh((size_t)kh * kw);
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipMemcpy(hh.data(), h, hh.size() * sizeof(float), hipMemcpyDeviceToHost));
  double hsum = 0.0;
  for (float v : hh) {
    if (!isfinite(v)) return fail(GFD_ERR_ARG, "PSF has a non-finite entry");
    hsum += v;
  }
  if (hsum == 0.0) return fail(GFD_ERR_ARG, "PSF sums to zero");

  gfd_ctx *c = new gfd_ctx;
  memset(c, 0, sizeof(*c));
  c->magic = kMagic;
  HIPCHK(hipGetDevice(&c->device));
  c->M = M;
  c->N = N;
  c->w = w;
  c->eps = eps;
  c->sigma2 = sigma2;
  c->lay = make_layout(M, N);
  c->pm = make_plan(M);
  c->pn = make_plan(N);
  c->hist_cap = 1024;
  c->use_graph = 1;
  const Layout &L = c->lay;
  const size_t P = (size_t)M * N, nb = L.bins();
  const int nparts = (int)std::max<size_t>((size_t)L.NT, 1024);
  hipError_t e = hipSuccess;
#define ALLOC(ptr, n) \
  if (e == hipSuccess) e = dalloc(&(ptr), (n))
  ALLOC(c->twM, M);
  ALLOC(c->twN, N);
  ALLOC(c->H, nb);
  ALLOC(c->Y, nb);
  ALLOC(c->HY, nb);
  ALLOC(c->H2, nb);
  ALLOC(c->dM, M);
  ALLOC(c->dN, L.Wh);
  ALLOC(c->uE, P);
  ALLOC(c->uI, P);
  ALLOC(c->uP, P);
  ALLOC(c->q, nb);
  ALLOC(c->S1, nb);
  ALLOC(c->SI, nb);
  ALLOC(c->SP, nb);
  ALLOC(c->st, 1);
  ALLOC(c->st_aux, 1);
  ALLOC(c->partials, (size_t)nparts * kLamAcc * 2);
  ALLOC(c->lam_hist, c->hist_cap);
  ALLOC(c->flag_hist, c->hist_cap);
  ALLOC(c->lam_hist_aux, 1);
  ALLOC(c->flag_hist_aux, 1);
  ALLOC(c->scales, c->hist_cap);
  ALLOC(c->rho_out, 2);
  // FP64 temporaries of the set-up
  double *hp = nullptr, *work = nullptr;
  cd *Hd = nullptr, *Yd = nullptr, *twMd = nullptr, *twNd = nullptr;
  ALLOC(hp, P);
  ALLOC(work, 4 * 256);
  ALLOC(Hd, nb);
  ALLOC(Yd, nb);
  ALLOC(twMd, M);
  ALLOC(twNd, N);
#undef ALLOC
  auto cleanup_tmp = [&]() {
    void *t[] = {hp, work, Hd, Yd, twMd, twNd};
    for (void *p : t)
      if (p) (void)hipFree(p);
  };
  if (e != hipSuccess) {
    cleanup_tmp();
    free_ctx(c);
    return fail(e == hipErrorOutOfMemory ? GFD_ERR_NOMEM : GFD_ERR_HIP, "allocation failed: %s",
                hipGetErrorString(e));
  }
  // twiddle tables, FP64 on the host
  std::vector<double> tm = twiddles(M), tn = twiddles(N);
  std::vector<float> tmf(tm.begin(), tm.end()), tnf(tn.begin(), tn.end());
  if (e == hipSuccess) e = hipMemcpy(twMd, tm.data(), tm.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(twNd, tn.data(), tn.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(c->twM, tmf.data(), tmf.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(c->twN, tnf.data(), tnf.size() * sizeof(float), hipMemcpyHostToDevice);
  // F(h) and F(y) in FP64, then the FP32 constants
  if (e == hipSuccess) e = launch_embed_psf(h, kh, kw, M, N, hp, s);
  if (e == hipSuccess) e = launch_row_fwd_d(hp, L, c->pn, twNd, Hd, s);
  if (e == hipSuccess) e = launch_col_fwd_d(Hd, L, c->pm, twMd, s);
  if (e == hipSuccess) e = launch_row_fwd_fd(y, L, c->pn, twNd, Yd, s);
  if (e == hipSuccess) e = launch_col_fwd_d(Yd, L, c->pm, twMd, s);
  if (e == hipSuccess) e = launch_init_consts(Hd, Yd, L, c->H, c->Y, c->HY, c->H2, s);
  if (e == hipSuccess) e = launch_d2_tables(M, N, L.Wh, c->dM, c->dN, s);
  if (e == hipSuccess) e = launch_rho_target(y, M, N, h, kh, kw, sigma2, rho, work, c->rho_out, c->st, s);
  if (e == hipSuccess) e = hipMemcpyAsync(c->st_aux, c->st, sizeof(LamState), hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = launch_state_reset(c->st, s);
  if (e == hipSuccess) e = launch_state_reset(c->st_aux, s);
  if (e == hipSuccess) e = launch_fill_f(c->uE, P, 0.0f, s);
  if (e == hipSuccess) e = launch_fill_f(c->scales, c->hist_cap, 1.0f, s);
  if (e == hipSuccess) e = enqueue_warm_start(c, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  double ro[2] = {0, 0};
  if (e == hipSuccess) e = hipMemcpy(ro, c->rho_out, sizeof(ro), hipMemcpyDeviceToHost);
  cleanup_tmp();
  if (e != hipSuccess) {
    free_ctx(c);
    return fail(GFD_ERR_HIP, "set-up failed: %s", hipGetErrorString(e));
  }
  c->rho = ro[0];
  c->T = ro[1];
  {
    std::lock_guard<std::mutex> g(g_live_mu);
    g_live.insert(c);
  }
  *out = c;
  return GFD_OK;
}

static gfd_status grow_history(gfd_ctx *c, int need) {
  if (need <= c->hist_cap) return GFD_OK;
  int cap = c->hist_cap;
  while (cap < need) cap *= 2;
  float *lh = nullptr, *sc = nullptr;
  int *fh = nullptr;
  HIPCHK(hipDeviceSynchronize());
  HIPCHK(hipMalloc((void **)&lh, cap * sizeof(float)));
  HIPCHK(hipMalloc((void **)&fh, cap * sizeof(int)));
  HIPCHK(hipMalloc((void **)&sc, cap * sizeof(float)));
  HIPCHK(launch_fill_f(sc, cap, 1.0f, nullptr));
  HIPCHK(hipMemcpy(lh, c->lam_hist, c->hist_cap * sizeof(float), hipMemcpyDeviceToDevice));
  HIPCHK(hipMemcpy(fh, c->flag_hist, c->hist_cap * sizeof(int), hipMemcpyDeviceToDevice));
  HIPCHK(hipMemcpy(sc, c->scales, c->hist_cap * sizeof(float), hipMemcpyDeviceToDevice));
  HIPCHK(hipDeviceSynchronize());
  (void)hipFree(c->lam_hist);
  (void)hipFree(c->flag_hist);
  (void)hipFree(c->scales);
  c->lam_hist = lh;
  c->flag_hist = fh;
  c->scales = sc;
  c->hist_cap = cap;
  if (c->gexec) {  // the captured graph holds the old pointers
    (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
  }
  return GFD_OK;
}

gfd_status deconv_iterate(gfd_ctx *ctx, int n_iter, float *u_out, float *lambda_out, void *stream) {
  g_err.clear();
  if (!live(ctx)) return fail(GFD_ERR_STATE, "invalid or destroyed context");
  if (n_iter < 0) return fail(GFD_ERR_ARG, "n_iter must be >= 0");
  hipStream_t s = (hipStream_t)stream;
  gfd_status rc = grow_history(ctx, ctx->iters + n_iter);
  if (rc != GFD_OK) return rc;
  if (ctx->use_graph && !ctx->gexec && n_iter > 0) {
    rc = capture_graph(ctx);
    if (rc != GFD_OK) return rc;
  }
  for (int i = 0; i < n_iter; ++i) {
    if (ctx->use_graph) HIPCHK(hipGraphLaunch(ctx->gexec, s));
    else HIPCHK(enqueue_iteration(ctx, s));
  }
  const size_t P = (size_t)ctx->M * ctx->N;
  if (u_out) HIPCHK(hipMemcpyAsync(u_out, ctx->uE, P * sizeof(float), hipMemcpyDeviceToDevice, s));
  if (lambda_out && n_iter > 0)
    HIPCHK(hipMemcpyAsync(lambda_out, ctx->lam_hist + ctx->iters, n_iter * sizeof(float), hipMemcpyDeviceToDevice, s));
  ctx->iters += n_iter;
  return GFD_OK;
}

gfd_status deconv_profile(gfd_ctx *ctx, int n_iter, float *stage_ms_host, int n_stages, void *stream) {
  g_err.clear();
  if (!live(ctx)) return fail(GFD_ERR_STATE, "invalid or destroyed context");
  if (n_iter < 0 || n_stages < 0 || n_stages > 6 || (n_stages > 0 && !stage_ms_host))
    return fail(GFD_ERR_ARG, "n_iter >= 0, 0 <= n_stages <= 6, stage_ms_host non-NULL");
  hipStream_t s = (hipStream_t)stream;
  gfd_status rc = grow_history(ctx, ctx->iters + n_iter);
  if (rc != GFD_OK) return rc;
  hipEvent_t ev[7];
  for (int i = 0; i < 7; ++i) HIPCHK(hipEventCreate(&ev[i]));
  double acc[6] = {0, 0, 0, 0, 0, 0};
  hipError_t e = hipSuccess;
  for (int it = 0; it < n_iter && e == hipSuccess; ++it) {
    e = enqueue_iteration_timed(ctx, s, ev);
    if (e == hipSuccess) e = hipEventSynchronize(ev[6]);
    for (int k = 0; k < 6 && e == hipSuccess; ++k) {
      float ms = 0.0f;
      e = hipEventElapsedTime(&ms, ev[k], ev[k + 1]);
      acc[k] += ms;
    }
  }
  for (int i = 0; i < 7; ++i) (void)hipEventDestroy(ev[i]);
  if (e != hipSuccess) return fail(GFD_ERR_HIP, "profiled iteration failed: %s", hipGetErrorString(e));
  ctx->iters += n_iter;
  for (int k = 0; k < n_stages; ++k) stage_ms_host[k] = (float)acc[k];
  return GFD_OK;
}

gfd_status guided_filter(const float *uI, const float *up, float *u, int M, int N, int w, float eps, void *stream) {
  g_err.clear();
  if (!uI || !up || !u) return fail(GFD_ERR_ARG, "uI, up and u must be device pointers");
  if (M < 1 || N < 1 || M > 65536 || N > 65536) return fail(GFD_ERR_SIZE, "M=%d, N=%d out of [1, 65536]", M, N);
  if (w < 1 || w % 2 == 0 || w > M || w > N) return fail(GFD_ERR_ARG, "w=%d must be odd, 1 <= w <= min(M, N)", w);
  if (!(eps > 0.0f) || !isfinite(eps)) return fail(GFD_ERR_ARG, "eps must be finite and > 0");
  const size_t bytes = (size_t)M * N * sizeof(float);
  auto overlap = [&](const void *a, const void *b) {
    const char *pa = (const char *)a, *pb = (const char *)b;
    return pa < pb + bytes && pb < pa + bytes;
  };
  if (overlap(u, uI) || overlap(u, up)) return fail(GFD_ERR_ARG, "u must not overlap uI or up");
  if (!guided_filter_supported(w)) return fail(GFD_ERR_UNIMPLEMENTED, "w=%d: windows wider than 17 are not built", w);
  HIPCHK(launch_guided_filter(uI, up, u, M, N, w, eps, uI, up, nullptr, (hipStream_t)stream));
  return GFD_OK;
}

gfd_status spectral_solve(gfd_ctx *ctx, const float *uE, float lambda, float *uI, float *up, void *stream) {
  g_err.clear();
  if (!live(ctx)) return fail(GFD_ERR_STATE, "invalid or destroyed context");
  if (!uE || !uI || !up) return fail(GFD_ERR_ARG, "uE, uI and up must be device pointers");
  if (!(lambda > 0.0f)) return fail(GFD_ERR_ARG, "lambda must be > 0 (or +inf)");
  hipStream_t s = (hipStream_t)stream;
  gfd_ctx *c = ctx;
  const Layout &L = c->lay;
  LamBuffers lb = lam_buffers(c, true);
  HIPCHK(launch_row_fwd(uE, L, c->pn, c->twN, c->S1, s));
  HIPCHK(launch_col_fwd_f(c->S1, L, c->pm, c->twM, s));
  HIPCHK(launch_state_set_lam(c->st_aux, lambda, s));
  HIPCHK(launch_col_inv(c->S1, c->HY, c->H2, c->dM, c->dN, L, c->pm, c->twM, lb, c->SI, c->SP, s));
  HIPCHK(launch_row_inv(c->SI, c->SP, L, c->pn, c->twN, uI, up, s));
  return GFD_OK;
}

gfd_status discrepancy_lambda(gfd_ctx *ctx, const float *uE, float *lambda_dev, void *stream) {
  g_err.clear();
  if (!live(ctx)) return fail(GFD_ERR_STATE, "invalid or destroyed context");
  if (!uE || !lambda_dev) return fail(GFD_ERR_ARG, "uE and lambda_dev must be device pointers");
  hipStream_t s = (hipStream_t)stream;
  gfd_ctx *c = ctx;
  const Layout &L = c->lay;
  LamBuffers lb = lam_buffers(c, true);
  HIPCHK(launch_state_reset(c->st_aux, s));
  HIPCHK(launch_row_fwd(uE, L, c->pn, c->twN, c->S1, s));
  HIPCHK(launch_col_fwd_resid(c->S1, c->q, c->H, c->Y, L, c->pm, c->twM, lb, s));
  for (int k = 0; k < kSweepsFull; ++k)
    HIPCHK(launch_lam_sweep(c->q, c->H2, L.bins(), lb, k == kSweepsFull - 1, s));
  HIPCHK(launch_copy_lam_star(c->st_aux, lambda_dev, s));
  return GFD_OK;
}

gfd_status deconv_set_scales(gfd_ctx *ctx, const float *s_dev, int n) {
  g_err.clear();
  if (!live(ctx)) return fail(GFD_ERR_STATE, "invalid or destroyed context");
  if (n < 0 || (n > 0 && !s_dev)) return fail(GFD_ERR_ARG, "n must be >= 0 and s_dev non-NULL when n > 0");
  gfd_status rc = grow_history(ctx, ctx->iters + n);
  if (rc != GFD_OK) return rc;
  HIPCHK(hipDeviceSynchronize());
  HIPCHK(launch_fill_f(ctx->scales, ctx->hist_cap, 1.0f, nullptr));
  if (n > 0)
    HIPCHK(hipMemcpy(ctx->scales + ctx->iters, s_dev, n * sizeof(float), hipMemcpyDeviceToDevice));
  int ns = n > 0 ? ctx->iters + n : 0;
  HIPCHK(hipMemcpy((char *)ctx->st + offsetof(LamState, nscale), &ns, sizeof(int), hipMemcpyHostToDevice));
  HIPCHK(hipDeviceSynchronize());
  return GFD_OK;
}

gfd_status deconv_set_estimate(gfd_ctx *ctx, const float *uE, void *stream) {
  g_err.clear();
  if (!live(ctx)) return fail(GFD_ERR_STATE, "invalid or destroyed context");
  if (!uE) return fail(GFD_ERR_ARG, "uE must be a device pointer");
  HIPCHK(hipMemcpyAsync(ctx->uE, uE, (size_t)ctx->M * ctx->N * sizeof(float), hipMemcpyDeviceToDevice,
                        (hipStream_t)stream));
  HIPCHK(enqueue_warm_start(ctx, (hipStream_t)stream));
  return GFD_OK;
}

gfd_status deconv_reset(gfd_ctx *ctx, void *stream) {
  g_err.clear();
  if (!live(ctx)) return fail(GFD_ERR_STATE, "invalid or destroyed context");
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(launch_fill_f(ctx->uE, (size_t)ctx->M * ctx->N, 0.0f, s));
  HIPCHK(launch_state_reset(ctx->st, s));
  HIPCHK(enqueue_warm_start(ctx, s));
  ctx->iters = 0;
  return GFD_OK;
}

gfd_status deconv_info(gfd_ctx *ctx, double *rho, double *target, int *iterations) {
  g_err.clear();
  if (!live(ctx)) return fail(GFD_ERR_STATE, "invalid or destroyed context");
  if (rho) *rho = ctx->rho;
  if (target) *target = ctx->T;
  if (iterations) *iterations = ctx->iters;
  return GFD_OK;
}

gfd_status deconv_get_status(gfd_ctx *ctx, unsigned *flags_host) {
  g_err.clear();
  if (!live(ctx)) return fail(GFD_ERR_STATE, "invalid or destroyed context");
  if (!flags_host) return fail(GFD_ERR_ARG, "flags_host is NULL");
  HIPCHK(hipDeviceSynchronize());
  unsigned f = 0;
  HIPCHK(hipMemcpy(&f, (char *)ctx->st + offsetof(LamState, flags_all), sizeof(unsigned), hipMemcpyDeviceToHost));
  *flags_host = f;
  return GFD_OK;
}

gfd_status deconv_set_graph(gfd_ctx *ctx, int use_graph) {
  g_err.clear();
  if (!live(ctx)) return fail(GFD_ERR_STATE, "invalid or destroyed context");
  ctx->use_graph = use_graph ? 1 : 0;
  return GFD_OK;
}

void deconv_destroy(gfd_ctx *ctx) {
  if (!ctx) return;
  {
    std::lock_guard<std::mutex> g(g_live_mu);
    if (!g_live.count(ctx)) return;
    g_live.erase(ctx);
  }
  (void)hipDeviceSynchronize();
  free_ctx(ctx);
}

}  // extern "C"
