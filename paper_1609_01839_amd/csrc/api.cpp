// C ABI of the library: argument checks, context lifetime, per-image set-up, the iteration
// (eager or as a replayed HIP graph) and the stand-alone entry points.
//
// A context holds one or more images.  Their device descriptors sit in one table and every
// pass of the iteration is a single launch per kernel variant over the work items of all
// images (plan builders in kernels_spec.hip / kernels_gf.hip), so a batch costs as many
// launches per iteration as one image.
#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "../../include/gfdeconv.h"
#include "gfd_internal.h"

using namespace gfd;

static const uint64_t kMagic = 0x6766646563763032ull;  // "gfdecv02"
static const int kMaxImages = 4096;
static const int kStages = 6;

struct ImgMeta {
  int M, N, w;    // M x N: the transform domain (the padded size for a padded observation)
  int Mo, No;     // the observed size (the caller's arrays)
  int pad, clip;  // GFD_BOUNDARY_PAD / GFD_BOUNDARY_CLIP
  float eps;
  double sigma2, rho, T;
};

struct gfd_ctx {
  uint64_t magic = 0;
  int device = 0;
  int count = 0;
  std::vector<ImgMeta> meta;
  ImgSet main, aux;  // aux: single-image contexts only (stand-alone solve and search)
  Plan stage[kStages];
  Plan iter, warm, aux_solve, aux_lam;
  std::vector<void *> allocs;  // every device allocation of the context
  LamState *st = nullptr;      // count states
  LamState *st_aux = nullptr;
  float *lam_hist = nullptr;   // count x hist_cap
  int *flag_hist = nullptr;
  float *lam_star_hist = nullptr;  // count x hist_cap
  std::vector<float *> u0;     // per image: the estimate the iterations started from
  float *scales = nullptr;     // hist_cap, shared by all images
  float *uE_aux = nullptr;
  double *rho_out = nullptr;   // 2 per image
  int hist_cap = 0;
  int iters = 0;
  int k_start = 0;  // first iteration since the estimate was last set (what the backward differentiates)
  int use_graph = 1;
  hipGraphExec_t gexec = nullptr;
  hipStream_t cap_stream = nullptr;  // graph capture and the context's own host reads (non-blocking)
  hipEvent_t done_ev = nullptr;      // recorded after the work of every stream-ordered call
  // graph branches: the launches of one pass (one per kernel variant, on disjoint images) are
  // captured on these streams, forked from and joined back into the capture stream
  std::vector<hipStream_t> branch;
  std::vector<hipEvent_t> branch_ev;
  struct Bwd *bwd = nullptr;   // reverse-mode buffers and plans, built on first use
  Tuning tune;                 // launch shapes in use (deconv_autotune)
  Arena *arena = nullptr;      // allocation-free context: every buffer is carved from here
};

// Reverse mode: descriptor sets over the same images.
//   bwd:  replays iterations (its own estimate uR and search state) and runs the adjoint
//   grad: two entries per image, the transforms of g_I and g_p
//   gout: the inverse transform of the adjoint spectrum into the gradient buffer
struct Bwd {
  ImgSet bwd, grad, gout;
  Plan fwd_a, fwd_b, gf, box[3], grad_fft, spec, col, gout_inv, inf;
  // a segment's replays filter with gf_save, which also leaves the first box pass's results of
  // the strip-kernel images; that pass (box[0]) then covers the other images only
  Plan gf_save;
  ItemRange one{0, 0};
  LamState *st = nullptr;
  AdjState *ad = nullptr;
  std::vector<float *> uR, gu;
  std::vector<std::vector<float *>> ck;  // per image, checkpoint slots
  // per image and segment position: what the adjoint of that iteration reads from its forward
  // pass (u_I, u_p, U_E and the filter's centring constants); the replay descriptors are pointed
  // at a position before the replay writes it and before the adjoint reads it
  std::vector<std::vector<BwdSlot>> seg;
  BwdSlot *seg_dev = nullptr;  // seg laid out image-major, nseg positions per image
  int nseg = 0;
  std::vector<void *> allocs;
  int hist_cap = 0;
};

static void free_bwd(Bwd *b) {
  if (!b) return;
  for (void *p : b->allocs)
    if (p) (void)hipFree(p);
  for (ImgSet *s : {&b->bwd, &b->grad, &b->gout}) {
    if (s->dev) (void)hipFree(s->dev);
    if (s->items_dev) (void)hipFree(s->items_dev);
    if (s->lamq) (void)hipFree(s->lamq);
  }
  delete b;
}

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

#define HIPCHK(call)                                                                               \
  do {                                                                                             \
    hipError_t e_ = (call);                                                                        \
    if (e_ != hipSuccess) return fail(GFD_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

static bool size_ok(int n) {
  if (n < 2 || n > 4096) return false;
  for (int p : {2, 3, 5})
    while (n % p == 0) n /= p;
  return n == 1;
}

// The smallest m >= n whose only prime factors are 2, 3 and 5.
static int good_size(int n) {
  for (int m = std::max(n, 1);; ++m) {
    int k = m;
    for (int p : {2, 3, 5})
      while (k % p == 0) k /= p;
    if (k == 1) return m;
  }
}

// Transform domain of an image: its own size, or the padded size (room for the PSF's support
// on every side of a non-circular observation).
static void domain_dims(const gfd_image &d, int &M, int &N) {
  const bool pad = (d.boundary & GFD_BOUNDARY_PAD) != 0;
  M = pad ? good_size(d.M + d.kh - 1) : d.M;
  N = pad ? good_size(d.N + d.kw - 1) : d.N;
}

static bool live(gfd_ctx *c) {
  std::lock_guard<std::mutex> g(g_live_mu);
  return c != nullptr && g_live.count(c) && c->magic == kMagic;
}

// The context's work is ordered on the caller's stream; every call that enqueues work records
// done_ev after it, so waiting for the context (before its buffers are replaced or read on the
// host) waits for that stream only, never for the whole device.
static hipError_t mark_done(gfd_ctx *c, hipStream_t s) { return hipEventRecord(c->done_ev, s); }
static hipError_t wait_done(gfd_ctx *c) { return hipEventSynchronize(c->done_ev); }

static void free_ctx(gfd_ctx *c) {
  free_bwd(c->bwd);
  c->bwd = nullptr;
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->done_ev) (void)hipEventDestroy(c->done_ev);
  for (hipStream_t s : c->branch) (void)hipStreamDestroy(s);
  for (hipEvent_t e : c->branch_ev) (void)hipEventDestroy(e);
  for (void *p : c->allocs)
    if (p) (void)hipFree(p);
  for (ImgSet *s : {&c->main, &c->aux}) {
    if (s->arena) continue;
    if (s->dev) (void)hipFree(s->dev);
    if (s->items_dev) (void)hipFree(s->items_dev);
    if (s->lamq) (void)hipFree(s->lamq);
  }
  c->magic = 0;
  delete c;
}

template <class T>
static hipError_t dalloc(gfd_ctx *c, T **p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  if (c->arena) return c->arena->take(count * sizeof(T), (void **)p);
  hipError_t e = hipMalloc((void **)p, count * sizeof(T));
  if (e == hipSuccess) c->allocs.push_back((void *)*p);
  return e;
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

static hipError_t upload_table(ImgSet &set) {
  if (set.arena) {
    if (!set.dev) {
      hipError_t e = set.arena->take(std::max<size_t>(set.imgs.size(), 1) * sizeof(Img), (void **)&set.dev);
      if (e == hipSuccess) e = set.arena->take(lam_queue_bytes((int)set.imgs.size()), (void **)&set.lamq);  // zeroed arena
      if (e != hipSuccess) return e;
    }
    if (set.arena->dry) return hipSuccess;
  } else if (!set.lamq) {
    const size_t qb = lam_queue_bytes((int)set.imgs.size());
    hipError_t e = hipMalloc((void **)&set.lamq, qb);
    if (e == hipSuccess) e = hipMemset(set.lamq, 0, qb);
    if (e != hipSuccess) {
      (void)hipFree(set.lamq);
      set.lamq = nullptr;
      return e;
    }
  }
  if (!set.arena && !set.dev) {
    hipError_t e = hipMalloc((void **)&set.dev, std::max<size_t>(set.imgs.size(), 1) * sizeof(Img));
    if (e != hipSuccess) {
      set.dev = nullptr;
      return e;
    }
  }
  return hipMemcpy(set.dev, set.imgs.data(), set.imgs.size() * sizeof(Img), hipMemcpyHostToDevice);
}

static void append(Plan &dst, const Plan &src) {
  dst.steps.insert(dst.steps.end(), src.steps.begin(), src.steps.end());
}

// Launch plans of the context: the six passes of an iteration (Steps 1-3 of Sec. 3.1), the
// warm-start search and, for one image, the stand-alone solve and search.
static hipError_t build_plans(gfd_ctx *c) {
  std::vector<int> all(c->count);
  for (int i = 0; i < c->count; ++i) all[i] = i;
  plan_row_fwd(c->stage[0], c->main, all);
  plan_col_fwd(c->stage[1], c->main, all, true);
  plan_lambda(c->stage[2], c->main, all, kLamSweeps, true);
  plan_col_inv(c->stage[3], c->main, all);
  plan_row_inv(c->stage[4], c->main, all);
  plan_guided_filter(c->stage[5], c->main, all);
  for (int k = 0; k < kStages; ++k) append(c->iter, c->stage[k]);
  append(c->warm, c->stage[0]);
  append(c->warm, c->stage[1]);
  plan_lambda(c->warm, c->main, all, kLamSweepsFull, false);
  hipError_t e = finalize_items(c->main);
  if (e != hipSuccess) return e;
  if (c->count == 1) {
    const std::vector<int> one{0};
    plan_row_fwd(c->aux_solve, c->aux, one);
    plan_col_fwd(c->aux_solve, c->aux, one, false);
    plan_col_inv(c->aux_solve, c->aux, one);
    plan_row_inv(c->aux_solve, c->aux, one);
    plan_row_fwd(c->aux_lam, c->aux, one);
    plan_col_fwd(c->aux_lam, c->aux, one, true);
    plan_lambda(c->aux_lam, c->aux, one, kLamSweepsFull, false);
    e = finalize_items(c->aux);
  }
  return e;
}

// One pass of the iteration into the capture: its launches (one per kernel variant, each on its
// own images) become parallel branches of the graph, so that the launches of a batch's image
// groups overlap and fill each other's tails; a pass with one launch stays on the capture stream.
static hipError_t capture_pass(gfd_ctx *c, const Plan &p, size_t &ev) {
  hipStream_t s = c->cap_stream;
  if (p.steps.size() <= 1) return p.enqueue(s);
  hipError_t e = hipEventRecord(c->branch_ev[ev], s);
  const size_t fork = ev++;
  for (size_t i = 0; i < p.steps.size() && e == hipSuccess; ++i) {
    e = hipStreamWaitEvent(c->branch[i], c->branch_ev[fork], 0);
    if (e == hipSuccess) e = p.steps[i](c->branch[i]);
    if (e == hipSuccess) e = hipEventRecord(c->branch_ev[ev], c->branch[i]);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, c->branch_ev[ev++], 0);
  }
  return e;
}

static gfd_status capture_graph(gfd_ctx *c) {
  if (!c->cap_stream) HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  // streams and events for the branches: one stream per launch of the widest pass, one event
  // per fork and per join (default priority, like every stream here)
  size_t widest = 0, nev = 0;
  for (const Plan &p : c->stage) {
    widest = std::max(widest, p.steps.size());
    if (p.steps.size() > 1) nev += 1 + p.steps.size();
  }
  while (c->branch.size() < widest) {
    hipStream_t s = nullptr;
    HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    c->branch.push_back(s);
  }
  while (c->branch_ev.size() < nev) {
    hipEvent_t e = nullptr;
    HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    c->branch_ev.push_back(e);
  }
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
  hipError_t e = hipSuccess;
  size_t ev = 0;
  for (int k = 0; k < kStages && e == hipSuccess; ++k) e = capture_pass(c, c->stage[k], ev);
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

static gfd_status check_image(const gfd_image &d, int idx) {
  const int M = d.M, N = d.N;
  if (!d.y || !d.h) return fail(GFD_ERR_ARG, "image %d: y and h must be device pointers", idx);
  if (d.boundary < 0 || d.boundary > (GFD_BOUNDARY_CLIP | GFD_BOUNDARY_PAD))
    return fail(GFD_ERR_ARG, "image %d: unknown boundary flags %d", idx, d.boundary);
  if (d.boundary & GFD_BOUNDARY_PAD) {
    if (M < 2 || N < 2 || M > 4096 || N > 4096)
      return fail(GFD_ERR_SIZE, "image %d: M=%d, N=%d out of [2, 4096]", idx, M, N);
    if (d.kh >= 1 && d.kw >= 1 && d.kh <= M && d.kw <= N) {
      int Md, Nd;
      domain_dims(d, Md, Nd);
      if (Md > 4096 || Nd > 4096)
        return fail(GFD_ERR_SIZE, "image %d: padded domain %dx%d exceeds 4096", idx, Md, Nd);
    }
  } else if (!size_ok(M) || !size_ok(N)) {
    return fail(GFD_ERR_SIZE, "image %d: M=%d, N=%d: each must be 2^a 3^b 5^c in [2, 4096]", idx, M, N);
  }
  if (d.kh < 1 || d.kw < 1 || d.kh % 2 == 0 || d.kw % 2 == 0 || d.kh > M || d.kw > N)
    return fail(GFD_ERR_SIZE, "image %d: PSF %dx%d: sides must be odd and at most the image sides", idx, d.kh, d.kw);
  if (!(d.sigma2 >= 0.0) || !isfinite(d.sigma2)) return fail(GFD_ERR_ARG, "image %d: sigma2 must be finite and >= 0", idx);
  if (d.w < 1 || d.w % 2 == 0 || d.w > M || d.w > N)
    return fail(GFD_ERR_ARG, "image %d: w=%d must be odd, 1 <= w <= min(M, N)", idx, d.w);
  if (!(d.eps > 0.0f) || !isfinite(d.eps)) return fail(GFD_ERR_ARG, "image %d: eps must be finite and > 0", idx);
  if (!(d.rho <= 1.0) || !isfinite(d.rho))
    return fail(GFD_ERR_ARG, "image %d: rho must be <= 1 (<= 0 selects Eq.(12))", idx);
  return GFD_OK;
}

// Per-image buffers that only the set-up uses: the FP64 twiddles and the starting estimate.
struct ImgExtra {
  float *u0 = nullptr;
  cd *twMd = nullptr, *twNd = nullptr;
};

// Device buffers and descriptor of image i (no device work).
static hipError_t alloc_image(gfd_ctx *c, int i, const gfd_image &src, Img &d, ImgExtra &x) {
  int M, N;
  domain_dims(src, M, N);
  memset(&d, 0, sizeof(d));
  d.L = make_layout(M, N);
  d.pm = make_plan(M, c->tune.radix);
  d.pn = make_plan(N, c->tune.radix);
  d.rm = make_reg_plan(reg_plan_ok(M) ? M : 256);
  d.rn = make_reg_plan(reg_plan_ok(N) ? N : 256);
  d.w = src.w;
  d.eps = src.eps;
  d.clip = (src.boundary & GFD_BOUNDARY_CLIP) ? 1 : 0;
  const Layout &L = d.L;
  const size_t P = (size_t)M * N, nb = L.bins();
  d.nchunk = lam_sweep_chunks(nb);
  d.npart = std::max(L.NT, d.nchunk);
  cf *twM, *twN, *twB = nullptr, *H, *Y, *HY, *S1, *SIP;
  float *H2, *dM, *dN, *uE, *uI, *uP, *q, *part;
  cd *twMd, *twNd;
  hipError_t e = hipSuccess;
#define ALLOC(ptr, n) \
  if (e == hipSuccess) e = dalloc(c, &(ptr), (n))
  ALLOC(twM, M);
  ALLOC(twN, N);
  if (reg_plan_ok(M)) ALLOC(twB, (size_t)kRegTwRows * 16);
  ALLOC(H, nb);
  ALLOC(Y, nb);
  ALLOC(HY, nb);
  ALLOC(H2, nb);
  ALLOC(dM, M);
  ALLOC(dN, L.Wh);
  ALLOC(uE, P);
  ALLOC(uI, P);
  ALLOC(uP, P);
  ALLOC(q, nb);
  ALLOC(S1, nb);
  ALLOC(SIP, 2 * nb);
  ALLOC(part, (size_t)2 * kLamAcc * d.npart);
  float *u0 = nullptr;
  ALLOC(u0, P);
  ALLOC(twMd, M);
  ALLOC(twNd, N);
  float *wV = nullptr, *wa = nullptr, *wb = nullptr;
  if (gf_wide(src.w)) {  // the separable filter passes' window sums and coefficients
    ALLOC(wV, 4 * P);
    ALLOC(wa, P);
    ALLOC(wb, P);
  }
#undef ALLOC
  if (e != hipSuccess) return e;
  d.wV = wV;
  d.wa = wa;
  d.wb = wb;
  d.twM = twM;
  d.twB = twB;
  d.twN = twN;
  d.H = H;
  d.Y = Y;
  d.HY = HY;
  d.H2 = H2;
  d.dM = dM;
  d.dN = dN;
  d.uE = uE;
  d.uI = uI;
  d.uP = uP;
  d.q = q;
  d.S1 = S1;
  d.SIP = SIP;
  d.part = part;
  d.st = c->st + i;
  d.lam_hist = c->lam_hist + (size_t)i * c->hist_cap;
  d.flag_hist = c->flag_hist + (size_t)i * c->hist_cap;
  d.lam_star_hist = c->lam_star_hist + (size_t)i * c->hist_cap;
  d.scales = c->scales;
  d.hist_cap = c->hist_cap;
  gf_geometry(d, c->tune.gf_ty);
  x.u0 = u0;
  x.twMd = twMd;
  x.twNd = twNd;
  return hipSuccess;
}

// FP64 set-up of image i (F(h), F(y), constants, rho and the target) into its buffers.
static hipError_t init_image(gfd_ctx *c, int i, const gfd_image &src, const Img &d, const ImgExtra &x, hipStream_t s,
                             double *hp, cd *Hd, cd *Yd, double *work, float *ypad) {
  const bool pad = (src.boundary & GFD_BOUNDARY_PAD) != 0;
  const Layout &L = d.L;
  const int M = L.M, N = L.N;
  const size_t P = (size_t)M * N, nb = L.bins();
  cd *twMd = x.twMd, *twNd = x.twNd;
  hipError_t e = hipSuccess;
  // twiddle tables, FP64 on the host
  std::vector<double> tm = twiddles(M), tn = twiddles(N);
  std::vector<float> tmf(tm.begin(), tm.end()), tnf(tn.begin(), tn.end());
  if (e == hipSuccess) e = hipMemcpy(twMd, tm.data(), tm.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(twNd, tn.data(), tn.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy((void *)d.twM, tmf.data(), tmf.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy((void *)d.twN, tnf.data(), tnf.size() * sizeof(float), hipMemcpyHostToDevice);
  if (d.twB) {  // the same FP32 values by butterfly (TwTable): row r, entry i = w_M^(i k TS)
    std::vector<float> tb((size_t)kRegTwRows * 16 * 2);
    for (int r = 0; r < kRegTwRows; ++r) {
      const int k = r < 16 ? r : r - 16, ts = r < 16 ? M / 256 : 1;
      for (int i = 0; i < 16; ++i) {
        const size_t e = (size_t)i * k * ts % (size_t)M;
        tb[2 * ((size_t)r * 16 + i)] = tmf[2 * e];
        tb[2 * ((size_t)r * 16 + i) + 1] = tmf[2 * e + 1];
      }
    }
    if (e == hipSuccess) e = hipMemcpy((void *)d.twB, tb.data(), tb.size() * sizeof(float), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = launch_embed_psf(src.h, src.kh, src.kw, M, N, hp, s);
  if (e == hipSuccess) e = launch_row_fwd_d(hp, L, d.pn, twNd, Hd, s);
  if (e == hipSuccess) e = launch_col_fwd_d(Hd, L, d.pm, twMd, s);
  const float *ydom = src.y;
  if (pad) {
    if (e == hipSuccess) e = launch_pad_ramp(src.y, src.M, src.N, ypad, M, N, s);
    ydom = ypad;
  }
  if (e == hipSuccess) e = launch_row_fwd_fd(ydom, L, d.pn, twNd, Yd, s);
  if (e == hipSuccess) e = launch_col_fwd_d(Yd, L, d.pm, twMd, s);
  if (e == hipSuccess)
    e = launch_init_consts(Hd, Yd, L, (cf *)d.H, (cf *)d.Y, (cf *)d.HY, (float *)d.H2, s);
  if (e == hipSuccess) e = launch_d2_tables(M, N, L.Wh, (float *)d.dM, (float *)d.dN, s);
  if (e == hipSuccess)
    e = launch_rho_target(src.y, src.M, src.N, P, src.h, src.kh, src.kw, src.sigma2, src.rho, work, c->rho_out + 2 * i,
                          d.st, s);
  if (e == hipSuccess) e = launch_state_reset(d.st, s);
  if (e == hipSuccess) e = launch_fill_f(d.uE, P, 0.0f, s);
  if (e == hipSuccess) e = launch_fill_f(x.u0, P, 0.0f, s);
  // q of the padding columns (and of the last tile, which a folded residual pass never writes)
  // stays zero: the lambda sweeps sum over every bin
  if (e == hipSuccess) e = launch_fill_f(d.q, nb, 0.0f, s);
  // the FP64 temporaries are shared by the images: finish before the next image reuses them
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e;
}

// Host bookkeeping of image i once its buffers exist.
static void record_image(gfd_ctx *c, const gfd_image &src, const Img &d, const ImgExtra &x) {
  const bool pad = (src.boundary & GFD_BOUNDARY_PAD) != 0;
  const int M = d.L.M, N = d.L.N;
  c->u0.push_back(x.u0);
  c->main.imgs.push_back(d);
  ImgMeta m;
  m.M = M;
  m.N = N;
  m.Mo = src.M;
  m.No = src.N;
  m.pad = pad ? 1 : 0;
  m.clip = d.clip;
  m.w = src.w;
  m.eps = src.eps;
  m.sigma2 = src.sigma2;
  m.rho = 0.0;
  m.T = 0.0;
  c->meta.push_back(m);
}

static hipError_t setup_image(gfd_ctx *c, int i, const gfd_image &src, hipStream_t s, double *hp, cd *Hd, cd *Yd,
                              double *work, float *ypad) {
  Img d;
  ImgExtra x;
  hipError_t e = alloc_image(c, i, src, d, x);
  if (e != hipSuccess) return e;
  e = init_image(c, i, src, d, x, s, hp, Hd, Yd, work, ypad);
  record_image(c, src, d, x);
  return e;
}

// The PSF sum decides solvability at the zero frequency: read the (small) PSFs first.
static gfd_status check_psfs(const gfd_image *imgs, int count, hipStream_t s) {
  HIPCHK(hipStreamSynchronize(s));
  for (int i = 0; i < count; ++i) {
    std::vector<float> hh((size_t)imgs[i].kh * imgs[i].kw);
    HIPCHK(hipMemcpy(hh.data(), imgs[i].h, hh.size() * sizeof(float), hipMemcpyDeviceToHost));
    double hsum = 0.0;
    for (float v : hh) {
      if (!isfinite(v)) return fail(GFD_ERR_ARG, "image %d: PSF has a non-finite entry", i);
      hsum += v;
    }
    if (hsum == 0.0) return fail(GFD_ERR_ARG, "image %d: PSF sums to zero", i);
  }
  return GFD_OK;
}

static gfd_status init_common(gfd_ctx **out, const gfd_image *imgs, int count, hipStream_t s) {
  if (!out) return fail(GFD_ERR_ARG, "out is NULL");
  if (!imgs || count < 1 || count > kMaxImages)
    return fail(GFD_ERR_ARG, "need 1 <= count <= %d image descriptors", kMaxImages);
  for (int i = 0; i < count; ++i) {
    gfd_status rc = check_image(imgs[i], i);
    if (rc != GFD_OK) return rc;
  }
  {
    gfd_status rc = check_psfs(imgs, count, s);
    if (rc != GFD_OK) return rc;
  }

  gfd_ctx *c = new gfd_ctx;
  c->magic = kMagic;
  c->count = count;
  c->hist_cap = 1024;
  auto bail = [&](hipError_t e, const char *what) {
    free_ctx(c);
    return fail(e == hipErrorOutOfMemory ? GFD_ERR_NOMEM : GFD_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
  };
  hipError_t e = hipGetDevice(&c->device);
  if (e != hipSuccess) return bail(e, "hipGetDevice");
  e = hipEventCreateWithFlags(&c->done_ev, hipEventDisableTiming);
  if (e != hipSuccess) return bail(e, "hipEventCreateWithFlags");
  e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) return bail(e, "hipStreamCreateWithFlags");
  size_t maxP = 0, maxB = 0;
  for (int i = 0; i < count; ++i) {
    int Md, Nd;
    domain_dims(imgs[i], Md, Nd);
    maxP = std::max(maxP, (size_t)Md * Nd);
    maxB = std::max(maxB, make_layout(Md, Nd).bins());
  }
  double *hp = nullptr, *work = nullptr;
  float *ypad = nullptr;
  cd *Hd = nullptr, *Yd = nullptr;
  if (e == hipSuccess) e = dalloc(c, &c->st, count);
  c->main.st_base = c->st;
  if (e == hipSuccess) e = dalloc(c, &c->lam_hist, (size_t)count * c->hist_cap);
  if (e == hipSuccess) e = dalloc(c, &c->flag_hist, (size_t)count * c->hist_cap);
  if (e == hipSuccess) e = dalloc(c, &c->lam_star_hist, (size_t)count * c->hist_cap);
  if (e == hipSuccess) e = dalloc(c, &c->scales, c->hist_cap);
  if (e == hipSuccess) e = dalloc(c, &c->rho_out, 2 * (size_t)count);
  if (e == hipSuccess) e = dalloc(c, &hp, maxP);
  if (e == hipSuccess) e = dalloc(c, &work, 4 * 256);
  if (e == hipSuccess) e = dalloc(c, &Hd, maxB);
  if (e == hipSuccess) e = dalloc(c, &Yd, maxB);
  if (e == hipSuccess) e = dalloc(c, &ypad, maxP);
  if (e == hipSuccess) e = launch_fill_f(c->scales, c->hist_cap, 1.0f, s);
  if (e != hipSuccess) return bail(e, "allocation failed");
  for (int i = 0; i < count && e == hipSuccess; ++i) e = setup_image(c, i, imgs[i], s, hp, Hd, Yd, work, ypad);
  if (e != hipSuccess) return bail(e, "set-up failed");
  // the shared FP64 temporaries are no longer needed
  for (void *p : {(void *)hp, (void *)work, (void *)Hd, (void *)Yd, (void *)ypad}) {
    c->allocs.erase(std::find(c->allocs.begin(), c->allocs.end(), p));
    (void)hipFree(p);
  }
  if (count == 1) {
    Img a = c->main.imgs[0];
    if (e == hipSuccess) e = dalloc(c, &c->st_aux, 1);
    if (e == hipSuccess) e = dalloc(c, &c->uE_aux, (size_t)a.L.M * a.L.N);
    float *lh = nullptr;
    int *fh = nullptr;
    if (e == hipSuccess) e = dalloc(c, &lh, 1);
    if (e == hipSuccess) e = dalloc(c, &fh, 1);
    if (e != hipSuccess) return bail(e, "allocation failed");
    a.uE = c->uE_aux;
    a.st = c->st_aux;
    a.lam_hist = lh;
    a.flag_hist = fh;
    a.lam_star_hist = nullptr;
    a.hist_cap = 1;
    a.scales = nullptr;
    c->aux.imgs.push_back(a);
    c->aux.st_base = c->st_aux;
    e = hipMemcpyAsync(c->st_aux, c->st, sizeof(LamState), hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = launch_state_reset(c->st_aux, s);
    if (e == hipSuccess) e = upload_table(c->aux);
  }
  if (e == hipSuccess) e = upload_table(c->main);
  if (e == hipSuccess) e = build_plans(c);
  if (e == hipSuccess) e = c->warm.enqueue(s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  std::vector<double> ro(2 * (size_t)count);
  if (e == hipSuccess) e = hipMemcpy(ro.data(), c->rho_out, ro.size() * sizeof(double), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return bail(e, "set-up failed");
  for (int i = 0; i < count; ++i) {
    c->meta[i].rho = ro[2 * i];
    c->meta[i].T = ro[2 * i + 1];
  }
  e = mark_done(c, s);
  if (e != hipSuccess) return bail(e, "hipEventRecord");
  {
    std::lock_guard<std::mutex> g(g_live_mu);
    g_live.insert(c);
  }
  *out = c;
  return GFD_OK;
}

// Larger per-iteration histories; the descriptors are rewritten in place, so a captured
// graph (which reads them at run time) stays valid.  The reverse-mode sets copy these
// pointers and are rebuilt on their next use.
static gfd_status grow_history(gfd_ctx *c, int need, hipStream_t s) {
  if (need <= c->hist_cap) return GFD_OK;
  int cap = c->hist_cap;
  while (cap < need) cap *= 2;
  float *lh = nullptr, *lsh = nullptr, *sc = nullptr;
  int *fh = nullptr;
  HIPCHK(wait_done(c));
  HIPCHK(hipMalloc((void **)&lh, (size_t)c->count * cap * sizeof(float)));
  HIPCHK(hipMalloc((void **)&lsh, (size_t)c->count * cap * sizeof(float)));
  HIPCHK(hipMalloc((void **)&fh, (size_t)c->count * cap * sizeof(int)));
  HIPCHK(hipMalloc((void **)&sc, cap * sizeof(float)));
  HIPCHK(launch_fill_f(sc, cap, 1.0f, s));
  for (int i = 0; i < c->count; ++i) {
    const size_t o = (size_t)i * cap, oo = (size_t)i * c->hist_cap;
    HIPCHK(hipMemcpyAsync(lh + o, c->lam_hist + oo, c->hist_cap * sizeof(float), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(lsh + o, c->lam_star_hist + oo, c->hist_cap * sizeof(float), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(fh + o, c->flag_hist + oo, c->hist_cap * sizeof(int), hipMemcpyDeviceToDevice, s));
  }
  HIPCHK(hipMemcpyAsync(sc, c->scales, c->hist_cap * sizeof(float), hipMemcpyDeviceToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  for (void *old : {(void *)c->lam_hist, (void *)c->lam_star_hist, (void *)c->flag_hist, (void *)c->scales}) {
    c->allocs.erase(std::find(c->allocs.begin(), c->allocs.end(), old));
    (void)hipFree(old);
  }
  c->allocs.push_back(lh);
  c->allocs.push_back(lsh);
  c->allocs.push_back(fh);
  c->allocs.push_back(sc);
  c->lam_hist = lh;
  c->lam_star_hist = lsh;
  c->flag_hist = fh;
  c->scales = sc;
  c->hist_cap = cap;
  for (int i = 0; i < c->count; ++i) {
    Img &d = c->main.imgs[i];
    d.lam_hist = lh + (size_t)i * cap;
    d.lam_star_hist = lsh + (size_t)i * cap;
    d.flag_hist = fh + (size_t)i * cap;
    d.scales = sc;
    d.hist_cap = cap;
  }
  HIPCHK(upload_table(c->main));
  free_bwd(c->bwd);
  c->bwd = nullptr;
  return GFD_OK;
}

// The estimates, images one after another at their observed sizes (a padded image's estimate is
// cropped to its top-left M x N corner, where the observation sits).
static gfd_status copy_estimates_out(gfd_ctx *c, float *u_out, hipStream_t s) {
  size_t off = 0;
  for (int i = 0; i < c->count; ++i) {
    const ImgMeta &m = c->meta[i];
    const size_t P = (size_t)m.Mo * m.No;
    if (m.pad)
      HIPCHK(hipMemcpy2DAsync(u_out + off, m.No * sizeof(float), c->main.imgs[i].uE, m.N * sizeof(float),
                              m.No * sizeof(float), m.Mo, hipMemcpyDeviceToDevice, s));
    else
      HIPCHK(hipMemcpyAsync(u_out + off, c->main.imgs[i].uE, P * sizeof(float), hipMemcpyDeviceToDevice, s));
    off += P;
  }
  return GFD_OK;
}

// ---------------------------------------------------------------- launch-shape tuning
// New launch shapes for every image: layouts and strip geometry are recomputed (buffer sizes
// do not depend on them), and every plan, the captured graph and the reverse-mode sets are
// rebuilt.
static hipError_t apply_tuning(gfd_ctx *c, const Tuning &t) {
  for (Img &d : c->main.imgs) {
    d.L = make_layout(d.L.M, d.L.N, t);
    d.pm = make_plan(d.L.M, t.radix);
    d.pn = make_plan(d.L.N, t.radix);
    gf_geometry(d, t.gf_ty);
  }
  if (c->count == 1) {
    Img &a = c->aux.imgs[0];
    const Img &m = c->main.imgs[0];
    a.L = m.L;
    a.pm = m.pm;
    a.pn = m.pn;
    a.gfTX = m.gfTX;
    a.gfTY = m.gfTY;
    a.gfNBY = m.gfNBY;
  }
  c->tune = t;
  for (Plan *p : {&c->iter, &c->warm, &c->aux_solve, &c->aux_lam}) p->steps.clear();
  for (Plan &p : c->stage) p.steps.clear();
  c->main.items_host.clear();
  c->aux.items_host.clear();
  if (c->gexec) {
    (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
  }
  free_bwd(c->bwd);
  c->bwd = nullptr;
  hipError_t e = upload_table(c->main);
  if (e == hipSuccess && c->count == 1) e = upload_table(c->aux);
  if (e == hipSuccess) e = build_plans(c);
  return e;
}

// ---------------------------------------------------------------- reverse mode
template <class T>
static hipError_t balloc(Bwd *b, T **p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc((void **)p, count * sizeof(T));
  if (e == hipSuccess) b->allocs.push_back((void *)*p);
  return e;
}

// Buffers, descriptor sets and launch plans of the reverse mode.
static hipError_t build_bwd(gfd_ctx *c) {
  Bwd *b = new Bwd;
  c->bwd = b;
  b->hist_cap = c->hist_cap;
  const int n = c->count;
  hipError_t e = balloc(b, &b->st, n);
  if (e == hipSuccess) e = balloc(b, &b->ad, n);
  for (int i = 0; i < n && e == hipSuccess; ++i) {
    const Img &m = c->main.imgs[i];
    const size_t P = (size_t)m.L.M * m.L.N, nb = m.L.bins();
    Img d = m;
    float *uR, *ga, *gmu, *gpb, *gve, *gc, *gd, *gu, *gI, *gP, *gpart, *geh, *gsh;
    cf *SgI, *SgP, *Gs;
#define BALLOC(ptr, cnt) \
  if (e == hipSuccess) e = balloc(b, &(ptr), (cnt))
    BALLOC(uR, P);
    BALLOC(ga, P);
    BALLOC(gmu, P);
    BALLOC(gpb, P);
    BALLOC(gve, P);
    BALLOC(gc, P);
    BALLOC(gd, P);
    BALLOC(gu, P);
    BALLOC(gI, P);
    BALLOC(gP, P);
    BALLOC(SgI, nb);
    BALLOC(SgP, nb);
    BALLOC(Gs, nb);
    BALLOC(geh, c->hist_cap);
    BALLOC(gsh, c->hist_cap);
#undef BALLOC
    if (e != hipSuccess) break;
    adj_geometry(d);
    e = balloc(b, &gpart, (size_t)adj_strips(d));
    if (e != hipSuccess) break;
    d.uE = uR;
    d.st = b->st + i;
    d.ga = ga;
    d.gmu = gmu;
    d.gpb = gpb;
    d.gve = gve;
    d.gc = gc;
    d.gd = gd;
    d.gu = gu;
    d.gI = gI;
    d.gP = gP;
    d.geps_part = gpart;
    d.SgI = SgI;
    d.SgP = SgP;
    d.G = Gs;
    d.ad = b->ad + i;
    d.geps_hist = geh;
    d.gs_hist = gsh;
    b->bwd.imgs.push_back(d);
    Img gi = d, gp = d;  // transforms of g_I and g_p
    gi.uE = gI;
    gi.S1 = SgI;
    gp.uE = gP;
    gp.S1 = SgP;
    b->grad.imgs.push_back(gi);
    b->grad.imgs.push_back(gp);
    Img go = d;          // inverse transform of the adjoint spectrum into the gradient: its column
                         // pass writes (G, 0) pairs into the solves' buffer
    go.SIP = m.SIP;
    go.uI = gu;
    go.uP = m.uP;
    b->gout.imgs.push_back(go);
    b->uR.push_back(uR);
    b->gu.push_back(gu);
  }
  if (e != hipSuccess) return e;
  b->bwd.st_base = b->st;
  b->grad.st_base = b->st;
  b->gout.st_base = b->st;
  std::vector<int> all(n), all2(2 * n);
  for (int i = 0; i < n; ++i) all[i] = i;
  for (int i = 0; i < 2 * n; ++i) all2[i] = i;
  plan_row_fwd(b->fwd_a, b->bwd, all);
  plan_col_fwd(b->fwd_a, b->bwd, all, false);
  plan_col_inv(b->fwd_b, b->bwd, all);
  plan_row_inv(b->fwd_b, b->bwd, all);
  plan_guided_filter(b->gf, b->bwd, all);
  plan_guided_filter(b->gf_save, b->bwd, all, true);
  {
    std::vector<int> rest;  // images whose filter runs as separable passes
    for (int i = 0; i < n; ++i)
      if (gf_wide(b->bwd.imgs[i].w)) rest.push_back(i);
    if (!rest.empty()) plan_box_stage(b->box[0], b->bwd, rest, 1);
  }
  for (int st = 1; st < 3; ++st) plan_box_stage(b->box[st], b->bwd, all, st + 1);
  plan_adj_spec(b->spec, b->bwd, all);
  plan_adj_col(b->col, b->bwd, all);
  plan_adj_inf(b->inf, b->bwd, all);
  b->one = plan_one_per_image(b->bwd, all);
  plan_row_fwd(b->grad_fft, b->grad, all2);
  plan_col_fwd(b->grad_fft, b->grad, all2, false);
  plan_row_inv(b->gout_inv, b->gout, all);
  for (ImgSet *set : {&b->bwd, &b->grad, &b->gout}) {
    if (e == hipSuccess) e = upload_table(*set);
    if (e == hipSuccess) e = finalize_items(*set);
  }
  return e;
}

// Slots for checkpoints and for the pre-estimates of one segment.
static hipError_t bwd_slots(gfd_ctx *c, int nck, int seg) {
  Bwd *b = c->bwd;
  b->ck.resize(c->count);
  b->seg.resize(c->count);
  hipError_t e = hipSuccess;
  for (int i = 0; i < c->count && e == hipSuccess; ++i) {
    const size_t P = (size_t)c->meta[i].M * c->meta[i].N, nb = c->main.imgs[i].L.bins();
    while ((int)b->ck[i].size() < nck && e == hipSuccess) {
      float *p = nullptr;
      e = balloc(b, &p, P);
      b->ck[i].push_back(p);
    }
    while ((int)b->seg[i].size() < seg && e == hipSuccess) {
      BwdSlot sl = {};
      e = balloc(b, &sl.uI, P);
      if (e == hipSuccess) e = balloc(b, &sl.uP, P);
      if (e == hipSuccess) e = balloc(b, &sl.S1, nb);
      if (e == hipSuccess) e = balloc(b, &sl.means, 2);
      for (float **q : {&sl.ga, &sl.gmu, &sl.gpb, &sl.gve})
        if (e == hipSuccess) e = balloc(b, q, P);
      b->seg[i].push_back(sl);
    }
  }
  if (e != hipSuccess || c->count == 0 || (int)b->seg[0].size() == b->nseg) return e;
  // the positions grew: a new device copy of the table (the previous one may still be read by
  // the last call's kernels, so it is kept until the buffers are freed)
  const int n = (int)b->seg[0].size();
  std::vector<BwdSlot> flat;
  for (int i = 0; i < c->count; ++i)
    for (int j = 0; j < n; ++j) flat.push_back(b->seg[i][j]);
  BwdSlot *dev = nullptr;
  e = balloc(b, &dev, flat.size());
  if (e == hipSuccess) e = hipMemcpy(dev, flat.data(), flat.size() * sizeof(BwdSlot), hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    b->seg_dev = dev;
    b->nseg = n;
  }
  return e;
}

static hipError_t copy_images(gfd_ctx *c, const std::vector<float *> &dst, const std::vector<float *> &src,
                              hipStream_t s) {
  for (int i = 0; i < c->count; ++i) {
    const size_t P = (size_t)c->meta[i].M * c->meta[i].N;
    hipError_t e = hipMemcpyAsync(dst[i], src[i], P * sizeof(float), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

static std::vector<float *> slot(const std::vector<std::vector<float *>> &v, int j) {
  std::vector<float *> r;
  for (const auto &x : v) r.push_back(x[j]);
  return r;
}

// Iteration k of the forward run again, with its logged lambda: u_I, u_p (and U_E in S1);
// with `filter` also the next pre-estimate, in place in uR.
static hipError_t replay(Bwd *b, int k, bool filter, hipStream_t s) {
  hipError_t e = b->fwd_a.enqueue(s);
  if (e == hipSuccess) e = launch_lam_replay(b->bwd, b->one, k, s);
  if (e == hipSuccess) e = b->fwd_b.enqueue(s);
  if (e == hipSuccess && filter) e = b->gf.enqueue(s);
  return e;
}

// Adjoint of iteration k, whose forward quantities (u_I, u_p, U_E, centring constants) are in
// place; gu holds the gradient with respect to its output on entry and with respect to its
// pre-estimate on exit.  The replay of iteration k ran the saving filter, which left the first
// box pass's results of the strip-kernel images; that pass runs for the other images only.
static hipError_t adjoint_step(Bwd *b, int k, hipStream_t s) {
  hipError_t e = launch_lam_replay(b->bwd, b->one, k, s);
  for (int st = 0; st < 3 && e == hipSuccess; ++st) e = b->box[st].enqueue(s);
  if (e == hipSuccess) e = b->grad_fft.enqueue(s);
  if (e == hipSuccess) e = b->spec.enqueue(s);
  if (e == hipSuccess) e = launch_adj_fin(b->bwd, b->one, k, s);
  if (e == hipSuccess) e = b->col.enqueue(s);
  if (e == hipSuccess) e = b->gout_inv.enqueue(s);
  if (e == hipSuccess) e = b->inf.enqueue(s);
  return e;
}


// ---------------------------------------------------------------- allocation-free path
// deconvolve_static keeps every device buffer of its problem in one file-scope array per device
// (`scratch`), so that it calls no hipMalloc or hipFree.  In host code the array's name is only a
// stand-in for the device symbol: its device address comes from hipGetSymbolAddress, taken once
// per device with that device current, and only that address is ever used.
static constexpr size_t kScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static std::mutex g_scratch_mu;
static std::map<int, unsigned char *> g_scratch_addr;  // device -> address of its `scratch`

static hipError_t scratch_address(int dev, unsigned char **out) {
  std::lock_guard<std::mutex> g(g_scratch_mu);
  auto it = g_scratch_addr.find(dev);
  if (it != g_scratch_addr.end()) {
    *out = it->second;
    return hipSuccess;
  }
  void *p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_addr[dev] = (unsigned char *)p;
  *out = (unsigned char *)p;
  return hipSuccess;
}

// Carve every buffer of a one-image problem from c->arena and build its launch plans; the
// descriptor and work-item tables are copied in unless the arena is dry.  No device work.
static hipError_t carve_static(gfd_ctx *c, const gfd_image &src, int n_iter, ImgExtra &x) {
  c->count = 1;
  c->hist_cap = std::max(n_iter, 1);
  c->main.arena = c->aux.arena = c->arena;
  int Md, Nd;
  domain_dims(src, Md, Nd);
  const size_t P = (size_t)Md * Nd;
  hipError_t e = dalloc(c, &c->st, 1);
  c->main.st_base = c->st;
  if (e == hipSuccess) e = dalloc(c, &c->lam_hist, c->hist_cap);
  if (e == hipSuccess) e = dalloc(c, &c->flag_hist, c->hist_cap);
  if (e == hipSuccess) e = dalloc(c, &c->lam_star_hist, c->hist_cap);
  if (e == hipSuccess) e = dalloc(c, &c->scales, c->hist_cap);
  if (e == hipSuccess) e = dalloc(c, &c->rho_out, 2);
  if (e != hipSuccess) return e;
  Img d;
  e = alloc_image(c, 0, src, d, x);
  if (e != hipSuccess) return e;
  record_image(c, src, d, x);
  Img a = d;  // the stand-alone solve's and search's descriptor (as deconv_init builds it)
  float *lh = nullptr;
  int *fh = nullptr;
  e = dalloc(c, &c->st_aux, 1);
  if (e == hipSuccess) e = dalloc(c, &c->uE_aux, P);
  if (e == hipSuccess) e = dalloc(c, &lh, 1);
  if (e == hipSuccess) e = dalloc(c, &fh, 1);
  if (e != hipSuccess) return e;
  a.uE = c->uE_aux;
  a.st = c->st_aux;
  a.lam_hist = lh;
  a.flag_hist = fh;
  a.lam_star_hist = nullptr;
  a.hist_cap = 1;
  a.scales = nullptr;
  c->aux.imgs.push_back(a);
  c->aux.st_base = c->st_aux;
  e = upload_table(c->aux);
  if (e == hipSuccess) e = upload_table(c->main);
  if (e == hipSuccess) e = build_plans(c);
  return e;
}

// FP64 set-up temporaries of the static path, carved after the problem's own buffers.
struct StaticTemps {
  double *hp = nullptr, *work = nullptr;
  cd *Hd = nullptr, *Yd = nullptr;
  float *ypad = nullptr;
};

static hipError_t carve_static_temps(gfd_ctx *c, const gfd_image &src, StaticTemps &t) {
  int Md, Nd;
  domain_dims(src, Md, Nd);
  const size_t P = (size_t)Md * Nd, nb = make_layout(Md, Nd).bins();
  hipError_t e = dalloc(c, &t.hp, P);
  if (e == hipSuccess) e = dalloc(c, &t.work, 4 * 256);
  if (e == hipSuccess) e = dalloc(c, &t.Hd, nb);
  if (e == hipSuccess) e = dalloc(c, &t.Yd, nb);
  if (e == hipSuccess) e = dalloc(c, &t.ypad, P);
  return e;
}

extern "C" {

const char *gfd_last_error(void) { return g_err.c_str(); }

gfd_status deconv_init(gfd_ctx **out, const float *y, int M, int N, const float *h, int kh, int kw, double sigma2,
                       int w, float eps, double rho, void *stream) {
  g_err.clear();
  gfd_image d;
  d.y = y;
  d.M = M;
  d.N = N;
  d.h = h;
  d.kh = kh;
  d.kw = kw;
  d.sigma2 = sigma2;
  d.w = w;
  d.eps = eps;
  d.rho = rho;
  d.boundary = GFD_BOUNDARY_PERIODIC;
  return init_common(out, &d, 1, (hipStream_t)stream);
}

gfd_status deconv_init_batch(gfd_ctx **out, const gfd_image *images, int count, void *stream) {
  g_err.clear();
  return init_common(out, images, count, (hipStream_t)stream);
}

gfd_status deconv_iterate(gfd_ctx *ctx, int n_iter, float *u_out, float *lambda_out, void *stream) {
  g_err.clear();
  if (!live(ctx)) return fail(GFD_ERR_STATE, "invalid or destroyed context");
  if (n_iter < 0) return fail(GFD_ERR_ARG, "n_iter must be >= 0");
  hipStream_t s = (hipStream_t)stream;
  gfd_status rc = grow_history(ctx, ctx->iters + n_iter, s);
  if (rc != GFD_OK) return rc;
  if (ctx->use_graph && !ctx->gexec && n_iter > 0) {
    rc = capture_graph(ctx);
    if (rc != GFD_OK) return rc;
  }
  for (int i = 0; i < n_iter; ++i) {
    if (ctx->use_graph) HIPCHK(hipGraphLaunch(ctx->gexec, s));
    else HIPCHK(ctx->iter.enqueue(s));
  }
  if (u_out) {
    rc = copy_estimates_out(ctx, u_out, s);
    if (rc != GFD_OK) return rc;
  }
  if (lambda_out && n_iter > 0)
    for (int i = 0; i < ctx->count; ++i)
      HIPCHK(hipMemcpyAsync(lambda_out + (size_t)i * n_iter, ctx->lam_hist + (size_t)i * ctx->hist_cap + ctx->iters,
                            n_iter * sizeof(float), hipMemcpyDeviceToDevice, s));
  ctx->iters += n_iter;
  HIPCHK(mark_done(ctx, s));
  return GFD_OK;
}

gfd_status deconv_profile(gfd_ctx *ctx, int n_iter, float *stage_ms_host, int n_stages, void *stream) {
  g_err.clear();
  if (!live(ctx)) return fail(GFD_ERR_STATE, "invalid or destroyed context");
  if (n_iter < 0 || n_stages < 0 || n_stages > kStages || (n_stages > 0 && !stage_ms_host))
    return fail(GFD_ERR_ARG, "n_iter >= 0, 0 <= n_stages <= 6, stage_ms_host non-NULL");
  hipStream_t s = (hipStream_t)stream;
  gfd_status rc = grow_history(ctx, ctx->iters + n_iter, s);
  if (rc != GFD_OK) return rc;
  hipEvent_t ev[kStages + 1];
  for (int i = 0; i <= kStages; ++i) HIPCHK(hipEventCreate(&ev[i]));
  double acc[kStages] = {0, 0, 0, 0, 0, 0};
  hipError_t e = hipSuccess;
  for (int it = 0; it < n_iter && e == hipSuccess; ++it) {
    e = hipEventRecord(ev[0], s);
    for (int k = 0; k < kStages && e == hipSuccess; ++k) {
      e = ctx->stage[k].enqueue(s);
      if (e == hipSuccess) e = hipEventRecord(ev[k + 1], s);
    }
    if (e == hipSuccess) e = hipEventSynchronize(ev[kStages]);
    for (int k = 0; k < kStages && e == hipSuccess; ++k) {
      float ms = 0.0f;
      e = hipEventElapsedTime(&ms, ev[k], ev[k + 1]);
      acc[k] += ms;
    }
  }
  for (int i = 0; i <= kStages; ++i) (void)hipEventDestroy(ev[i]);
  if (e != hipSuccess) return fail(GFD_ERR_HIP, "profiled iteration failed: %s", hipGetErrorString(e));
  ctx->iters += n_iter;
  HIPCHK(mark_done(ctx, s));
  for (int k = 0; k < n_stages; ++k) stage_ms_host[k] = (float)acc[k];
  return GFD_OK;
}

static gfd_status guided_filter_any(const float *uI, const float *up, float *u, int M, int N, int w, float eps,
                                    bool clip, void *stream) {
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
  HIPCHK(launch_guided_filter_plain(uI, up, u, M, N, w, eps, clip, (hipStream_t)stream));
  return GFD_OK;
}

gfd_status guided_filter(const float *uI, const float *up, float *u, int M, int N, int w, float eps, void *stream) {
  return guided_filter_any(uI, up, u, M, N, w, eps, false, stream);
}

gfd_status guided_filter_clipped(const float *uI, const float *up, float *u, int M, int N, int w, float eps,
                                 void *stream) {
  return guided_filter_any(uI, up, u, M, N, w, eps, true, stream);
}

gfd_status guided_filter_color(const float *I3, const float *up, float *u, int M, int N, int w, float eps,
                               void *stream) {
  g_err.clear();
  if (!I3 || !up || !u) return fail(GFD_ERR_ARG, "I3, up and u must be device pointers");
  if (M < 1 || N < 1 || M > 65536 || N > 65536) return fail(GFD_ERR_SIZE, "M=%d, N=%d out of [1, 65536]", M, N);
  if (w < 1 || w % 2 == 0 || w > M || w > N) return fail(GFD_ERR_ARG, "w=%d must be odd, 1 <= w <= min(M, N)", w);
  if (!(eps > 0.0f) || !isfinite(eps)) return fail(GFD_ERR_ARG, "eps must be finite and > 0");
  const size_t bytes = (size_t)M * N * sizeof(float);
  const char *pu = (const char *)u, *pi = (const char *)I3, *pp = (const char *)up;
  if ((pu < pi + 3 * bytes && pi < pu + bytes) || (pu < pp + bytes && pp < pu + bytes))
    return fail(GFD_ERR_ARG, "u must not overlap I3 or up");
  HIPCHK(launch_guided_filter_color(I3, up, u, M, N, w, eps, (hipStream_t)stream));
  return GFD_OK;
}

gfd_status spectral_solve(gfd_ctx *ctx, const float *uE, float lambda, float *uI, float *up, void *stream) {
  g_err.clear();
  if (!live(ctx)) return fail(GFD_ERR_STATE, "invalid or destroyed context");
  if (ctx->count != 1) return fail(GFD_ERR_STATE, "spectral_solve needs a single-image context");
  if (!uE || !uI || !up) return fail(GFD_ERR_ARG, "uE, uI and up must be device pointers");
  if (!(lambda > 0.0f)) return fail(GFD_ERR_ARG, "lambda must be > 0 (or +inf)");
  hipStream_t s = (hipStream_t)stream;
  const Img &a = ctx->aux.imgs[0];
  const size_t bytes = (size_t)a.L.M * a.L.N * sizeof(float);
  HIPCHK(hipMemcpyAsync(ctx->uE_aux, uE, bytes, hipMemcpyDeviceToDevice, s));
  HIPCHK(launch_state_set_lam(ctx->st_aux, lambda, s));
  HIPCHK(ctx->aux_solve.enqueue(s));
  HIPCHK(hipMemcpyAsync(uI, a.uI, bytes, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(up, a.uP, bytes, hipMemcpyDeviceToDevice, s));
  HIPCHK(mark_done(ctx, s));
  return GFD_OK;
}

gfd_status discrepancy_lambda(gfd_ctx *ctx, const float *uE, float *lambda_dev, void *stream) {
  g_err.clear();
  if (!live(ctx)) return fail(GFD_ERR_STATE, "invalid or destroyed context");
  if (ctx->count != 1) return fail(GFD_ERR_STATE, "discrepancy_lambda needs a single-image context");
  if (!uE || !lambda_dev) return fail(GFD_ERR_ARG, "uE and lambda_dev must be device pointers");
  hipStream_t s = (hipStream_t)stream;
  const Img &a = ctx->aux.imgs[0];
  HIPCHK(hipMemcpyAsync(ctx->uE_aux, uE, (size_t)a.L.M * a.L.N * sizeof(float), hipMemcpyDeviceToDevice, s));
  HIPCHK(launch_state_reset(ctx->st_aux, s));
  HIPCHK(ctx->aux_lam.enqueue(s));
  HIPCHK(launch_copy_lam_star(ctx->st_aux, lambda_dev, s));
  HIPCHK(mark_done(ctx, s));
  return GFD_OK;
}

gfd_status deconv_set_scales(gfd_ctx *ctx, const float *s_dev, int n, void *stream) {
  g_err.clear();
  if (!live(ctx)) return fail(GFD_ERR_STATE, "invalid or destroyed context");
  if (n < 0 || (n > 0 && !s_dev)) return fail(GFD_ERR_ARG, "n must be >= 0 and s_dev non-NULL when n > 0");
  hipStream_t s = (hipStream_t)stream;
  gfd_status rc = grow_history(ctx, ctx->iters + n, s);
  if (rc != GFD_OK) return rc;
  HIPCHK(launch_fill_f(ctx->scales, ctx->hist_cap, 1.0f, s));
  if (n > 0)
    HIPCHK(hipMemcpyAsync(ctx->scales + ctx->iters, s_dev, n * sizeof(float), hipMemcpyDeviceToDevice, s));
  HIPCHK(launch_state_set_nscale(ctx->st, ctx->count, n > 0 ? ctx->iters + n : 0, s));
  HIPCHK(mark_done(ctx, s));
  return GFD_OK;
}

gfd_status deconv_set_estimate(gfd_ctx *ctx, const float *uE, void *stream) {
  g_err.clear();
  if (!live(ctx)) return fail(GFD_ERR_STATE, "invalid or destroyed context");
  if (!uE) return fail(GFD_ERR_ARG, "uE must be a device pointer");
  hipStream_t s = (hipStream_t)stream;
  size_t off = 0;
  for (int i = 0; i < ctx->count; ++i) {
    const ImgMeta &m = ctx->meta[i];
    const size_t P = (size_t)m.Mo * m.No;
    if (m.pad) {  // extended over the padding like the observation
      HIPCHK(launch_pad_ramp(uE + off, m.Mo, m.No, ctx->main.imgs[i].uE, m.M, m.N, s));
      HIPCHK(launch_pad_ramp(uE + off, m.Mo, m.No, ctx->u0[i], m.M, m.N, s));
    } else {
      HIPCHK(hipMemcpyAsync(ctx->main.imgs[i].uE, uE + off, P * sizeof(float), hipMemcpyDeviceToDevice, s));
      HIPCHK(hipMemcpyAsync(ctx->u0[i], uE + off, P * sizeof(float), hipMemcpyDeviceToDevice, s));
    }
    off += P;
  }
  HIPCHK(ctx->warm.enqueue(s));
  ctx->k_start = ctx->iters;
  HIPCHK(mark_done(ctx, s));
  return GFD_OK;
}

gfd_status deconv_reset(gfd_ctx *ctx, void *stream) {
  g_err.clear();
  if (!live(ctx)) return fail(GFD_ERR_STATE, "invalid or destroyed context");
  hipStream_t s = (hipStream_t)stream;
  for (int i = 0; i < ctx->count; ++i) {
    HIPCHK(launch_fill_f(ctx->main.imgs[i].uE, (size_t)ctx->meta[i].M * ctx->meta[i].N, 0.0f, s));
    HIPCHK(launch_fill_f(ctx->u0[i], (size_t)ctx->meta[i].M * ctx->meta[i].N, 0.0f, s));
    HIPCHK(launch_state_reset(ctx->st + i, s));
  }
  HIPCHK(ctx->warm.enqueue(s));
  ctx->iters = 0;
  ctx->k_start = 0;
  HIPCHK(mark_done(ctx, s));
  return GFD_OK;
}

gfd_status deconv_info(gfd_ctx *ctx, double *rho, double *target, int *iterations) {
  g_err.clear();
  if (!live(ctx)) return fail(GFD_ERR_STATE, "invalid or destroyed context");
  if (rho) *rho = ctx->meta[0].rho;
  if (target) *target = ctx->meta[0].T;
  if (iterations) *iterations = ctx->iters;
  return GFD_OK;
}

gfd_status deconv_image_info(gfd_ctx *ctx, int index, int *M, int *N, double *rho, double *target) {
  g_err.clear();
  if (!live(ctx)) return fail(GFD_ERR_STATE, "invalid or destroyed context");
  if (index < 0 || index >= ctx->count) return fail(GFD_ERR_ARG, "index %d outside [0, %d)", index, ctx->count);
  const ImgMeta &m = ctx->meta[index];
  if (M) *M = m.Mo;
  if (N) *N = m.No;
  if (rho) *rho = m.rho;
  if (target) *target = m.T;
  return GFD_OK;
}

gfd_status deconv_image_domain(gfd_ctx *ctx, int index, int *M, int *N, int *boundary) {
  g_err.clear();
  if (!live(ctx)) return fail(GFD_ERR_STATE, "invalid or destroyed context");
  if (index < 0 || index >= ctx->count) return fail(GFD_ERR_ARG, "index %d outside [0, %d)", index, ctx->count);
  const ImgMeta &m = ctx->meta[index];
  if (M) *M = m.M;
  if (N) *N = m.N;
  if (boundary) *boundary = (m.pad ? GFD_BOUNDARY_PAD : 0) | (m.clip ? GFD_BOUNDARY_CLIP : 0);
  return GFD_OK;
}

gfd_status deconv_get_status(gfd_ctx *ctx, unsigned *flags_host) {
  g_err.clear();
  if (!live(ctx)) return fail(GFD_ERR_STATE, "invalid or destroyed context");
  if (!flags_host) return fail(GFD_ERR_ARG, "flags_host is NULL");
  // read on the context's own stream, after the context's last enqueued work
  std::vector<unsigned> f(ctx->count, 0u);
  hipError_t e = hipStreamWaitEvent(ctx->cap_stream, ctx->done_ev, 0);
  for (int i = 0; i < ctx->count && e == hipSuccess; ++i)
    e = hipMemcpyAsync(&f[i], (char *)(ctx->st + i) + offsetof(LamState, flags_all), sizeof(unsigned),
                       hipMemcpyDeviceToHost, ctx->cap_stream);
  // the copies land in f: wait for them whatever happened above, before f goes out of scope
  const hipError_t es = hipStreamSynchronize(ctx->cap_stream);
  if (e == hipSuccess) e = es;
  if (e != hipSuccess) return fail(GFD_ERR_HIP, "deconv_get_status failed: %s", hipGetErrorString(e));
  unsigned all = 0;
  for (unsigned v : f) all |= v;
  *flags_host = all;
  return GFD_OK;
}

gfd_status deconv_set_graph(gfd_ctx *ctx, int use_graph) {
  g_err.clear();
  if (!live(ctx)) return fail(GFD_ERR_STATE, "invalid or destroyed context");
  ctx->use_graph = use_graph ? 1 : 0;
  return GFD_OK;
}

gfd_status deconv_autotune(gfd_ctx *ctx, int iters, int *choice_host, void *stream) {
  g_err.clear();
  if (!live(ctx)) return fail(GFD_ERR_STATE, "invalid or destroyed context");
  if (ctx->iters != 0) return fail(GFD_ERR_STATE, "deconv_autotune needs a context with no iterations run");
  if (iters < 0 || iters > 64) return fail(GFD_ERR_ARG, "iters must be in [0, 64] (0: default 4)");
  // Multi-image contexts are not tuned: their trials (a graph of parallel branches captured,
  // instantiated, replayed and destroyed a dozen times in a row) twice ended in a host
  // segmentation fault inside the HIP runtime whose cause has not been found; set their launch
  // shapes with deconv_set_tuning.
  if (ctx->count > 1)
    return fail(GFD_ERR_UNIMPLEMENTED, "deconv_autotune tunes single-image contexts only (use deconv_set_tuning)");
  const int n = iters == 0 ? 4 : std::max(iters, 2);
  hipStream_t s = (hipStream_t)stream;
  gfd_ctx *c = ctx;
  // the trial iterations advance the estimate and the search state: keep copies
  HIPCHK(hipStreamSynchronize(s));
  // the search states are kept on the device, so every trial restores them with a device copy
  LamState *st_save = nullptr;
  HIPCHK(hipMalloc((void **)&st_save, c->count * sizeof(LamState)));
  std::vector<float *> ue_save(c->count, nullptr);
  auto release = [&]() {
    for (float *p : ue_save)
      if (p) (void)hipFree(p);
    (void)hipFree(st_save);
  };
  {
    const hipError_t e = hipMemcpy(st_save, c->st, c->count * sizeof(LamState), hipMemcpyDeviceToDevice);
    if (e != hipSuccess) {
      release();
      return fail(GFD_ERR_HIP, "autotune set-up failed: %s", hipGetErrorString(e));
    }
  }
  for (int i = 0; i < c->count; ++i) {
    const size_t P = (size_t)c->meta[i].M * c->meta[i].N;
    hipError_t e = hipMalloc((void **)&ue_save[i], P * sizeof(float));
    if (e == hipSuccess) e = hipMemcpy(ue_save[i], c->main.imgs[i].uE, P * sizeof(float), hipMemcpyDeviceToDevice);
    if (e != hipSuccess) {
      release();
      return fail(e == hipErrorOutOfMemory ? GFD_ERR_NOMEM : GFD_ERR_HIP, "autotune set-up failed: %s",
                  hipGetErrorString(e));
    }
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  gfd_status rc = GFD_OK;
  auto trial = [&](const Tuning &t, float &ms) -> bool {
    hipError_t e = apply_tuning(c, t);
    if (e != hipSuccess) {
      rc = fail(GFD_ERR_HIP, "autotune rebuild failed: %s", hipGetErrorString(e));
      return false;
    }
    if ((rc = capture_graph(c)) != GFD_OK) return false;
    // every trial runs the same iterations: from the saved estimate and search state
    for (int i = 0; i < c->count && e == hipSuccess; ++i) {
      const size_t P = (size_t)c->meta[i].M * c->meta[i].N;
      e = hipMemcpyAsync(c->main.imgs[i].uE, ue_save[i], P * sizeof(float), hipMemcpyDeviceToDevice, s);
    }
    if (e == hipSuccess)
      e = hipMemcpyAsync(c->st, st_save, c->count * sizeof(LamState), hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipGraphLaunch(c->gexec, s);  // warm-up replay
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int k = 0; k < n && e == hipSuccess; ++k) e = hipGraphLaunch(c->gexec, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) {
      rc = fail(GFD_ERR_HIP, "autotune trial failed: %s", hipGetErrorString(e));
      return false;
    }
    return true;
  };
  // coordinate descent over the knobs, starting from the defaults with the filter's strip height
  // set to the lowest one whose strips of image 0 fit on the device at once (when there is one);
  // the strip heights tried are a ladder plus that one
  const int fill = gf_fill_height(c->main.imgs[0]);
  Tuning best{};
  best.gf_ty = fill;
  float best_ms = 0.0f;
  bool ok = trial(best, best_ms);
  int gf_ty[8] = {32, 48, 64, 80, 96, 112, 128, 0};
  int ngf = 7;
  {
    bool have = fill == 0;
    for (int i = 0; i < ngf; ++i) have = have || gf_ty[i] == fill;
    if (!have) gf_ty[ngf++] = fill;
  }
  const int seqs[] = {1, 2, 4};
  const int rows[] = {2, 4, 8, 16};
  const int radices[] = {8, 4};
  // the LDS-resident transforms' knobs only where an image uses them (a side that is not a
  // power of two in [256, 4096])
  bool lds_rows = false, lds_any = false;
  for (const Img &d : c->main.imgs) {
    lds_rows = lds_rows || !reg_plan_ok(d.L.N);
    lds_any = lds_any || !reg_plan_ok(d.L.N) || !reg_plan_ok(d.L.M);
  }
  for (int knob = 0; knob < kTuningKnobs && ok; ++knob) {
    if ((knob == 3 && !lds_rows) || (knob == 4 && !lds_any)) continue;
    const int *vals = knob == 0 ? gf_ty : knob <= 2 ? seqs : knob == 3 ? rows : radices;
    const int nv = knob == 0 ? ngf : knob <= 2 ? 3 : knob == 3 ? 4 : 2;
    for (int v = 0; v < nv && ok; ++v) {
      Tuning t = best;
      int &field = knob == 0 ? t.gf_ty : knob == 1 ? t.seq_fwd : knob == 2 ? t.seq_inv : knob == 3 ? t.rows_lds : t.radix;
      field = vals[v];
      float ms = 0.0f;
      ok = trial(t, ms);
      if (ok && ms < 0.99f * best_ms) {
        best = t;
        best_ms = ms;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  hipError_t e = ok ? apply_tuning(c, best) : hipSuccess;
  // back to the state before the trials
  for (int i = 0; i < c->count && e == hipSuccess; ++i) {
    const size_t P = (size_t)c->meta[i].M * c->meta[i].N;
    e = hipMemcpy(c->main.imgs[i].uE, ue_save[i], P * sizeof(float), hipMemcpyDeviceToDevice);
  }
  if (e == hipSuccess) e = hipMemcpy(c->st, st_save, c->count * sizeof(LamState), hipMemcpyDeviceToDevice);
  release();
  if (!ok) return rc;
  if (e != hipSuccess) return fail(GFD_ERR_HIP, "autotune restore failed: %s", hipGetErrorString(e));
  if (choice_host) {
    const Img &d = c->main.imgs[0];
    choice_host[0] = d.gfTY;
    choice_host[1] = d.L.Rf / 2;
    choice_host[2] = d.L.Ri;
    choice_host[3] = d.L.R;
    choice_host[4] = best.radix == 4 ? 4 : 8;
  }
  return GFD_OK;
}

gfd_status deconv_set_tuning(gfd_ctx *ctx, const int *choice_host) {
  g_err.clear();
  if (!live(ctx)) return fail(GFD_ERR_STATE, "invalid or destroyed context");
  if (ctx->iters != 0) return fail(GFD_ERR_STATE, "deconv_set_tuning needs a context with no iterations run");
  if (!choice_host) return fail(GFD_ERR_ARG, "choice_host must point to %d ints", kTuningKnobs);
  for (int i = 0; i < kTuningKnobs; ++i)
    if (choice_host[i] < 0) return fail(GFD_ERR_ARG, "launch shapes must be >= 0 (0: default)");
  if (choice_host[4] != 0 && choice_host[4] != 4 && choice_host[4] != 8)
    return fail(GFD_ERR_ARG, "the radix schedule is 0 (default), 8 or 4");
  Tuning t;
  t.gf_ty = choice_host[0];
  t.seq_fwd = choice_host[1];
  t.seq_inv = choice_host[2];
  t.rows_lds = choice_host[3];
  t.radix = choice_host[4] == 8 ? 0 : choice_host[4];
  const hipError_t e = apply_tuning(ctx, t);
  if (e != hipSuccess) return fail(GFD_ERR_HIP, "deconv_set_tuning rebuild failed: %s", hipGetErrorString(e));
  return GFD_OK;
}

gfd_status deconv_backward(gfd_ctx *ctx, const float *grad_u, float *grad_eps_dev, float *grad_scales_dev,
                           int checkpoint_every, void *stream) {
  g_err.clear();
  if (!live(ctx)) return fail(GFD_ERR_STATE, "invalid or destroyed context");
  if (!grad_u) return fail(GFD_ERR_ARG, "grad_u must be a device pointer");
  if (checkpoint_every < 0) return fail(GFD_ERR_ARG, "checkpoint_every must be >= 0 (0: default 5)");
  hipStream_t s = (hipStream_t)stream;
  const int K = ctx->iters - ctx->k_start, k0 = ctx->k_start;
  const int c = checkpoint_every == 0 ? 5 : checkpoint_every;
  if (ctx->bwd && ctx->bwd->hist_cap != ctx->hist_cap) {
    HIPCHK(wait_done(ctx));
    free_bwd(ctx->bwd);
    ctx->bwd = nullptr;
  }
  if (!ctx->bwd) {
    hipError_t e = build_bwd(ctx);
    if (e != hipSuccess) {
      free_bwd(ctx->bwd);
      ctx->bwd = nullptr;
      return fail(e == hipErrorOutOfMemory ? GFD_ERR_NOMEM : GFD_ERR_HIP, "reverse-mode set-up failed: %s",
                  hipGetErrorString(e));
    }
  }
  Bwd *b = ctx->bwd;
  const int nck = K > 0 ? (K + c - 1) / c : 0;
  {
    hipError_t e = bwd_slots(ctx, nck, std::min(c, std::max(K, 1)));
    if (e != hipSuccess)
      return fail(e == hipErrorOutOfMemory ? GFD_ERR_NOMEM : GFD_ERR_HIP, "checkpoint allocation failed: %s",
                  hipGetErrorString(e));
  }
  // incoming gradient (images one after another) and a private copy of the search constants
  size_t off = 0;
  for (int i = 0; i < ctx->count; ++i) {
    const ImgMeta &m = ctx->meta[i];
    const size_t P = (size_t)m.Mo * m.No;
    if (m.pad) {  // the crop's adjoint: zeros over the padding
      HIPCHK(launch_fill_f(b->gu[i], (size_t)m.M * m.N, 0.0f, s));
      HIPCHK(hipMemcpy2DAsync(b->gu[i], m.N * sizeof(float), grad_u + off, m.No * sizeof(float), m.No * sizeof(float),
                              m.Mo, hipMemcpyDeviceToDevice, s));
    } else {
      HIPCHK(hipMemcpyAsync(b->gu[i], grad_u + off, P * sizeof(float), hipMemcpyDeviceToDevice, s));
    }
    off += P;
  }
  HIPCHK(hipMemcpyAsync(b->st, ctx->st, ctx->count * sizeof(LamState), hipMemcpyDeviceToDevice, s));
  // forward replay from the starting estimate, keeping every c-th pre-estimate
  HIPCHK(copy_images(ctx, b->uR, ctx->u0, s));
  for (int k = 0; k < (nck - 1) * c; ++k) {
    if (k % c == 0) HIPCHK(copy_images(ctx, slot(b->ck, k / c), b->uR, s));
    HIPCHK(replay(b, k0 + k, true, s));
  }
  if (nck > 0) HIPCHK(copy_images(ctx, slot(b->ck, nck - 1), b->uR, s));
  // segments in reverse: recompute the segment's pre-estimates, then differentiate it
  for (int j = nck - 1; j >= 0; --j) {
    const int a = j * c, z = std::min(a + c, K);
    if (j != nck - 1) HIPCHK(copy_images(ctx, b->uR, slot(b->ck, j), s));
    for (int k = a; k < z; ++k) {  // forward over the segment, into the positions the adjoint reads
      HIPCHK(launch_bwd_bind(b->bwd, b->seg_dev, b->nseg, k - a, 0, s));
      HIPCHK(replay(b, k0 + k, false, s));
      HIPCHK(launch_bwd_bind(b->bwd, b->seg_dev, b->nseg, k - a, +1, s));
      // the filter also after the segment's last iteration, whose output (in uR) nothing reads:
      // every iteration's first box pass results then come from the same kernel, so gradients
      // do not depend on where the segments end
      HIPCHK(b->gf_save.enqueue(s));
    }
    for (int k = z - 1; k >= a; --k) {
      HIPCHK(launch_bwd_bind(b->bwd, b->seg_dev, b->nseg, k - a, -1, s));
      HIPCHK(adjoint_step(b, k0 + k, s));
    }
  }
  HIPCHK(launch_adj_out(b->bwd, b->one, K, k0, grad_eps_dev, grad_scales_dev, s));
  HIPCHK(mark_done(ctx, s));
  return GFD_OK;
}

gfd_status deconvolve_static(const float *y, int M, int N, const float *h, int kh, int kw, double sigma2, int w,
                             float eps, double rho, int n_iter, float *u_out, float *lambda_out, void *stream) {
  g_err.clear();
  gfd_image d;
  d.y = y;
  d.M = M;
  d.N = N;
  d.h = h;
  d.kh = kh;
  d.kw = kw;
  d.sigma2 = sigma2;
  d.w = w;
  d.eps = eps;
  d.rho = rho;
  d.boundary = GFD_BOUNDARY_PERIODIC;
  {
    gfd_status rc = check_image(d, 0);
    if (rc != GFD_OK) return rc;
  }
  if (n_iter < 0) return fail(GFD_ERR_ARG, "n_iter must be >= 0");
  if (!u_out) return fail(GFD_ERR_ARG, "u_out must be a device pointer");
  // the bytes this problem needs, counted on a dry arena before anything is enqueued
  size_t need = 0;
  {
    Arena dry;
    dry.cap = ~(size_t)0;
    dry.dry = true;
    gfd_ctx c;
    c.arena = &dry;
    StaticTemps t;
    ImgExtra x;
    hipError_t e = carve_static(&c, d, n_iter, x);
    if (e == hipSuccess) e = carve_static_temps(&c, d, t);
    if (e != hipSuccess) return fail(GFD_ERR_HIP, "static layout failed: %s", hipGetErrorString(e));
    need = dry.off;
  }
  if (need > kScratchBytes)
    return fail(GFD_ERR_SIZE, "%dx%d needs %zu bytes of device scratch; the static scratch holds %zu", M, N, need,
                kScratchBytes);
  hipStream_t s = (hipStream_t)stream;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  unsigned char *base = nullptr;
  HIPCHK(scratch_address(dev, &base));
  {
    gfd_status rc = check_psfs(&d, 1, s);  // (waits for `stream`, so also for an earlier call on it)
    if (rc != GFD_OK) return rc;
  }
  // the array keeps the previous call's contents: start from zeros, before the tables go in
  HIPCHK(launch_fill_f((float *)base, (need + 3) / 4, 0.0f, s));
  HIPCHK(hipStreamSynchronize(s));
  Arena arena;
  arena.base = base;
  arena.cap = kScratchBytes;
  gfd_ctx c;
  c.arena = &arena;
  StaticTemps t;
  ImgExtra x;
  HIPCHK(carve_static(&c, d, n_iter, x));
  HIPCHK(carve_static_temps(&c, d, t));
  HIPCHK(launch_fill_f(c.scales, c.hist_cap, 1.0f, s));
  const Img &img = c.main.imgs[0];
  HIPCHK(init_image(&c, 0, d, img, x, s, t.hp, t.Hd, t.Yd, t.work, t.ypad));
  HIPCHK(hipMemcpyAsync(c.st_aux, c.st, sizeof(LamState), hipMemcpyDeviceToDevice, s));
  HIPCHK(launch_state_reset(c.st_aux, s));
  HIPCHK(c.warm.enqueue(s));
  for (int k = 0; k < n_iter; ++k) HIPCHK(c.iter.enqueue(s));
  HIPCHK(hipMemcpyAsync(u_out, img.uE, (size_t)M * N * sizeof(float), hipMemcpyDeviceToDevice, s));
  if (lambda_out && n_iter > 0)
    HIPCHK(hipMemcpyAsync(lambda_out, c.lam_hist, n_iter * sizeof(float), hipMemcpyDeviceToDevice, s));
  return GFD_OK;
}

void deconv_destroy(gfd_ctx *ctx) {
  if (!ctx) return;
  {
    std::lock_guard<std::mutex> g(g_live_mu);
    if (!g_live.count(ctx)) return;
    g_live.erase(ctx);
  }
  (void)wait_done(ctx);
  free_ctx(ctx);
}

}  // extern "C"
