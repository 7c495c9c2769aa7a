/*
 * gfdeconv.h -- C ABI of the MI355X (gfx950) guided-filter non-blind deconvolution library.
 *
 * Method: Yang, Zhu, Zhang, Huang, "Guided Filter based Edge-preserving Image Non-blind
 * Deconvolution".  The observation model is y = h * u + gamma with white Gaussian noise of
 * variance sigma^2 (Sec. 1, Eq.(1)).  Each iteration (Sec. 3.1, Steps 1-3) chooses lambda by the
 * discrepancy principle (Sec. 3.2, Eqs.(10)-(12)), solves the two Fourier-domain least-squares
 * problems (Eqs.(8)-(9)) for the guidance image u_I and the filtering input u_p, and applies the
 * guided filter u = guidfilter(u_I, u_p, w, eps) (Sec. 2, Eqs.(3)-(5)) to get the next estimate.
 *
 * Conventions shared by every entry point:
 *  - Images are M rows x N columns of contiguous row-major float32 (pitch N), P = M*N.
 *  - Pointers named *_dev or documented as device pointers are device memory on the current
 *    HIP device; they are owned by the caller and must stay valid until the stream has passed
 *    the call.  `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *  - Calls are stream-ordered and asynchronous unless stated otherwise.  The calls on one
 *    context must be ordered: use one stream, or order the streams yourself.  A call that has
 *    to wait for the context's earlier work (deconv_get_status, deconv_destroy, a history
 *    that grows) waits for the stream of the context's last call, never for the whole device.
 *  - Boundaries are periodic everywhere: the blur is a circular convolution and the guided
 *    filter's w x w windows wrap around the image edges.
 *  - Sizes: M and N are products of powers of 2, 3 and 5, each in [2, 4096].
 *  - Arguments are checked before anything is enqueued.  On error a negative status is
 *    returned, a message is stored for gfd_last_error() (per thread) and nothing is written.
 *  - Conditions that arise on the device (NaN input, lambda clamped at its floor, the
 *    lambda = +inf branch) are recorded as flags read with deconv_get_status().
 */
#ifndef GFDECONV_H
#define GFDECONV_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gfd_ctx gfd_ctx; /* opaque, library-owned; bound to the device current at init */
typedef int gfd_status;

enum {
  GFD_OK = 0,
  GFD_ERR_ARG = -1,           /* invalid argument (NULL pointer, w even, eps <= 0, ...) */
  GFD_ERR_SIZE = -2,          /* unsupported image or PSF size */
  GFD_ERR_HIP = -3,           /* a HIP runtime call failed */
  GFD_ERR_NOMEM = -4,         /* device allocation failed */
  GFD_ERR_STATE = -5,         /* context destroyed, foreign, or not usable for this call */
  GFD_ERR_UNIMPLEMENTED = -6  /* valid request outside what this build supports */
};

/* Device-side condition flags (deconv_get_status). */
enum {
  GFD_FLAG_INF_BRANCH = 1u, /* some iteration found u_E in K and used lambda = +inf (Sec. 3.2) */
  GFD_FLAG_NO_ROOT = 2u,    /* some iteration clamped lambda at its floor (no root of Eq.(11)) */
  GFD_FLAG_NONFINITE = 4u,  /* a non-finite value reached a reduction (NaN/Inf in the data) */
  GFD_FLAG_UNCONVERGED = 8u /* some lambda search ran out of evaluation rounds before its bracket
                               met the convergence test: that lambda is the interpolated estimate
                               and Eq.(11) holds only approximately (3 rounds after the first per
                               iteration, 10 for a warm start or a stand-alone search) */
};

/* Widest guided-filter window of the single-pass strip kernels (r = (w-1)/2 <= 8): they keep the
 * last w rows of their inputs and coefficients in registers, one slot per row.  Wider windows,
 * up to w = min(M, N), run as separable box passes (vertical sliding sums, then horizontal FP64
 * prefix sums, each a launch) whose cost per pixel does not depend on w; they need window-sum and
 * coefficient planes: a context allocates 6 float planes per such image at set-up, and each call
 * of a context-free filter allocates its planes stream-ordered (hipMallocAsync / hipFreeAsync on
 * the call's stream: 6 for the grey filters, 17 for the colour filter, plus M x (N + 1) doubles
 * when N > 4096). */
#define GFD_STRIP_MAX_WINDOW 17

/*
 * deconv_init -- per-image set-up (Sec. 3.1 Step 0, plus the transforms the solves need).
 *   y      device, M x N float32: the observation of Eq.(1).
 *   h      device, kh x kw float32, row-major, odd kh <= M and kw <= N: the PSF, centred at
 *          (kh/2, kw/2); it is embedded periodically so that entry (i, j) acts at offset
 *          (i - kh/2, j - kw/2).  Its sum must be non-zero (the solve for u_I divides by F(h) at
 *          the zero frequency).
 *   sigma2 noise variance, >= 0 (on the same intensity scale as y).
 *   w, eps guided-filter window side (odd, 1 <= w <= min(M, N), else GFD_ERR_ARG; windows
 *          wider than GFD_STRIP_MAX_WINDOW take the separable passes) and regulariser (> 0,
 *          finite).
 *   rho    discrepancy factor of the set K (Sec. 3.2), 0 < rho <= 1; rho <= 0 selects Eq.(12).
 * The estimate starts at u_E = 0 (Step 0).  Allocates device memory; synchronises `stream`
 * once at the end so that *out is ready.  *out is untouched on error.
 */
gfd_status deconv_init(gfd_ctx **out, const float *y, int M, int N, const float *h, int kh, int kw,
                       double sigma2, int w, float eps, double rho, void *stream);

/* Boundary handling of an image (gfd_image.boundary, flags that combine). */
enum {
  GFD_BOUNDARY_PERIODIC = 0, /* the paper's model: circular blur, periodic filter windows */
  GFD_BOUNDARY_CLIP = 1,     /* filter windows clipped to the image, means over the pixels inside */
  GFD_BOUNDARY_PAD = 2       /* y is a non-circular blur: solved on a padded domain, then cropped */
};

/*
 * gfd_image -- one image of a batch: the arguments of deconv_init, same meaning and rules,
 * plus `boundary` (0 = GFD_BOUNDARY_PERIODIC gives exactly deconv_init's problem).  Both
 * variants are readings for non-periodic images; the paper's solves (Eqs.(8)-(9)) assume a
 * circular blur and its filter (Eqs.(3)-(5)) full windows.
 *   GFD_BOUNDARY_CLIP: every window mean of the guided filter averages over the window's pixels
 *     inside the (transform-domain) image and divides by their count; windows centred outside
 *     do not exist.  The reverse mode uses the transposed means this implies.
 *   GFD_BOUNDARY_PAD: y (M x N, any sizes in [2, 4096]) sits in the top-left corner of an
 *     M' x N' domain, M' >= M + kh - 1 and N' >= N + kw - 1 the smallest 2^a 3^b 5^c sizes
 *     (<= 4096), filled so that its periodic extension is continuous (each row ramps linearly
 *     from its last value towards its first, then each column likewise).  rho of Eq.(12) is
 *     computed from y, the target counts the observed pixels only (T = rho M N sigma^2), the
 *     iteration runs on the domain, and the caller's arrays (u_out, deconv_set_estimate's uE,
 *     deconv_backward's grad_u) stay M x N: estimates are cropped, a set estimate is extended
 *     like y, a gradient by zeros.  spectral_solve and discrepancy_lambda work on the domain.
 */
typedef struct gfd_image {
  const float *y; /* device, M x N */
  int M, N;
  const float *h; /* device, kh x kw */
  int kh, kw;
  double sigma2;
  int w;
  float eps;
  double rho;
  int boundary; /* GFD_BOUNDARY_* flags */
} gfd_image;

/*
 * deconv_init_batch -- one context for `count` independent images (1 <= count <= 4096), each
 * deconvolved exactly as by its own deconv_init context (Sec. 3.1 per image, its own lambda).
 *   images  host array of `count` descriptors, read during the call only.
 * Every pass of an iteration is one launch over all images (per kernel variant: images are
 * grouped by transform kind and filter radius), so a batch of small images fills the device.
 * On a batch context:
 *   deconv_iterate's u_out holds the estimates one after another in image order (image b
 *   starts at sum_{c<b} M_c N_c floats) and lambda_out is count x n_iter, image-major;
 *   deconv_set_estimate takes the same concatenated layout; deconv_set_scales applies the
 *   scales to every image; deconv_get_status ORs the flags of all images; deconv_info reports
 *   image 0 (deconv_image_info any image).  spectral_solve and discrepancy_lambda need a
 *   single-image context (GFD_ERR_STATE otherwise).
 * Errors name the index of the first offending descriptor; nothing is allocated on error.
 */
gfd_status deconv_init_batch(gfd_ctx **out, const gfd_image *images, int count, void *stream);

/* deconv_image_info -- size, rho and target rho*P*sigma^2 of image `index` of the context. */
gfd_status deconv_image_info(gfd_ctx *ctx, int index, int *M, int *N, double *rho, double *target);

/* deconv_image_domain -- transform-domain size (the padded size under GFD_BOUNDARY_PAD, else
 * the image size) and boundary flags of image `index`; NULL outputs are skipped. */
gfd_status deconv_image_domain(gfd_ctx *ctx, int index, int *M, int *N, int *boundary);

/*
 * deconv_iterate -- run n_iter iterations of Steps 1-3 (Sec. 3.1) from the current estimate.
 *   u_out       device M x N or NULL: receives the estimate after the last iteration.
 *   lambda_out  device, n_iter floats, or NULL: the lambda used at each iteration
 *               (scale * lambda_star), +inf where the Sec. 3.2 branch u_E in K was taken.
 * The whole iteration runs on the device with no host round trip; one iteration is captured
 * once into a HIP graph and replayed.  Iterating in chunks gives the same result as one call.
 */
gfd_status deconv_iterate(gfd_ctx *ctx, int n_iter, float *u_out, float *lambda_out, void *stream);

/*
 * guided_filter -- u = guidfilter(u_I, u_p, w, eps), Sec. 2 Eqs.(3)-(5); context-free.
 *   uI (guidance), up (filtering input), u (output): device M x N float32; u must not alias
 *   uI or up.  Windows are w x w (odd w, 1 <= w <= min(M, N), else GFD_ERR_ARG), wrap
 *   periodically, and every mean divides by w^2.  M, N in [1, 65536] (no factorisation
 *   constraint here).  w > GFD_STRIP_MAX_WINDOW allocates temporaries stream-ordered
 *   (GFD_ERR_HIP if that fails).
 */
gfd_status guided_filter(const float *uI, const float *up, float *u, int M, int N, int w, float eps,
                         void *stream);

/*
 * guided_filter_clipped -- guided_filter with windows clipped to the image: every window mean of
 * Eqs.(3)-(5) averages over the window's pixels inside the M x N image and divides by their
 * count, and only windows centred inside the image carry coefficients (a boundary reading for
 * non-periodic images; the paper's model is periodic).  Arguments and errors as guided_filter.
 */
gfd_status guided_filter_clipped(const float *uI, const float *up, float *u, int M, int N, int w, float eps,
                                 void *stream);

/*
 * guided_filter_color -- the guided filter with a three-channel guide, the colour case of the
 * Sec. 3.1 complexity remark, taken as the multichannel form of Eqs.(3)-(5): per window,
 * a = (Sigma + eps U)^-1 (mean(I p) - mu pbar) with Sigma the guide's 3 x 3 window covariance
 * and U the identity, b = pbar - a . mu, and u = mean(a) . I + mean(b); context-free.
 *   I3 (guidance): device 3 x M x N float32, channel planes one after the other;
 *   up (filtering input) and u (output): device M x N float32; u must not alias I3 or up.
 *   Windows, w, M and N as for guided_filter; eps > 0 and finite.  The 3 x 3 systems are
 *   solved in FP64, everything else in FP32.
 */
gfd_status guided_filter_color(const float *I3, const float *up, float *u, int M, int N, int w, float eps,
                               void *stream);

/*
 * spectral_solve -- the two regularised least-squares solves, Eqs.(8)-(9), for a given
 * pre-estimate and lambda, using the context's F(h), F(y) and gradient symbol.
 *   uE device M x N (input), uI and up device M x N (outputs: gradient- and identity-
 *   regularised solutions).  lambda > 0, or +inf for u_I = u_p = u_E.
 */
gfd_status spectral_solve(gfd_ctx *ctx, const float *uE, float lambda, float *uI, float *up,
                          void *stream);

/*
 * discrepancy_lambda -- lambda_star for the pre-estimate uE by the discrepancy principle
 * (Sec. 3.2, Eqs.(10)-(11)): +inf if ||h*uE - y||^2 <= rho*P*sigma^2, else the root of Eq.(11)
 * (the floor value 1e-30 with GFD_FLAG_NO_ROOT if there is none).
 *   uE device M x N (input); lambda_dev device, 1 float (output).  Does not change the
 *   context's estimate or iteration count.
 */
gfd_status discrepancy_lambda(gfd_ctx *ctx, const float *uE, float *lambda_dev, void *stream);

/*
 * deconv_set_scales -- per-iteration lambda scales s_k (lambda_k = s_k * lambda_star_k),
 * counted from the context's next iteration.  s_dev: device, n floats, copied on `stream`
 * (stream-ordered).  Iterations beyond n use scale 1.  n = 0 clears.
 */
gfd_status deconv_set_scales(gfd_ctx *ctx, const float *s_dev, int n, void *stream);

/* deconv_set_estimate -- replace the current estimate u_E (device M x N, copied). */
gfd_status deconv_set_estimate(gfd_ctx *ctx, const float *uE, void *stream);

/* deconv_reset -- back to Step 0: u_E = 0, iteration count 0, flags cleared. */
gfd_status deconv_reset(gfd_ctx *ctx, void *stream);

/* deconv_info -- host copies of rho, the target rho*P*sigma^2 and the iteration count. */
gfd_status deconv_info(gfd_ctx *ctx, double *rho, double *target, int *iterations);

/* deconv_get_status -- waits for the context's last call (its stream) and returns the OR of the
 * GFD_FLAG_* device flags of every iteration and search since deconv_init or deconv_reset. */
gfd_status deconv_get_status(gfd_ctx *ctx, unsigned *flags_host);

/* deconv_set_graph -- 1 (default): deconv_iterate replays a captured HIP graph; 0: launches
 * the same kernels one by one (same results, bitwise). */
gfd_status deconv_set_graph(gfd_ctx *ctx, int use_graph);

/*
 * deconv_profile -- run n_iter iterations (exactly as deconv_iterate, advancing the estimate)
 * launching the kernels one by one with HIP events between the passes, and return in
 * stage_ms_host[0 .. n_stages) the summed device time of each pass, in this order:
 *   0 row transform of u_E, 1 column transform + residual + first lambda candidates,
 *   2 remaining lambda evaluation rounds, 3 solves (Eqs.(8)-(9)) + column inverse transforms,
 *   4 row inverse transforms, 5 guided filter.
 * n_stages <= 6; synchronises `stream` before returning.
 */
gfd_status deconv_profile(gfd_ctx *ctx, int n_iter, float *stage_ms_host, int n_stages, void *stream);

/*
 * deconv_autotune -- pick launch shapes for this context by timing, one knob at a time
 * (coordinate descent from the defaults, the strip height starting at the lowest one whose
 * strips all fit on the device at once), each candidate over `iters` replays of the captured
 * iteration (0 selects 4; at most 64), keeping the fastest.  The knobs, in choice order:
 *   0 the guided filter's strip height (rows),
 *   1 row pairs per block of the forward power-of-two (register-resident) row transforms,
 *   2 rows per block of the inverse power-of-two row transforms,
 *   3 rows per block of the mixed-radix (LDS-resident) row transforms (only tried when some
 *     image has a side that is not a power of two in [256, 4096]),
 *   4 the radix schedule of the mixed-radix transforms: 8 (radix-8 passes) or 4 (radix-4 passes)
 *     (tried likewise).
 * The transforms give the same result to rounding in every schedule, the filter in every
 * strip height (its running sums restart at strip edges).  Needs a context with no iterations
 * run (after deconv_init or deconv_reset); the estimate and the search state are restored
 * afterwards.  choice_host (5 ints, host, or NULL) receives the five choices for image 0.
 * Synchronises `stream`.  Single-image contexts only: a multi-image context returns
 * GFD_ERR_UNIMPLEMENTED (its trials, graphs of parallel branches re-instantiated in a row, have
 * ended in a host fault inside the HIP runtime); give it launch shapes with deconv_set_tuning.
 */
gfd_status deconv_autotune(gfd_ctx *ctx, int iters, int *choice_host, void *stream);

/*
 * deconv_set_tuning -- set the launch shapes without timing them, in deconv_autotune's order:
 * choice_host (5 ints, host) holds the guided filter's strip height in rows, the row pairs per
 * block of the forward power-of-two row pass, the rows per block of the inverse one, the rows
 * per block of the mixed-radix row passes and the mixed-radix schedule (8 or 4); 0 keeps a
 * default, and a value an image does not admit (not a power of two, odd, or beyond the block's
 * threads or LDS) falls back to the default.  The results agree with other shapes to rounding
 * (as for deconv_autotune).  For repeating a measurement in a chosen shape.  Needs a context
 * with no iterations run; GFD_ERR_ARG for a NULL pointer, a negative value or a schedule other
 * than 0, 4 or 8.
 */
gfd_status deconv_set_tuning(gfd_ctx *ctx, const int *choice_host);

/*
 * deconv_backward -- reverse mode of the iterations run since the estimate was last set
 * (deconv_init, deconv_reset or deconv_set_estimate): given g_u = dLoss/du for the current
 * estimate u^K, the gradient of the loss with respect to the guided-filter regulariser eps
 * (Sec. 2, Eqs.(3)-(5); one eps for all iterations) and to the per-iteration lambda scales s_k
 * (lambda_k = s_k lambda*_k, deconv_set_scales), differentiating through the guided filter, the
 * two solves (Eqs.(8)-(9)), the transforms and, implicitly, through lambda* defined by the
 * discrepancy equation (Sec. 3.2, Eq.(11)).  An iteration that took lambda = +inf passes the
 * gradient through the identity solves and has zero scale gradient.
 *   grad_u           device: the images' g_u, one after another (M x N each).
 *   grad_eps_dev     device, one float per image, or NULL.
 *   grad_scales_dev  device, count x K floats (image-major), or NULL.
 *   checkpoint_every the forward iterations are replayed from their logged lambdas; every
 *                    c-th pre-estimate is kept and each segment of c iterations is recomputed
 *                    before it is differentiated (0 selects c = 5).  Memory: about
 *                    (K / c + 3 c + 16) images per image.  The result does not depend on c.
 * Stream-ordered; allocates device memory on first use.  The context's own estimate, search
 * state and histories are left unchanged.
 */
gfd_status deconv_backward(gfd_ctx *ctx, const float *grad_u, float *grad_eps_dev, float *grad_scales_dev,
                           int checkpoint_every, void *stream);

/*
 * deconvolve_static -- deconv_init followed by deconv_iterate(n_iter) on a one-image problem,
 * for callers that cannot allocate device memory (code that must not call hipMalloc, such as
 * tight serving loops or harnesses that forbid allocation): every device buffer of the problem
 * lives in a fixed 32 MiB array compiled into the library, one per device, held until the
 * process ends.  The call makes no hipMalloc/hipFree and uses no allocating library routine.
 *   y, M, N, h, kh, kw, sigma2, w, eps, rho: as deconv_init (same rules and errors).
 *   n_iter   iterations of Steps 1-3 (Sec. 3.1) from u_E = 0, >= 0.
 *   u_out    device M x N float32: the estimate after n_iter iterations (required).
 *   lambda_out  device, n_iter floats, or NULL: the lambda of each iteration, as deconv_iterate.
 * Results equal those of deconv_init + deconv_iterate bit for bit (same kernels, launched one
 * by one).  A problem whose buffers exceed the array returns GFD_ERR_SIZE before anything is
 * enqueued (512 x 512 and 480 x 640 fit; 1024 x 1024 does not).  The array keeps the previous
 * call's contents and every call clears it first.  Calls that overlap on one device race for
 * its array (this includes calls on different streams and from different threads); order them.
 * Waits for `stream` while it sets up (as deconv_init does); the iterations and the copies to
 * u_out and lambda_out are stream-ordered.
 */
gfd_status deconvolve_static(const float *y, int M, int N, const float *h, int kh, int kw, double sigma2, int w,
                             float eps, double rho, int n_iter, float *u_out, float *lambda_out, void *stream);

/* deconv_destroy -- frees the context; NULL and already-destroyed contexts are ignored. */
void deconv_destroy(gfd_ctx *ctx);

/* gfd_last_error -- message of the last failing call on this thread ("" if none). */
const char *gfd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GFDECONV_H */
