// Discrepancy-principle search for lambda (Sec. 3.2, Eqs.(10)-(11)) as a small state machine.
//
// The device kernels evaluate, for a handful of candidate values lambda_j, the compensated
// FP32 sums   S_j  = sum_b q_b g_j(b),   D_j = sum_b q_b g_j(b) (1 - r_j(b)),
// with q_b the Hermitian-weighted |R_b|^2, t_b = |H_b|^2, r = 1 / (1 + t_b / lambda_j) and
// g = r^2, so that f(lambda_j) = S_j / P is the left-hand side of Eq.(11) and
// d ln f / d ln lambda = 2 D_j / S_j.  The root f = T is unique because f increases with
// lambda (Sec. 3.2).  After every evaluation round one thread calls the functions below,
// which keep a bracket [llo, lhi] with f(llo) < T <= f(lhi) and choose the next candidates:
// uniform k-section while the bracket is wide, then points clustered around the root of the
// cubic Hermite interpolant of ln f over ln lambda.  Only FP32 arithmetic is used.
//
// The code is plain C++ usable on the host (unit tests) and on the device.
#pragma once
#include <math.h>

#if defined(__HIPCC__)
#define GFD_HD __host__ __device__
#else
#define GFD_HD
#endif

// Quotients and exponentials whose last bits do not matter (candidate placement, bracket
// bookkeeping, Newton steps) use the hardware approximations on the device: this code runs on
// one thread, where every accurately rounded division or exponential is a long dependent chain.
#if defined(__HIP_DEVICE_COMPILE__)
#define GFD_QDIV(a, b) __fdividef((a), (b))
#define GFD_QEXP(x) __expf(x)
#else
#define GFD_QDIV(a, b) ((a) / (b))
#define GFD_QEXP(x) expf(x)
#endif

namespace gfd {

constexpr int kLamMaxCand = 8;     // candidates per evaluation round
// candidates folded into the residual pass: around the previous lambda_star the first round
// decides as often with 4 as with 8 (the spacing follows the last change), and each one costs
// a reciprocal and six more operations per bin in that pass
constexpr int kLamFirstCand = 4;
constexpr float kLamFloor = 1e-30f;
constexpr float kLamCeil = 1e30f;
// evaluation rounds after the first one: per iteration (the rounds a captured iteration
// holds) and for a search that may start cold (warm start, stand-alone search)
constexpr int kLamSweeps = 3;
constexpr int kLamSweepsFull = 10;

// kFlagUnconverged: the round limit forced a decision while the bracket was still wider than
// the convergence test allows (lambda is then the interpolated estimate, not a root to FP32
// accuracy)
enum : int { kFlagInf = 1, kFlagNoRoot = 2, kFlagNonFinite = 4, kFlagUnconverged = 8 };

struct LamState {
  // constants of the image
  float TP;          // target times P: rho * P^2 * sigma^2 (sums are compared against this)
  float invP;
  // iteration bookkeeping
  int k;             // index of the current iteration
  int nscale;        // number of valid entries in the scale array
  int phase;         // 0: searching, 1: lambda fixed for this iteration
  int flags;         // flags of the current iteration
  unsigned flags_all;
  int rounds;        // evaluation rounds used this iteration
  float Einf;        // ||h * u_E - y||^2 of this iteration
  float lam_star, lam;
  float lam_prev;    // last finite lambda_star (0 = none): centre of the first candidates
  float lam_prev2;   // the one before (0 = none): their ratio sets the first spacing
  // bracket
  int haslo, hashi;
  float llo, lhi, Flo, Fhi, Dlo, Dhi;
  int nc;
  float cand[kLamMaxCand];
  float mu[kLamMaxCand];  // 1 / cand
  // offsets subtracted from u_I and u_p inside the guided filter (their means)
  float meanI, meanP;
  int done;   // blocks of the running evaluation round that have stored their partial sums
  int round;  // -1: search opened by the residual pass; r >= 0: candidates of round r published
};

// Work queue of one launch of the search (shared by the images of the launch), all zero between
// launches: next entry to take, blocks that have left, images whose lambda the launch has fixed,
// starts done, and the images whose start left the search open (open[0 .. nopen), room for
// every image of the set follows the header).
struct LamQueue {
  int next, exits, closed, begun, nopen;
  int open[1];
};
inline size_t lam_queue_bytes(int nimg) { return sizeof(LamQueue) + sizeof(int) * (size_t)(nimg > 1 ? nimg - 1 : 0); }

GFD_HD inline float lam_relF(float hi, float lo, float TP) {
  // f / T - 1 with the subtraction done exactly when hi is close to TP
  return GFD_QDIV((hi - TP) + lo, TP);
}

GFD_HD inline void lam_set_cand(LamState &s, int n, const float *c) {
  s.nc = n;
  for (int j = 0; j < n; ++j) {
    float v = fminf(fmaxf(c[j], kLamFloor), kLamCeil);
    s.cand[j] = v;
    s.mu[j] = GFD_QDIV(1.0f, v);
  }
}

// First candidates of an iteration: around the previous lambda_star when there is one, spaced
// by the size of the last change (so that a settled sequence is bracketed tightly and a jump
// is still caught), otherwise spread over the whole admissible range.  Around the previous
// root two close candidates (+-sp/2) give a tight bracket for a settled sequence and two far
// ones (+-3.5 sp) catch a jump.
GFD_HD inline void lam_first_candidates(LamState &s) {
  static_assert(kLamFirstCand == 4, "offsets below are for four candidates");
  const float off[kLamFirstCand] = {-3.5f, -0.5f, 0.5f, 3.5f};
  float c[kLamFirstCand];
  if (s.lam_prev > 0.0f) {
    float sp = 1.0f;
    if (s.lam_prev2 > 0.0f) sp = fminf(fmaxf(1.5f * fabsf(logf(s.lam_prev / s.lam_prev2)), 0.02f), 1.0f);
    for (int j = 0; j < kLamFirstCand; ++j) c[j] = s.lam_prev * GFD_QEXP(sp * off[j]);
  } else {
    const float x0 = logf(kLamFloor), x1 = logf(kLamCeil);
    for (int j = 0; j < kLamFirstCand; ++j)
      c[j] = expf(x0 + (x1 - x0) * ((float)j + 0.5f) / (float)kLamFirstCand);
  }
  lam_set_cand(s, kLamFirstCand, c);
}

// Fold one round of evaluations into the bracket.
GFD_HD inline void lam_absorb(LamState &s, int n, const float *cand, const float *Shi, const float *Slo,
                              const float *Dsum) {
  for (int j = 0; j < n; ++j) {
    float F = lam_relF(Shi[j], Slo[j], s.TP);
    float S = Shi[j] + Slo[j];
    float D = S > 0.0f ? GFD_QDIV(2.0f * Dsum[j], S) : 0.0f;
    if (F < 0.0f) {
      if (!s.haslo || cand[j] > s.llo) { s.haslo = 1; s.llo = cand[j]; s.Flo = F; s.Dlo = D; }
    } else {
      if (!s.hashi || cand[j] < s.lhi) { s.hashi = 1; s.lhi = cand[j]; s.Fhi = F; s.Dhi = D; }
    }
  }
}

// Root in tau in [0, 1] of the cubic Hermite interpolant with values G0 < 0 <= G1 and slopes
// d0, d1 (already multiplied by the interval length).
GFD_HD inline float hermite_root(float G0, float G1, float d0, float d1, float tau_guess) {
  float lo = 0.0f, hi = 1.0f, t = fminf(fmaxf(tau_guess, 0.0f), 1.0f);
  for (int it = 0; it < 30; ++it) {
    float t2 = t * t, t3 = t2 * t;
    float p = (2 * t3 - 3 * t2 + 1) * G0 + (t3 - 2 * t2 + t) * d0 + (-2 * t3 + 3 * t2) * G1 + (t3 - t2) * d1;
    float dp = (6 * t2 - 6 * t) * G0 + (3 * t2 - 4 * t + 1) * d0 + (-6 * t2 + 6 * t) * G1 + (3 * t2 - 2 * t) * d1;
    if (p < 0.0f) lo = t; else hi = t;
    float tn = (dp > 0.0f) ? t - GFD_QDIV(p, dp) : -1.0f;
    if (!(tn > lo && tn < hi)) tn = 0.5f * (lo + hi);
    // converged to FP32 resolution (Newton may then alternate between neighbouring floats)
    if (fabsf(tn - t) <= 4.0f * 1.1920929e-7f * fmaxf(t, 1e-3f)) { t = tn; break; }
    t = tn;
  }
  return t;
}

// Estimate of the root from the current bracket; returns the ln-lambda error proxy.
GFD_HD inline float lam_estimate(const LamState &s, float &lam_est, float &width) {
  width = log1pf((s.lhi - s.llo) / s.llo);          // ln(lhi / llo)
  float G0 = log1pf(s.Flo), G1 = log1pf(s.Fhi);     // ln(f / T) at both ends
  float ts = (G1 > G0) ? -G0 / (G1 - G0) : 0.5f;    // secant
  float th = hermite_root(G0, G1, s.Dlo * width, s.Dhi * width, ts);
  lam_est = s.llo + s.llo * expm1f(th * width);
  return fabsf(th - ts) * width;
}

// Decide after a round: either fix lambda (phase = 1) or load the next candidates.
// `last` forces a decision (and raises kFlagUnconverged if the bracket has not converged).
// Returns 1 if lambda is fixed.
GFD_HD inline int lam_decide(LamState &s, bool last) {
  s.rounds += 1;
  float next[kLamMaxCand];
  const int n = kLamMaxCand;
  if (s.haslo && s.hashi) {
    if (!(s.llo < s.lhi)) {  // inconsistent (rounding noise at the root): take the midpoint
      s.lam_star = 0.5f * (s.llo + s.lhi);
      s.phase = 1;
      return 1;
    }
    float est, width;
    float err = lam_estimate(s, est, width);
    // The secant-Hermite gap err is the secant's error; the Hermite estimate's own error is of
    // the order of err^2 once the bracket is narrow enough for ln f to be smooth across it.
    const bool conv = width <= 1e-6f || (err <= 1e-4f && width <= 0.05f);
    if (last || conv) {
      if (!conv) s.flags |= kFlagUnconverged;
      s.lam_star = est;
      s.phase = 1;
      return 1;
    }
    // One end still the floor or the ceiling while the other is a measured point (the root moved
    // past the first candidates): march geometrically away from the measured end, doubling the
    // step, so that a moderate jump is bracketed tightly in one round.
    const bool lo_open = s.llo <= kLamFloor, hi_open = s.lhi >= kLamCeil;
    if (width > 1.0f && lo_open != hi_open) {
      const float d0 = 0.125f;
      for (int j = 0; j < n; ++j) {
        const float x = fminf(d0 * (float)(1 << j), 0.999f * width);
        next[j] = hi_open ? s.llo * GFD_QEXP(x) : s.lhi * GFD_QEXP(-x);
      }
    } else if (width > 1.0f || !(err > 0.0f)) {
      for (int j = 0; j < n; ++j) next[j] = s.llo * GFD_QEXP(width * (float)(j + 1) / (float)(n + 1));
    } else {
      float h = fmaxf(4.0f * err, 1e-7f);
      if (h * (float)(n + 1) >= width) {
        for (int j = 0; j < n; ++j) next[j] = s.llo * GFD_QEXP(width * (float)(j + 1) / (float)(n + 1));
      } else {
        // clustered around the estimate, kept strictly inside the bracket
        float xe = logf(est / s.llo);
        xe = fminf(fmaxf(xe, 0.5f * h * (float)(n + 1)), width - 0.5f * h * (float)(n + 1));
        for (int j = 0; j < n; ++j) next[j] = s.llo * GFD_QEXP(xe + h * ((float)j - 0.5f * (float)(n - 1)));
      }
    }
    lam_set_cand(s, n, next);
    return 0;
  }
  // not bracketed yet: march outwards in large geometric steps
  const float step = 6.0f;
  if (s.haslo) {
    if (last || s.llo >= kLamCeil) {
      if (s.llo < kLamCeil) s.flags |= kFlagUnconverged;
      s.lam_star = s.llo;
      s.phase = 1;
      return 1;
    }
    for (int j = 0; j < kLamMaxCand; ++j) next[j] = s.llo * GFD_QEXP(step * (float)(j + 1));
  } else {
    if (last || s.lhi <= kLamFloor) {
      if (s.lhi > kLamFloor) s.flags |= kFlagUnconverged;
      s.lam_star = s.lhi;
      s.phase = 1;
      return 1;
    }
    for (int j = 0; j < kLamMaxCand; ++j) next[j] = s.lhi * GFD_QEXP(-step * (float)(j + 1));
  }
  lam_set_cand(s, kLamMaxCand, next);
  return 0;
}

// Start of an iteration after the residual pass: Einf = sum q / P, Sfloor = sum q g(floor).
// Returns 1 if lambda is already fixed (infinite branch or no root).
GFD_HD inline int lam_begin(LamState &s, float Ehi, float Elo, float Fl_hi, float Fl_lo, int n,
                            const float *cand, const float *Shi, const float *Slo, const float *Dsum) {
  s.rounds = 0;
  s.haslo = s.hashi = 0;
  s.Einf = (Ehi + Elo) * s.invP;
  if (!(Ehi == Ehi) || isinf(Ehi)) {
    s.flags |= kFlagNonFinite;
  }
  if ((Ehi - s.TP) + Elo <= 0.0f) {          // u_E in K: lambda = +inf (ties take the branch)
    s.flags |= kFlagInf;
    s.lam_star = INFINITY;
    s.phase = 1;
    return 1;
  }
  if ((Fl_hi - s.TP) + Fl_lo >= 0.0f) {      // even the floor overshoots: no root
    s.flags |= kFlagNoRoot;
    s.lam_star = kLamFloor;
    s.phase = 1;
    return 1;
  }
  s.haslo = 1;                                // the floor is a valid lower end
  s.llo = kLamFloor;
  s.Flo = lam_relF(Fl_hi, Fl_lo, s.TP);
  s.Dlo = 0.0f;
  s.hashi = 1;                                // lambda -> inf gives Einf > T
  s.lhi = kLamCeil;
  s.Fhi = lam_relF(Ehi, Elo, s.TP);
  s.Dhi = 0.0f;
  lam_absorb(s, n, cand, Shi, Slo, Dsum);
  return lam_decide(s, false);
}

}  // namespace gfd
