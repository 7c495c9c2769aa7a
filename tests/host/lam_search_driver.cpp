// Host driver for the lambda-search state machine of the HIP library (lam_search.h): the
// candidate sums are evaluated here in double and handed over as (hi, lo) float pairs, the
// way the device reductions deliver them.  Test infrastructure only.
#include <math.h>
#include <stddef.h>

#include "lam_search.h"

using namespace gfd;

static void sums(const float *q, const float *t, size_t n, int nc, const float *mu, float *hi, float *lo, float *ds) {
  for (int j = 0; j < nc; ++j) {
    double s = 0.0, d = 0.0;
    for (size_t i = 0; i < n; ++i) {
      float r = 1.0f / fmaf(t[i], mu[j], 1.0f);
      double qg = (double)q[i] * (double)r * (double)r;
      s += qg;
      d += qg * (1.0 - (double)r);
    }
    hi[j] = (float)s;
    lo[j] = (float)(s - (double)hi[j]);
    ds[j] = (float)d;
  }
}

// The round limits the library launches: after the first round, per iteration (full = 0) and
// for a warm start or a stand-alone search (full = 1).
extern "C" int lam_rounds(int full) { return full ? kLamSweepsFull : kLamSweeps; }

extern "C" int lam_search_host(const float *q, const float *t, size_t n, float TP, float lam_prev, int rounds,
                               float *lam_out, int *rounds_used) {
  LamState s = {};
  s.TP = TP;
  s.invP = 1.0f;
  s.lam_prev = lam_prev;
  lam_first_candidates(s);
  float hi[2 + kLamMaxCand], lo[2 + kLamMaxCand], ds[kLamMaxCand];
  // Einf and the floor
  double E = 0.0, Fl = 0.0;
  for (size_t i = 0; i < n; ++i) {
    E += q[i];
    float r = 1.0f / fmaf(t[i], 1.0f / kLamFloor, 1.0f);
    Fl += (double)q[i] * r * r;
  }
  float Eh = (float)E, El = (float)(E - (double)Eh), Fh = (float)Fl, Flo = (float)(Fl - (double)Fh);
  sums(q, t, n, s.nc, s.mu, hi, lo, ds);
  float cand[kLamMaxCand];
  for (int j = 0; j < s.nc; ++j) cand[j] = s.cand[j];
  int done = lam_begin(s, Eh, El, Fh, Flo, s.nc, cand, hi, lo, ds);
  for (int k = 0; k < rounds && !done; ++k) {
    sums(q, t, n, s.nc, s.mu, hi, lo, ds);
    for (int j = 0; j < s.nc; ++j) cand[j] = s.cand[j];
    lam_absorb(s, s.nc, cand, hi, lo, ds);
    done = lam_decide(s, k == rounds - 1);
  }
  *lam_out = s.lam_star;
  *rounds_used = s.rounds;
  return s.flags;
}

// Sequence of searches with the warm start carried over, as the iteration does: the lambda,
// rounds used and flags of every search.
extern "C" int lam_search_sequence(const float *q, const float *t, size_t n, const float *TP, int nseq, int rounds,
                                   float *lam_out, int *rounds_used, int *flags_out) {
  LamState s = {};
  s.invP = 1.0f;
  float hi[kLamMaxCand], lo[kLamMaxCand], ds[kLamMaxCand], cand[kLamMaxCand];
  for (int it = 0; it < nseq; ++it) {
    s.TP = TP[it];
    s.phase = 0;
    s.flags = 0;
    lam_first_candidates(s);
    double E = 0.0, Fl = 0.0;
    for (size_t i = 0; i < n; ++i) {
      E += q[i];
      float r = 1.0f / fmaf(t[i], 1.0f / kLamFloor, 1.0f);
      Fl += (double)q[i] * r * r;
    }
    float Eh = (float)E, El = (float)(E - (double)Eh), Fh = (float)Fl, Flo = (float)(Fl - (double)Fh);
    sums(q, t, n, s.nc, s.mu, hi, lo, ds);
    for (int j = 0; j < s.nc; ++j) cand[j] = s.cand[j];
    int done = lam_begin(s, Eh, El, Fh, Flo, s.nc, cand, hi, lo, ds);
    for (int k = 0; k < rounds && !done; ++k) {
      sums(q, t, n, s.nc, s.mu, hi, lo, ds);
      for (int j = 0; j < s.nc; ++j) cand[j] = s.cand[j];
      lam_absorb(s, s.nc, cand, hi, lo, ds);
      done = lam_decide(s, k == rounds - 1);
    }
    lam_out[it] = s.lam_star;
    rounds_used[it] = s.rounds;
    flags_out[it] = s.flags;
    if (!isinf(s.lam_star) && !(s.flags & kFlagNoRoot)) {
      s.lam_prev2 = s.lam_prev;
      s.lam_prev = s.lam_star;
    }
  }
  return 0;
}
