// Register-resident Stockham FFT for power-of-two lengths L = 256 .. 4096.
//
// T = L / 16 threads cooperate on one sequence; thread t keeps the 16 elements
// x[t + T m], m = 0..15, in registers.  A pass of radix R (16, 8, 4 or 2) gives each thread
// 16 / R butterflies j = t + T v whose inputs x[j + i L/R] are exactly its registers
// v + i 16/R; the twiddled R-point DFT outputs go to the Stockham positions
// (j - k) R + k + i s (s = product of the earlier radices, k = j mod s) through LDS, and the
// thread reads back its next inputs.  After the last pass (s R = L) the outputs land on the
// thread's own positions t + T m, so no exchange follows it.  LDS positions are padded by one
// slot every 16 to keep the stride-16 writes of the first pass off a single bank.
#pragma once
#include "fft_lds.h"

namespace gfd {

struct RegPlan {
  int L, T, npass;
  int radix[3];  // radix of each pass (16, 8, 4 or 2)
};

__device__ __forceinline__ int lds_pad(int p) { return p + (p >> 4); }

// 16-point DFT as 4 x 4 with the W16 twiddles in between.
template <int DIR>
__device__ __forceinline__ void dft16(cf *x) {
  const float c1 = 0.92387953251128675613f, s1 = 0.38268343236508977173f, h = 0.70710678118654752440f;
  cf a[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    cf y[4] = {x[n2], x[n2 + 4], x[n2 + 8], x[n2 + 12]};
    dft4<DIR>(y);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) a[n2][k1] = y[k1];
  }
  // a[n2][k1] *= W16^(n2 k1), W16 = exp(DIR i 2 pi / 16)
  const float D = (float)DIR;
  a[1][1] = cmul(a[1][1], cf{c1, D * s1});
  a[1][2] = cmul(a[1][2], cf{h, D * h});
  a[1][3] = cmul(a[1][3], cf{s1, D * c1});
  a[2][1] = cmul(a[2][1], cf{h, D * h});
  a[2][2] = mul_i<DIR>(a[2][2]);
  a[2][3] = cmul(a[2][3], cf{-h, D * h});
  a[3][1] = cmul(a[3][1], cf{s1, D * c1});
  a[3][2] = cmul(a[3][2], cf{-h, D * h});
  a[3][3] = cmul(a[3][3], cf{-c1, -D * s1});
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    cf z[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
    dft4<DIR>(z);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) x[k1 + 4 * k2] = z[k2];
  }
}

template <int R, int DIR>
__device__ __forceinline__ void dftR(cf *x) {
  if constexpr (R == 16) dft16<DIR>(x);
  else if constexpr (R == 8) dft8<DIR>(x);
  else if constexpr (R == 4) dft4<DIR>(x);
  else dft2<DIR>(x);
}

// Twiddle source from the image's FP32 table in global memory, tw[e] = w_L^e (the column
// inverse's transforms).
struct TwGlobal {
  const GFD_AS1 cf *__restrict__ tw;
  __device__ __forceinline__ cf operator()(int e) const { return E(tw, (uint32_t)e); }
  // twiddle i of butterfly k of the compile-time pass with span S and stride TS: w_L^(i k TS)
  template <int S, int TS>
  __device__ __forceinline__ cf at(int k, int i) const { return (*this)(i * (k * TS)); }
};

// Twiddle source from two 64-entry tables in LDS: w_L^e = w_L^(64 (e / 64)) w_L^(e % 64) for
// e < 4096 (`lo` holds w_L^j, `hi` w_L^(64 j)).  Reads of LDS leave the vector-memory counter
// alone, so loads issued before a transform are not waited for at its twiddles.
struct TwSplit {
  const cf *lo, *hi;
  __device__ __forceinline__ cf operator()(int e) const { return cmul(hi[e >> 6], lo[e & 63]); }
  template <int S, int TS>
  __device__ __forceinline__ cf at(int k, int i) const { return (*this)(i * (k * TS)); }
};

// Twiddle source from a butterfly-major table in global memory for the compile-time transforms:
// row r holds the 16 twiddles w_L^(i k TS), i = 0..15, of butterfly k of one pass (rows 0..15:
// the pass of span 16, k < 16, TS = L / 256; rows 16..271: the pass of span 256, k < 256,
// TS = 1).  A butterfly's twiddles are then one 128-byte row reached from one address with
// immediate offsets, where w_L^(i k TS) taken from the plain table needs an index per i.
constexpr int kRegTwRows = 16 + 256;
struct TwTable {
  const GFD_AS1 cf *__restrict__ tab;
  template <int S, int TS>
  __device__ __forceinline__ cf at(int k, int i) const {
    static_assert(S == 16 || S == 256, "passes after the first");
    constexpr int row0 = S == 16 ? 0 : 16;
    return E(tab, (uint32_t)((row0 + k) * 16 + i));
  }
};

// One pass.  `lds` addresses the sequence's region: slot(p) = lds[lds_pad(p) * ls].
// Inactive threads (blocks sized for a larger image of a batch) only join the barriers.
template <int R, int DIR>
__device__ __forceinline__ void reg_pass(cf (&v)[16], int t, int T, int s, int L, bool last, bool active, cf *lds,
                                         int ls, const GFD_AS1 cf *__restrict__ tw) {
  constexpr int NBF = 16 / R;
  const int tstride = L / (s * R);
#pragma unroll
  for (int b = 0; b < NBF; ++b) {
    const int j = t + T * b;
    const int k = j & (s - 1);
    cf x[R];
#pragma unroll
    for (int i = 0; i < R; ++i) x[i] = v[b + i * NBF];
    if (s > 1 && active) {
#pragma unroll
      for (int i = 1; i < R; ++i) {
        cf w = E(tw, (uint32_t)(i * k * tstride));
        if (DIR > 0) w.im = -w.im;
        x[i] = cmul(x[i], w);
      }
    }
    dftR<R, DIR>(x);
    if (last) {
#pragma unroll
      for (int i = 0; i < R; ++i) v[b + i * NBF] = x[i];
    } else if (active) {
      const int base = (j - k) * R + k;
#pragma unroll
      for (int i = 0; i < R; ++i) lds[lds_pad(base + i * s) * ls] = x[i];
    }
  }
  if (!last) {
    __syncthreads();
    if (active) {
#pragma unroll
      for (int m = 0; m < 16; ++m) v[m] = lds[lds_pad(t + T * m) * ls];
    }
    __syncthreads();
  }
}

// Whole transform.  On entry v[m] = x[t + T m]; on exit v[m] = X[t + T m] (unnormalised).
// Every thread of the block must call this (it contains barriers).
template <int DIR>
__device__ __forceinline__ void reg_fft(cf (&v)[16], int t, bool active, const RegPlan &p, cf *lds, int ls,
                                        const GFD_AS1 cf *__restrict__ tw) {
  int s = 1;
  for (int q = 0; q < p.npass; ++q) {
    const bool last = q == p.npass - 1;
    switch (p.radix[q]) {
      case 16: reg_pass<16, DIR>(v, t, p.T, s, p.L, last, active, lds, ls, tw); break;
      case 8: reg_pass<8, DIR>(v, t, p.T, s, p.L, last, active, lds, ls, tw); break;
      case 4: reg_pass<4, DIR>(v, t, p.T, s, p.L, last, active, lds, ls, tw); break;
      default: reg_pass<2, DIR>(v, t, p.T, s, p.L, last, active, lds, ls, tw); break;
    }
    s *= p.radix[q];
  }
}

// Compile-time form for one length L and LDS stride LS (the column passes interleave LS
// sequences).  Every pass's stride, butterfly count and LDS positions are constants: an
// exchange computes one LDS address per thread and reaches the other slots through immediate
// offsets (slot p sits at lds_pad(p) = p + p / 16, and both the write positions base + i s and
// the read positions t + T m advance by a multiple of 16, so their padded positions advance by
// a constant), and a butterfly's twiddle indices are multiples of one product.
template <int R, int DIR, int L, int S, int LS, bool LAST, bool GUARD, class TW>
__device__ __forceinline__ void reg_pass_c(cf (&v)[16], int t, bool active_, cf *lds, const TW &tw) {
  const bool active = !GUARD || active_;
  constexpr int T = L / 16, NBF = 16 / R, TSTRIDE = L / (S * R);
  static_assert(T % 16 == 0 && ((S == 1 && R == 16) || S % 16 == 0), "padded positions advance linearly");
  constexpr int WSTEP = S == 1 ? 1 : S + S / 16;  // lds_pad(base + (i + 1) S) - lds_pad(base + i S)
  constexpr int RSTEP = T + T / 16;               // lds_pad(t + T (m + 1)) - lds_pad(t + T m)
#pragma unroll
  for (int b = 0; b < NBF; ++b) {
    const int j = t + T * b;
    const int k = j & (S - 1);
    cf x[R];
#pragma unroll
    for (int i = 0; i < R; ++i) x[i] = v[b + i * NBF];
    if constexpr (S > 1) {
      if (active) {
#pragma unroll
        for (int i = 1; i < R; ++i) {
          cf w = tw.template at<S, TSTRIDE>(k, i);
          if (DIR > 0) w.im = -w.im;
          x[i] = cmul(x[i], w);
        }
      }
    }
    dftR<R, DIR>(x);
    if constexpr (LAST) {
#pragma unroll
      for (int i = 0; i < R; ++i) v[b + i * NBF] = x[i];
    } else if (active) {
      cf *w0 = lds + lds_pad((j - k) * R + k) * LS;
#pragma unroll
      for (int i = 0; i < R; ++i) w0[i * WSTEP * LS] = x[i];
    }
  }
  if constexpr (!LAST) {
    __syncthreads();
    if (active) {
      const cf *r0 = lds + lds_pad(t) * LS;
#pragma unroll
      for (int m = 0; m < 16; ++m) v[m] = r0[m * RSTEP * LS];
    }
    __syncthreads();
  }
}

// GUARD = false: every thread of the block holds a sequence (`active` is ignored), so the
// passes carry no per-thread branches.
template <int L, int DIR, int LS, bool GUARD = true, class TW>
__device__ __forceinline__ void reg_fft_c(cf (&v)[16], int t, bool active, cf *lds, const TW &tw) {
  static_assert(L >= 256 && L <= 4096 && (L & (L - 1)) == 0, "power of two in [256, 4096]");
  constexpr int rest = L / 256;
  if constexpr (rest == 1) {
    reg_pass_c<16, DIR, L, 1, LS, false, GUARD>(v, t, active, lds, tw);
    reg_pass_c<16, DIR, L, 16, LS, true, GUARD>(v, t, active, lds, tw);
  } else {
    reg_pass_c<16, DIR, L, 1, LS, false, GUARD>(v, t, active, lds, tw);
    reg_pass_c<16, DIR, L, 16, LS, false, GUARD>(v, t, active, lds, tw);
    reg_pass_c<rest, DIR, L, 256, LS, true, GUARD>(v, t, active, lds, tw);
  }
}

inline bool reg_plan_ok(int L) { return L >= 256 && L <= 4096 && (L & (L - 1)) == 0; }

// Tile width of the column passes for M = L (a power of two in [256, 4096]): the widest C with
// M x 2C complex values in 64 KiB, at most 16 (make_layout), which is also the LDS interleave of
// the compile-time column transforms.  Narrow images can have narrower tiles; they take the
// run-time transform.
__host__ __device__ constexpr int col_ls(int L) { return L >= 4096 ? 2 : L == 2048 ? 4 : L == 1024 ? 8 : 16; }

inline RegPlan make_reg_plan(int L) {
  RegPlan p;
  p.L = L;
  p.T = L / 16;
  int rest = L / 256;  // 1, 2, 4, 8, 16
  p.npass = rest == 1 ? 2 : 3;
  p.radix[0] = 16;
  p.radix[1] = 16;
  p.radix[2] = rest == 1 ? 1 : rest;
  return p;
}

}  // namespace gfd
