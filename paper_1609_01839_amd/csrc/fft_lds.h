// Mixed-radix (2, 3, 4, 5, 8) Stockham autosort FFT on data resident in LDS.
//
// A workgroup transforms `nb` sequences of length L in place.  Element i of sequence b lives
// at buf[b * bs + i * es].  Each pass of radix r splits every sequence into L/r butterflies;
// butterfly j (with k = j mod s, s = product of the earlier radices) reads x[j + i*L/r],
// multiplies input i by W_{s r}^{i k}, applies the r-point DFT and writes output i to
// y[(j - k) r + k + i s].  After the last pass the data are in natural order.  Reads and
// writes of one pass are separated by a barrier, so one buffer serves as input and output.
//
// Twiddles come from a table tw[n] = exp(-2 pi i n / L) (computed in double precision on the
// host and rounded); DIR = -1 is the forward transform, DIR = +1 the unnormalised inverse.
#pragma once
#include "gfd_device.h"

namespace gfd {

constexpr int kMaxPasses = 12;

struct FftPlan {
  int L;
  int npass;
  int radix[kMaxPasses];
  int s[kMaxPasses];          // product of the radices of the earlier passes
  int nbf[kMaxPasses];        // L / radix
  int tstride[kMaxPasses];    // L / (s * radix): twiddle-table stride
  FastDiv sdiv[kMaxPasses];   // division by s
  FastDiv nbfdiv[kMaxPasses]; // division by L / radix
};

// ------------------------------------------------------------------ small DFTs
template <int DIR, class T> __device__ __forceinline__ void dft2(cpx<T> *v) {
  cpx<T> a = v[0], b = v[1];
  v[0] = a + b;
  v[1] = a - b;
}

template <int DIR, class T> __device__ __forceinline__ void dft4(cpx<T> *v) {
  cpx<T> t0 = v[0] + v[2], t1 = v[0] - v[2], t2 = v[1] + v[3], t3 = mul_i<DIR>(v[1] - v[3]);
  v[0] = t0 + t2;
  v[2] = t0 - t2;
  v[1] = t1 + t3;
  v[3] = t1 - t3;
}

template <int DIR, class T> __device__ __forceinline__ void dft8(cpx<T> *v) {
  const T c = (T)0.70710678118654752440;
  cpx<T> e[4] = {v[0], v[2], v[4], v[6]};
  cpx<T> o[4] = {v[1], v[3], v[5], v[7]};
  dft4<DIR>(e);
  dft4<DIR>(o);
  // o_k *= W8^k, W8 = exp(DIR * i pi / 4)
  cpx<T> o1 = {c * (o[1].re - DIR * o[1].im), c * (o[1].im + DIR * o[1].re)};
  cpx<T> o2 = mul_i<DIR>(o[2]);
  cpx<T> o3 = mul_i<DIR>(cpx<T>{c * (o[3].re - DIR * o[3].im), c * (o[3].im + DIR * o[3].re)});
  v[0] = e[0] + o[0];
  v[4] = e[0] - o[0];
  v[1] = e[1] + o1;
  v[5] = e[1] - o1;
  v[2] = e[2] + o2;
  v[6] = e[2] - o2;
  v[3] = e[3] + o3;
  v[7] = e[3] - o3;
}

template <int DIR, class T> __device__ __forceinline__ void dft3(cpx<T> *v) {
  const T h = (T)0.86602540378443864676;  // sin(2 pi / 3)
  cpx<T> t1 = v[1] + v[2], t2 = v[1] - v[2];
  cpx<T> m = v[0] - cscale(t1, (T)0.5);
  cpx<T> n = cscale(mul_i<DIR>(t2), h);
  v[0] = v[0] + t1;
  v[1] = m + n;
  v[2] = m - n;
}

template <int DIR, class T> __device__ __forceinline__ void dft5(cpx<T> *v) {
  const T c1 = (T)0.30901699437494742410, c2 = (T)-0.80901699437494742410;
  const T s1 = (T)0.95105651629515357212, s2 = (T)0.58778525229247312917;
  cpx<T> t1 = v[1] + v[4], t2 = v[2] + v[3], t3 = v[1] - v[4], t4 = v[2] - v[3];
  cpx<T> a0 = v[0];
  cpx<T> m1 = a0 + cscale(t1, c1) + cscale(t2, c2);
  cpx<T> m2 = a0 + cscale(t1, c2) + cscale(t2, c1);
  cpx<T> n1 = mul_i<DIR>(cscale(t3, s1) + cscale(t4, s2));
  cpx<T> n2 = mul_i<DIR>(cscale(t3, s2) - cscale(t4, s1));
  v[0] = a0 + t1 + t2;
  v[1] = m1 + n1;
  v[4] = m1 - n1;
  v[2] = m2 + n2;
  v[3] = m2 - n2;
}

template <int R, int DIR, class T> __device__ __forceinline__ void dft(cpx<T> *v) {
  if constexpr (R == 2) dft2<DIR>(v);
  else if constexpr (R == 3) dft3<DIR>(v);
  else if constexpr (R == 4) dft4<DIR>(v);
  else if constexpr (R == 5) dft5<DIR>(v);
  else dft8<DIR>(v);
}

// ------------------------------------------------------------------ one pass
// E bounds the number of elements a thread touches per pass: nb * L <= E * blockDim.x.
// COLMODE: sequences are interleaved (bs = 1, nb a power of two); consecutive threads take
// consecutive sequences.  Otherwise consecutive threads take consecutive butterflies.
template <class T, int R, int E, int DIR, bool COLMODE>
__device__ __forceinline__ void stockham_pass(cpx<T> *buf, int nb, int lognb, int es, int bs,
                                              const FftPlan &p, int q, const GFD_AS1 cpx<T> *__restrict__ tw) {
  constexpr int NBF = (E + R - 1) / R;
  const int nthr = blockDim.x, tid = threadIdx.x;
  const int nbf = p.nbf[q];
  const int total = nb * nbf;
  const int s = p.s[q];
  const int os = s * es;
  cpx<T> v[NBF][R];
  int dst[NBF];
#pragma unroll
  for (int u = 0; u < NBF; ++u) {
    const int idx = tid + u * nthr;
    dst[u] = -1;
    if (idx < total) {
      int b, j;
      if (COLMODE) {
        b = idx & (nb - 1);
        j = idx >> lognb;
      } else {
        b = fdiv(idx, p.nbfdiv[q]);
        j = idx - b * nbf;
      }
      const int base = b * bs;
#pragma unroll
      for (int i = 0; i < R; ++i) v[u][i] = buf[base + (j + i * nbf) * es];
      if (s > 1) {
        const int jq = fdiv(j, p.sdiv[q]);
        const int k = j - jq * s;
        const int ts = k * p.tstride[q];
#pragma unroll
        for (int i = 1; i < R; ++i) {
          cpx<T> w = tw[i * ts];
          if (DIR > 0) w.im = -w.im;
          v[u][i] = cmul(v[u][i], w);
        }
        dst[u] = base + (jq * s * R + k) * es;
      } else {
        dst[u] = base + j * R * es;
      }
      dft<R, DIR>(v[u]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < NBF; ++u) {
    if (dst[u] >= 0) {
#pragma unroll
      for (int i = 0; i < R; ++i) buf[dst[u] + i * os] = v[u][i];
    }
  }
  __syncthreads();
}

// Full transform; the caller has written the input to `buf` and synchronised.
template <class T, int E, int DIR, bool COLMODE>
__device__ __forceinline__ void lds_fft(cpx<T> *buf, int nb, int lognb, int es, int bs, const FftPlan &p,
                        const GFD_AS1 cpx<T> *__restrict__ tw) {
  for (int q = 0; q < p.npass; ++q) {
    switch (p.radix[q]) {
      case 2: stockham_pass<T, 2, E, DIR, COLMODE>(buf, nb, lognb, es, bs, p, q, tw); break;
      case 3: stockham_pass<T, 3, E, DIR, COLMODE>(buf, nb, lognb, es, bs, p, q, tw); break;
      case 4: stockham_pass<T, 4, E, DIR, COLMODE>(buf, nb, lognb, es, bs, p, q, tw); break;
      case 5: stockham_pass<T, 5, E, DIR, COLMODE>(buf, nb, lognb, es, bs, p, q, tw); break;
      default: stockham_pass<T, 8, E, DIR, COLMODE>(buf, nb, lognb, es, bs, p, q, tw); break;
    }
  }
}

}  // namespace gfd
