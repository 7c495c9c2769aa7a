// Device helpers shared by the gfx950 kernels: complex arithmetic, error-free sums,
// wave/block reductions and cheap integer division by run-time constants.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gfd {

// Pointers loaded from device memory (descriptor tables) are generic to the compiler, which
// then emits flat accesses with 64-bit VGPR addresses; G() marks them as global memory so
// that loads and stores take an SGPR base and their own wait counter.  The qualifier exists
// in the device pass only: the host pass parses kernel bodies but never generates them.
#if defined(__HIP_DEVICE_COMPILE__)
#define GFD_AS1 __attribute__((address_space(1)))
#else
#define GFD_AS1
#endif
template <class T> __device__ __forceinline__ GFD_AS1 T *G(T *p) { return (GFD_AS1 T *)p; }
template <class T> __device__ __forceinline__ const GFD_AS1 T *G(const T *p) { return (const GFD_AS1 T *)p; }

// Element i of a global array through a 32-bit unsigned byte offset (every array here is far
// below 4 GiB): the access then takes the SGPR base plus one VGPR offset instead of a 64-bit
// address computed per element.
template <class T> __device__ __forceinline__ const GFD_AS1 T &E(const GFD_AS1 T *p, uint32_t i) {
  return *reinterpret_cast<const GFD_AS1 T *>(reinterpret_cast<const GFD_AS1 char *>(p) + i * (uint32_t)sizeof(T));
}
template <class T> __device__ __forceinline__ GFD_AS1 T &E(GFD_AS1 T *p, uint32_t i) {
  return *reinterpret_cast<GFD_AS1 T *>(reinterpret_cast<GFD_AS1 char *>(p) + i * (uint32_t)sizeof(T));
}

// A global array addressed in bytes as base + soff + voff: soff is the same for the whole
// block (scalar arithmetic), voff a 32-bit per-thread offset, so the accesses of one thread at
// block-uniform distances share one address register and need no 64-bit arithmetic.
struct GBytes {
  GFD_AS1 char *p;
};
__device__ __forceinline__ GBytes gbytes(const void *base) { return GBytes{(GFD_AS1 char *)base}; }
__device__ __forceinline__ float ld_f(GBytes b, uint32_t voff, uint32_t soff) {
  return *reinterpret_cast<const GFD_AS1 float *>(b.p + soff + voff);
}
__device__ __forceinline__ void st_f(float v, GBytes b, uint32_t voff, uint32_t soff) {
  *reinterpret_cast<GFD_AS1 float *>(b.p + soff + voff) = v;
}
__device__ __forceinline__ void st_f4(float x, float y, float z, float w, GBytes b, uint32_t voff, uint32_t soff) {
  *reinterpret_cast<GFD_AS1 float4 *>(b.p + soff + voff) = make_float4(x, y, z, w);
}

template <class T>
struct alignas(2 * sizeof(T)) cpx {
  T re, im;
};
using cf = cpx<float>;
using cd = cpx<double>;

__device__ __forceinline__ cf ld_cf(GBytes b, uint32_t voff, uint32_t soff) {
  return *reinterpret_cast<const GFD_AS1 cf *>(b.p + soff + voff);
}
__device__ __forceinline__ void st_cf(cf v, GBytes b, uint32_t voff, uint32_t soff) {
  *reinterpret_cast<GFD_AS1 cf *>(b.p + soff + voff) = v;
}

template <class T> __device__ __forceinline__ cpx<T> mk(T a, T b) { return cpx<T>{a, b}; }
template <class T> __device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <class T> __device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <class T> __device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a * conj(b)
template <class T> __device__ __forceinline__ cpx<T> cmulc(cpx<T> a, cpx<T> b) {
  return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
template <class T> __device__ __forceinline__ cpx<T> cscale(cpx<T> a, T s) { return {a.re * s, a.im * s}; }
// multiply by -i (forward sign) or +i (inverse sign): DIR = -1 gives -i
template <int DIR, class T> __device__ __forceinline__ cpx<T> mul_i(cpx<T> a) {
  return DIR < 0 ? cpx<T>{a.im, -a.re} : cpx<T>{-a.im, a.re};
}
// |z|^2 with one fixed evaluation order (callers that must agree bit for bit use this)
__device__ __forceinline__ float abs2f(cf z) { return __fmaf_rn(z.re, z.re, __fmul_rn(z.im, z.im)); }

// ---------------------------------------------------------------- error-free transformations
// TwoSum (Knuth): s + e == a + b exactly.
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e) {
  s = __fadd_rn(a, b);
  float bb = __fsub_rn(s, a);
  e = __fadd_rn(__fsub_rn(a, __fsub_rn(s, bb)), __fsub_rn(b, bb));
}
// (hi, lo) += (bh, bl): compensated (double-float) accumulation.
__device__ __forceinline__ void df_add(float &hi, float &lo, float bh, float bl) {
  float s, e;
  two_sum(hi, bh, s, e);
  e = __fadd_rn(e, __fadd_rn(lo, bl));
  hi = __fadd_rn(s, e);
  lo = __fsub_rn(e, __fsub_rn(hi, s));
}

// ---------------------------------------------------------------- reductions
// Compensated sum of NV (hi, lo) pairs over the whole block.  The waves' results are combined
// by NV threads in parallel (thread v sums value v over the waves in wave order), then thread 0
// collects them: every thread below NV ends with its value in hi[v], lo[v] and thread 0 with all.
// `scratch` must hold 2 * NV * max(blockDim.x / 64, 1) floats.  Fixed order: deterministic.
// A block of fewer than 64 threads (a power of two) keeps its butterfly within its lanes.
template <int NV>
__device__ __forceinline__ void block_reduce_df(float (&hi)[NV], float (&lo)[NV], float *scratch) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    if (off >= (int)blockDim.x) continue;  // uniform
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      float oh = __shfl_down(hi[v], off, 64);
      float ol = __shfl_down(lo[v], off, 64);
      df_add(hi[v], lo[v], oh, ol);
    }
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      scratch[(wid * NV + v) * 2] = hi[v];
      scratch[(wid * NV + v) * 2 + 1] = lo[v];
    }
  }
  __syncthreads();
  const int t = threadIdx.x;
  float h = 0.0f, l = 0.0f;
  if (t < NV) {
    h = scratch[t * 2];
    l = scratch[t * 2 + 1];
    for (int w = 1; w < nw; ++w) df_add(h, l, scratch[(w * NV + t) * 2], scratch[(w * NV + t) * 2 + 1]);
  }
  __syncthreads();
  if (t < NV) {
    scratch[t * 2] = h;
    scratch[t * 2 + 1] = l;
  }
  __syncthreads();
  if (t == 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      hi[v] = scratch[v * 2];
      lo[v] = scratch[v * 2 + 1];
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------- integer division
// Quotient of x / d for 0 <= x < 2^22 and 1 <= d < 2^22 using a float reciprocal and one
// correction step (exact in that range).
struct FastDiv {
  int d;
  float inv;
};
__device__ __forceinline__ int fdiv(int x, FastDiv f) {
  int q = (int)((float)x * f.inv);
  int r = x - q * f.d;
  q += (r >= f.d) - (r < 0);
  return q;
}

// Remap a linear block index so that each of the 8 XCDs (which receive blocks round-robin)
// works on a contiguous range of logical tiles.
__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  const int nx = 8;
  int per = (nblocks + nx - 1) / nx;
  int xcd = bid % nx, local = bid / nx;
  int full = nblocks - (per - 1) * nx;  // XCDs that receive `per` blocks
  int start = xcd < full ? xcd * per : full * per + (xcd - full) * (per - 1);
  return start + local;
}

}  // namespace gfd
