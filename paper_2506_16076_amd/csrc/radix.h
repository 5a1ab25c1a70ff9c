// In-register small DFTs for the mixed-radix line engine (gfx950, FP32).
//
// Dft<R, INV>::run(x): x_q <- sum_t x_t w^(+-t q), w = exp(-2 pi i / R); INV
// uses the conjugate root (no 1/R scaling).  Odd R: the generated symmetric
// butterflies of radix_gen.h; R = 2, 4, 8: the trivial roots.
#pragma once
#include <hip/hip_runtime.h>

#include "radix_gen.h"

namespace fcsd {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {  // a * conj(b)
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 rot(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

template <int R, bool INV>
struct Dft;

template <bool INV>
struct Dft<2, INV> {
  __device__ __forceinline__ static void run(float2* x) {
    float2 a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  }
};

template <bool INV>
struct Dft<4, INV> {
  __device__ __forceinline__ static void run(float2* x) {
    float2 s0 = cadd(x[0], x[2]), d0 = csub(x[0], x[2]);
    float2 s1 = cadd(x[1], x[3]), d1 = rot<INV>(csub(x[1], x[3]));
    x[0] = cadd(s0, s1);
    x[2] = csub(s0, s1);
    x[1] = cadd(d0, d1);
    x[3] = csub(d0, d1);
  }
};

template <bool INV>
struct Dft<8, INV> {
  __device__ __forceinline__ static void run(float2* x) {
    constexpr float h = 0.70710678118654752440f;
    float2 e[4] = {x[0], x[2], x[4], x[6]};
    float2 o[4] = {x[1], x[3], x[5], x[7]};
    Dft<4, INV>::run(e);
    Dft<4, INV>::run(o);
    // o_q *= w8^(+-q)
    float2 o1 = o[1], o3 = o[3];
    o[1] = INV ? make_float2(h * (o1.x - o1.y), h * (o1.x + o1.y)) : make_float2(h * (o1.x + o1.y), h * (o1.y - o1.x));
    o[2] = rot<INV>(o[2]);
    o[3] = INV ? make_float2(-h * (o3.x + o3.y), h * (o3.x - o3.y)) : make_float2(h * (o3.y - o3.x), -h * (o3.x + o3.y));
    for (int q = 0; q < 4; ++q) {
      x[q] = cadd(e[q], o[q]);
      x[q + 4] = csub(e[q], o[q]);
    }
  }
};

template <bool INV>
struct Dft<3, INV> {
  __device__ __forceinline__ static void run(float2* x) {
    if (INV)
      dft3_inv(x);
    else
      dft3_fwd(x);
  }
};

template <bool INV>
struct Dft<5, INV> {
  __device__ __forceinline__ static void run(float2* x) {
    if (INV)
      dft5_inv(x);
    else
      dft5_fwd(x);
  }
};

template <bool INV>
struct Dft<7, INV> {
  __device__ __forceinline__ static void run(float2* x) {
    if (INV)
      dft7_inv(x);
    else
      dft7_fwd(x);
  }
};

template <bool INV>
struct Dft<11, INV> {
  __device__ __forceinline__ static void run(float2* x) {
    if (INV)
      dft11_inv(x);
    else
      dft11_fwd(x);
  }
};

template <bool INV>
struct Dft<13, INV> {
  __device__ __forceinline__ static void run(float2* x) {
    if (INV)
      dft13_inv(x);
    else
      dft13_fwd(x);
  }
};

}  // namespace fcsd
