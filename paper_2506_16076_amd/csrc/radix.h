// In-register small DFTs for the mixed-radix line engine (gfx950, FP32).
//
// Dft<R, INV>::run(x): x_q <- sum_t x_t w^(+-t q), w = exp(-2 pi i / R); INV
// uses the conjugate root (no 1/R scaling).  Odd primes: the generated
// symmetric butterflies of radix_gen.h; R = 2, 4, 8: the trivial roots;
// composite R = R1 R2 (one LDS round trip instead of two): the prime-factor
// split for coprime R1, R2 and the Cooley-Tukey split otherwise, both with
// natural order in and out.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "radix_gen.h"

namespace fcsd {

__host__ __device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ __forceinline__ float2 cmulc(float2 a, float2 b) {  // a * conj(b)
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__host__ __device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__host__ __device__ __forceinline__ float2 rot(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

template <int R, bool INV>
struct Dft;

template <bool INV>
struct Dft<2, INV> {
  __host__ __device__ __forceinline__ static void run(float2* x) {
    float2 a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  }
};

template <bool INV>
struct Dft<4, INV> {
  __host__ __device__ __forceinline__ static void run(float2* x) {
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
  __host__ __device__ __forceinline__ static void run(float2* x) {
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
  __host__ __device__ __forceinline__ static void run(float2* x) {
    if (INV)
      dft3_inv(x);
    else
      dft3_fwd(x);
  }
};

template <bool INV>
struct Dft<5, INV> {
  __host__ __device__ __forceinline__ static void run(float2* x) {
    if (INV)
      dft5_inv(x);
    else
      dft5_fwd(x);
  }
};

template <bool INV>
struct Dft<7, INV> {
  __host__ __device__ __forceinline__ static void run(float2* x) {
    if (INV)
      dft7_inv(x);
    else
      dft7_fwd(x);
  }
};

template <bool INV>
struct Dft<11, INV> {
  __host__ __device__ __forceinline__ static void run(float2* x) {
    if (INV)
      dft11_inv(x);
    else
      dft11_fwd(x);
  }
};

template <bool INV>
struct Dft<13, INV> {
  __host__ __device__ __forceinline__ static void run(float2* x) {
    if (INV)
      dft13_inv(x);
    else
      dft13_fwd(x);
  }
};

// R = R1 R2 with gcd(R1, R2) = 1 (Good-Thomas): with n = (R2 n1 + R1 n2)
// mod R and k = k1 (mod R1), k = k2 (mod R2), w_R^(n k) = w_R1^(n1 k1)
// w_R2^(n2 k2), so the transform is R2 transforms of length R1 followed by
// R1 of length R2, with no twiddles; the index maps are fixed at compile
// time and cost no instructions.
constexpr int inv_mod(int a, int m) {
  int x = 1;
  while ((a * x) % m != 1) ++x;
  return x;
}

template <int R1, int R2, bool INV>
struct DftPfa {
  __host__ __device__ __forceinline__ static void run(float2* x) {
    constexpr int R = R1 * R2;
    constexpr int E1 = R2 * inv_mod(R2 % R1, R1);  // = 1 mod R1, 0 mod R2
    constexpr int E2 = R1 * inv_mod(R1 % R2, R2);  // = 0 mod R1, 1 mod R2
    float2 y[R1][R2];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
      float2 t[R1];
#pragma unroll
      for (int n1 = 0; n1 < R1; ++n1) t[n1] = x[(R2 * n1 + R1 * n2) % R];
      Dft<R1, INV>::run(t);
#pragma unroll
      for (int k1 = 0; k1 < R1; ++k1) y[k1][n2] = t[k1];
    }
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
      Dft<R2, INV>::run(y[k1]);
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) x[(k1 * E1 + k2 * E2) % R] = y[k1][k2];
    }
  }
};

// Root w_R^(+-e) from the generated tables; quarter turns are exact.
#define FCSD_CT_TWIDDLE(RR)                                                                  \
  template <int R, int E, bool INV>                                                          \
  __host__ __device__ __forceinline__ typename std::enable_if<R == RR, float2>::type ct_tw(float2 v) { \
    constexpr int e = E % RR;                                                                \
    if constexpr (e == 0) {                                                                  \
      return v;                                                                              \
    } else if constexpr (4 * e == RR) {                                                      \
      return rot<INV>(v);                                                                    \
    } else if constexpr (2 * e == RR) {                                                      \
      return make_float2(-v.x, -v.y);                                                        \
    } else if constexpr (4 * e == 3 * RR) {                                                  \
      return rot<!INV>(v);                                                                   \
    } else {                                                                                 \
      constexpr float c = kRootCos##RR[e], sn = INV ? kRootSin##RR[e] : -kRootSin##RR[e];    \
      return make_float2(v.x * c - v.y * sn, v.x * sn + v.y * c);                            \
    }                                                                                        \
  }
FCSD_CT_TWIDDLE(9)
FCSD_CT_TWIDDLE(16)
#undef FCSD_CT_TWIDDLE

// R = R1 R2 (Cooley-Tukey): X[k1 + R1 k2] = sum_n2 w_R2^(n2 k2) w_R^(n2 k1)
// sum_n1 x[R2 n1 + n2] w_R1^(n1 k1).
template <int R1, int R2, bool INV>
struct DftCt {
  template <int N2, int K1>
  __host__ __device__ __forceinline__ static void twiddle(float2 (&y)[R2][R1]) {
    if constexpr (K1 < R1) {
      y[N2][K1] = ct_tw<R1 * R2, N2 * K1, INV>(y[N2][K1]);
      twiddle<N2, K1 + 1>(y);
    } else if constexpr (N2 + 1 < R2) {
      twiddle<N2 + 1, 0>(y);
    }
  }
  __host__ __device__ __forceinline__ static void run(float2* x) {
    float2 y[R2][R1];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
#pragma unroll
      for (int n1 = 0; n1 < R1; ++n1) y[n2][n1] = x[R2 * n1 + n2];
      Dft<R1, INV>::run(y[n2]);
    }
    twiddle<0, 0>(y);
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
      float2 u[R2];
#pragma unroll
      for (int n2 = 0; n2 < R2; ++n2) u[n2] = y[n2][k1];
      Dft<R2, INV>::run(u);
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) x[k1 + R1 * k2] = u[k2];
    }
  }
};

#define FCSD_DFT_PFA(R, R1, R2)                                              \
  template <bool INV>                                                        \
  struct Dft<R, INV> {                                                       \
    __host__ __device__ __forceinline__ static void run(float2* x) { DftPfa<R1, R2, INV>::run(x); } \
  };
#define FCSD_DFT_CT(R, R1, R2)                                               \
  template <bool INV>                                                        \
  struct Dft<R, INV> {                                                       \
    __host__ __device__ __forceinline__ static void run(float2* x) { DftCt<R1, R2, INV>::run(x); } \
  };
FCSD_DFT_PFA(6, 2, 3)
FCSD_DFT_PFA(10, 2, 5)
FCSD_DFT_PFA(12, 4, 3)
FCSD_DFT_PFA(14, 2, 7)
FCSD_DFT_PFA(15, 3, 5)
FCSD_DFT_CT(9, 3, 3)
FCSD_DFT_CT(16, 4, 4)
#undef FCSD_DFT_PFA
#undef FCSD_DFT_CT

}  // namespace fcsd
