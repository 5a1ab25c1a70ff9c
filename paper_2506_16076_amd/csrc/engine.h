// FC line engine for gfx950: a tile of up to 64 complex lines of one patch
// (each complex line packs two real lines, re and im) held in LDS as
// z[pos * ld + c] (pos = sample index along the line, c = line in the tile,
// ld odd so that both the line-fastest FFT accesses and the pos-fastest
// row-tile loads are bank-conflict free).
//
// FC derivative of every line (paper Sec. 2.2, eqs. continuation and fc_der):
//   1. tail: z[N + m] = sum_j ArQ[m][j] z[N-d+j] + ArQ[C-1-m][d-1-j] z[j]
//      (FP64 accumulation: the matrix entries reach 1e4 while the tail is of
//      the size of the data);
//   2. forward FFT of length L = N + C: in-place mixed-radix decimation in
//      frequency, output in digit-reversed order;
//   3. multiplication by i k 2 pi / beta / L (table kmul, indexed by the
//      digit-reversed position, Nyquist zeroed);
//   4. inverse FFT: in-place decimation in time from digit-reversed input to
//      natural order.
// Positions 0..N-1 then hold the derivatives (re of line A, im of line B).
#pragma once
#include <hip/hip_runtime.h>

#include "radix.h"

namespace fcsd {

constexpr int kMaxStages = 8;
constexpr int kMaxTile = 64;     // complex lines per tile
constexpr int kBlock = 256;      // threads per workgroup

struct PlanDev {
  int N, L, C, nst;
  int rad[kMaxStages];
  int tw;        // offset of the twiddle table (float2) for this L
  int km;        // offset of the multiplier table (float) for this (N, L)
  int aq;        // offset of A_r Q^T (double) for this C, C*d entries
  int nlines;    // lines along this direction
  int n1, n2;    // patch shape
  int patch;     // patch index
  int periodic;  // C == 0
  long long off; // patch offset in a plane
};

struct TileDev {
  int plan;   // index into the plan array of the direction
  int line0;  // first line of the tile
  int nl;     // lines in the tile
  int ld;     // LDS stride in float2 (odd, >= nl)
};

// n = q*d + r for 0 <= n < 2^23 using a float reciprocal and one correction
struct FastDiv {
  int d;
  float r;
};
__device__ __forceinline__ FastDiv make_div(int d) { return FastDiv{d, 1.0f / (float)d}; }
__device__ __forceinline__ int divq(int n, FastDiv f, int& rem) {
  int q = (int)((float)n * f.r);
  int r = n - q * f.d;
  if (r < 0) {
    --q;
    r += f.d;
  } else if (r >= f.d) {
    ++q;
    r -= f.d;
  }
  rem = r;
  return q;
}

// One radix-R stage.  Forward (DIF): block of M points, m = M/R, butterfly j
// reads x_t = z[base + j + t m], y = DFT_R(x), y_q *= w_M^(j q), stores back.
// Inverse (DIT): the exact reverse with conjugate twiddles.
template <int R, bool INV>
__device__ __forceinline__ void fft_stage(float2* __restrict__ z, int ld, int nl, int L, int M,
                                          const float2* __restrict__ tw) {
  const int m = M / R;
  const int stride = L / M;
  const int items = (L / R) * nl;
  const FastDiv fnl = make_div(nl), fm = make_div(m);
  for (int it = threadIdx.x; it < items; it += blockDim.x) {
    int c;
    const int b = divq(it, fnl, c);
    int j;
    const int blk = divq(b, fm, j);
    const int base = blk * M + j;
    float2 x[R];
#pragma unroll
    for (int t = 0; t < R; ++t) x[t] = z[(base + t * m) * ld + c];
    if (!INV) {
      Dft<R, false>::run(x);
      if (j) {
#pragma unroll
        for (int q = 1; q < R; ++q) x[q] = cmul(x[q], tw[stride * j * q]);
      }
    } else {
      if (j) {
#pragma unroll
        for (int q = 1; q < R; ++q) x[q] = cmulc(x[q], tw[stride * j * q]);
      }
      Dft<R, true>::run(x);
    }
#pragma unroll
    for (int t = 0; t < R; ++t) z[(base + t * m) * ld + c] = x[t];
  }
}

template <bool INV>
__device__ __forceinline__ void fft_dispatch(int R, float2* z, int ld, int nl, int L, int M,
                                             const float2* tw) {
  switch (R) {
    case 2: fft_stage<2, INV>(z, ld, nl, L, M, tw); break;
    case 3: fft_stage<3, INV>(z, ld, nl, L, M, tw); break;
    case 4: fft_stage<4, INV>(z, ld, nl, L, M, tw); break;
    case 5: fft_stage<5, INV>(z, ld, nl, L, M, tw); break;
    case 7: fft_stage<7, INV>(z, ld, nl, L, M, tw); break;
    case 8: fft_stage<8, INV>(z, ld, nl, L, M, tw); break;
    case 11: fft_stage<11, INV>(z, ld, nl, L, M, tw); break;
    case 13: fft_stage<13, INV>(z, ld, nl, L, M, tw); break;
    default: break;
  }
}

// Tail of every line (continuation); periodic plans have no tail.
__device__ __forceinline__ void fc_tail(float2* __restrict__ z, int ld, int nl, const PlanDev& P,
                                        const double* __restrict__ aq, int d) {
  const int N = P.N, C = P.C;
  const int items = C * nl;
  const FastDiv fnl = make_div(nl);
  for (int it = threadIdx.x; it < items; it += blockDim.x) {
    int c;
    const int m = divq(it, fnl, c);
    double sx = 0.0, sy = 0.0;
    const double* ar = aq + m * d;                 // right blend row m
    const double* al = aq + (C - 1 - m) * d;       // mirrored row for the left blend
    for (int j = 0; j < d; ++j) {
      const float2 fr = z[(N - d + j) * ld + c];
      const float2 fl = z[j * ld + c];
      const double a = ar[j], b = al[d - 1 - j];
      sx = fma(a, (double)fr.x, sx);
      sy = fma(a, (double)fr.y, sy);
      sx = fma(b, (double)fl.x, sx);
      sy = fma(b, (double)fl.y, sy);
    }
    z[(N + m) * ld + c] = make_float2((float)sx, (float)sy);
  }
}

// z <- i * kmul[pos] * z (sign -1 for the transpose)
__device__ __forceinline__ void spectral_mul(float2* __restrict__ z, int ld, int nl, int L,
                                             const float* __restrict__ km, float sign) {
  const int items = L * nl;
  const FastDiv fnl = make_div(nl);
  for (int it = threadIdx.x; it < items; it += blockDim.x) {
    int c;
    const int p = divq(it, fnl, c);
    const float k = sign * km[p];
    const float2 v = z[p * ld + c];
    z[p * ld + c] = make_float2(-k * v.y, k * v.x);
  }
}

// E^T of the continuation: add sum_m (A Q^T)[m][j] tail[m] to the 2d end
// samples (reads positions N.., writes positions < N; distinct for N >= 2d).
__device__ __forceinline__ void fold_tail(float2* __restrict__ z, int ld, int nl, const PlanDev& P,
                                          const double* __restrict__ aq, int d) {
  const int items = 2 * d * nl;
  const int N = P.N, C = P.C;
  for (int it = threadIdx.x; it < items; it += blockDim.x) {
    const int e = it / nl, c = it - e * nl;
    double sx = 0.0, sy = 0.0;
    int pos;
    if (e < d) {  // right end sample j = e at N-d+e: sum_m ArQ[m][j] tail[m]
      pos = N - d + e;
      for (int m = 0; m < C; ++m) {
        const float2 t = z[(N + m) * ld + c];
        sx = fma(aq[m * d + e], (double)t.x, sx);
        sy = fma(aq[m * d + e], (double)t.y, sy);
      }
    } else {  // left end sample j = e-d: sum_m ArQ[C-1-m][d-1-j] tail[m]
      const int j = e - d;
      pos = j;
      for (int m = 0; m < C; ++m) {
        const float2 t = z[(N + m) * ld + c];
        const double a = aq[(C - 1 - m) * d + (d - 1 - j)];
        sx = fma(a, (double)t.x, sx);
        sy = fma(a, (double)t.y, sy);
      }
    }
    const float2 v = z[pos * ld + c];
    z[pos * ld + c] = make_float2(v.x + (float)sx, v.y + (float)sy);
  }
}

// Derivative of the tile in place (steps 2-4); the caller has filled
// positions 0..N-1 and synchronised.  adj = transpose (zero tail, -i k).
template <bool ADJ>
__device__ void line_derivative(float2* __restrict__ z, int ld, int nl, const PlanDev* __restrict__ Pg,
                                const PlanDev& P,
                                const float2* __restrict__ twp, const float* __restrict__ kmp,
                                const double* __restrict__ aqp, int d) {
  const float2* tw = twp + P.tw;
  if (!P.periodic) {
    if (!ADJ) {
      fc_tail(z, ld, nl, P, aqp + P.aq, d);
    } else {
      const int items = P.C * nl;
      for (int it = threadIdx.x; it < items; it += blockDim.x) {
        const int m = it / nl, c = it - m * nl;
        z[(P.N + m) * ld + c] = make_float2(0.f, 0.f);
      }
    }
    __syncthreads();
  }
  // radices are read from the (uniform) plan in global memory: a private
  // array indexed by the stage counter would live in scratch
  const int* rad = Pg->rad;
  const int nst = P.nst;
  int M = P.L;
  for (int s = 0; s < nst; ++s) {
    const int R = rad[s];
    fft_dispatch<false>(R, z, ld, nl, P.L, M, tw);
    M /= R;
    __syncthreads();
  }
  spectral_mul(z, ld, nl, P.L, kmp + P.km, ADJ ? -1.f : 1.f);
  __syncthreads();
  M = 1;
  for (int s = nst - 1; s >= 0; --s) {
    const int R = rad[s];
    M *= R;
    fft_dispatch<true>(R, z, ld, nl, P.L, M, tw);
    __syncthreads();
  }
  if (ADJ && !P.periodic) {
    fold_tail(z, ld, nl, P, aqp + P.aq, d);
    __syncthreads();
  }
}

}  // namespace fcsd
