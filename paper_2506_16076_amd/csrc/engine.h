// FC line engine for gfx950: a tile of up to 64 complex lines of one patch
// (each complex line packs two real lines, re and im) held in LDS as
// z[pos * ld + c] (pos = sample index along the line, c = line in the tile,
// ld odd so that both the line-fastest FFT accesses and the pos-fastest
// row-tile loads are bank-conflict free).
//
// FC derivative of every line (paper Sec. 2.2, eqs. continuation and fc_der).
// The extension ext = [f; A_l Q^T f_l + A_r Q^T f_r] of length L = N + C is
// periodic; its derivative is the circulant operator F^-1 diag(i w_k) F.
// Because every circulant commutes with the cyclic first difference
// (Delta x)[n] = x[n+1] - x[n], whose symbol is exp(2 pi i k / L) - 1, the
// engine transforms Delta ext and multiplies by i w_k / (exp(2 pi i k/L) - 1)
// instead: the same operator in exact arithmetic, but FP32 rounding in the
// forward FFT now scales with |Delta ext| ~ h |f'| instead of |f|, and the
// multiplier is bounded by pi / (2 h) at every k instead of growing to
// pi / h, so the derivative keeps a relative accuracy of a few ulp.
//   1. differences: Delta ext[n] for n < N-1 in FP32 (exact for close
//      neighbours), the C + 1 differences that involve the tail in FP64 from
//      the differenced continuation rows (matrix entries reach 1e4 while the
//      tail is of the size of the data);
//   2. forward FFT of length L: in-place mixed-radix decimation in
//      frequency, output in digit-reversed order;
//   3. complex multiplier (table kmul, indexed by the digit-reversed
//      position; k = 0 and the Nyquist zeroed);
//   4. inverse FFT: in-place decimation in time from digit-reversed input to
//      natural order.
// Positions 0..N-1 then hold the derivatives (re of line A, im of line B).
// The transpose applies Delta^T to the zero-padded cotangent, the conjugate
// multipliers and the transposed continuation (fold of the tail).
#pragma once
#include <hip/hip_runtime.h>

#include "radix.h"

namespace fcsd {

constexpr int kMaxStages = 8;
constexpr int kMaxTile = 64;     // complex lines per tile
constexpr int kBlock = 256;      // threads per workgroup

struct PlanDev {
  int N, L, C, nst;  // L: transform length (N + C, or the embedding length of a circulant of N + C)
  int Lx;            // extension length N + C
  int rad[kMaxStages];
  int tw;        // offset of the twiddle table (float2) for this L
  int km;        // offset of the multiplier table (float2) for this (N, L)
  int aq;        // offset of A_r Q^T (double) for this C, C*d entries
  int dq;        // offset of the differenced rows (double), (C+1)*2d entries
  int kf;        // offset of the spectral filter factors (float2) for this L
  int gq;        // offset of the derivative's fold matrix (float), N*2d entries, for this (N, C)
  int gf;        // offset of the filter's fold matrix (float), N*2d entries (filter configured)
  int wallp;     // the patch has a wall side (energy derivatives by the product rule)
  int nlines;    // lines along this direction
  int n1, n2;    // patch shape
  int patch;     // patch index
  int periodic;  // C == 0
  int nb1;       // 0: row-major patch storage; else 8x4 blocks, nb1 per block row
  long long off; // patch offset in a plane
};

struct TileDev {
  int plan;   // index into the plan array of the direction
  int line0;  // first line of the tile
  int nl;     // lines in the tile
  int ld;     // LDS stride in float2 (odd, >= nl)
};

// Per-thread view of a tile in LDS.  Layout of the dynamic LDS block:
//   z   [L * ld] float2   the lines, z[pos * ld + c]
//   tw  [L]      float2   exp(-2 pi i n / L)
//   km  [L]      float2   derivative multipliers by digit-reversed position
//   side[2d * ld] float2  end samples of every line (differencing loads)
// Thread t works on line c = t % nl and on butterflies t / nl, t / nl + BS,
// ... of every stage (BS = blockDim / nl), so consecutive lanes touch
// consecutive lines (conflict-free LDS rows) and share their twiddle
// (broadcast).  Threads t >= BS * nl only take part in the element loops.
struct LineCtx {
  float2* z;
  const float2* tw;
  const float2* km;
  float2* side;  // [2 kMaxD][ld]: the 2d end samples of every line (loads that difference)
  int ld, nl, c, b0, BS;
  bool active;
};

constexpr int kMaxD = 8;

__device__ __forceinline__ size_t tile_lds_bytes(int L, int ld, int d) {
  return (size_t)L * ld * sizeof(float2) + (size_t)L * 2 * sizeof(float2) + (size_t)2 * d * ld * sizeof(float2);
}

// Copy the plan's twiddles and multipliers (table kmg at offset kmo; the
// derivative multipliers by default) into LDS; the caller syncs.
__device__ __forceinline__ LineCtx line_setup(float2* lds, const TileDev& T, const PlanDev& P,
                                              const float2* __restrict__ twg, const float2* __restrict__ kmg,
                                              int kmo = -1) {
  LineCtx X;
  X.z = lds;
  float2* tw = lds + (size_t)P.L * T.ld;
  float2* km = tw + P.L;
  if (kmo < 0) kmo = P.km;
  for (int i = threadIdx.x; i < P.L; i += blockDim.x) {
    tw[i] = twg[P.tw + i];
    km[i] = kmg[kmo + i];
  }
  X.tw = tw;
  X.km = km;
  X.side = km + P.L;
  X.ld = T.ld;
  X.nl = T.nl;
  X.BS = blockDim.x / T.nl;
  X.c = threadIdx.x % T.nl;
  X.b0 = threadIdx.x / T.nl;
  X.active = X.b0 < X.BS;
  return X;
}

// The same tile viewed as nlc complex lines (a multiple of the lines the
// context was set up for, within its row stride): thread mapping only, the
// tables stay where line_setup put them.
__device__ __forceinline__ LineCtx line_view(const LineCtx& X0, int nlc) {
  LineCtx X = X0;
  X.nl = nlc;
  X.BS = blockDim.x / nlc;
  X.c = threadIdx.x % nlc;
  X.b0 = threadIdx.x / nlc;
  X.active = X.b0 < X.BS;
  return X;
}

// Walk over the elements (pos, c) of a tile in global-memory storage order.
// Thread t visits elements t, t + blockDim, ... of the tile's storage and
// carries, per element, two byte offsets updated by uniform increments:
//   g: from the tile's first stored element, the same in every plane (the
//      caller adds it to a per-plane tile base pointer, which stays uniform:
//      loads and stores take a scalar base and one vector offset);
//   l: of z[pos * ld + c] in LDS.
// Storage of a patch (element (i, j), i along q1, off = patch offset):
//   row-major:  off + j n1 + i
//   8x4 blocks: off + 32 ((j/4) nb1 + i/8) + 8 (j%4) + i%8, nb1 = ceil(n1/8);
//               tiles start on block boundaries (q1 tiles: line0 % 4 = 0,
//               q2 tiles: line0 % 8 = 0), so a thread keeps its place w in a
//               block (blockDim % 32 = 0) and steps whole blocks.
// The walk splits the tile into blocks of W elements (W = 32 blocked, 1
// row-major) arranged slow x fast; (fast, slow) advance by (dF, dS) blocks
// per step with one carry.  Padding elements of the blocked storage (pos >=
// N or c >= nl) lie inside the patch's storage and are skipped by valid().
struct Walk {
  unsigned g, l;            // byte offsets of the current element
  int fast, slow;           // block coordinates
  int flim, slim;           // valid while fast < flim and slow < slim
  int nbf, nslow, dF, dS;   // uniform: blocks along fast, slow extent, step
  unsigned dG, dL, wG, wL;  // uniform: offset steps, extra on carry
  unsigned gnext;           // byte distance to the next sample along the line

  __host__ __device__ __forceinline__ bool more() const { return slow < nslow; }
  __host__ __device__ __forceinline__ bool valid() const { return fast < flim && slow < slim; }
  __host__ __device__ __forceinline__ void next() {
    fast += dF;
    slow += dS;
    g += dG;
    l += dL;
    if (fast >= nbf) {
      fast -= nbf;
      ++slow;
      g += wG;
      l += wL;
    }
  }
};

// Walk of thread t of bd (a multiple of 32) over a tile of nl lines of N
// samples along direction DIR (1: lines are rows i = pos, j = line0 + c;
// 2: columns i = line0 + c, j = pos); nb1 = 0 for row-major storage with
// row length n1.
template <int DIR>
__host__ __device__ __forceinline__ Walk make_walk_t(int t, int bd, int N, int nl, int ld, int nb1, int n1) {
  Walk w;
  int gf, gs, lf, ls, b0, wq = 0, gw, lw;  // element steps along fast/slow, first block, place in block
  if (nb1) {
    wq = t & 31;
    b0 = t >> 5;
    bd >>= 5;
    gf = 32;
    gs = 32 * nb1;
    gw = wq;
    if (DIR == 1) {  // fast: blocks of 8 samples, slow: strips of 4 lines
      w.nbf = (N + 7) >> 3;
      w.nslow = (nl + 3) >> 2;
      w.flim = (N - (wq & 7) + 7) >> 3;
      w.slim = (nl - (wq >> 3) + 3) >> 2;
      lf = 8 * ld;
      ls = 4;
      lw = (wq & 7) * ld + (wq >> 3);
      w.gnext = 4u * ((wq & 7) < 7 ? 1u : 25u);
    } else {         // fast: blocks of 8 lines, slow: groups of 4 samples
      w.nbf = (nl + 7) >> 3;
      w.nslow = (N + 3) >> 2;
      w.flim = (nl - (wq & 7) + 7) >> 3;
      w.slim = (N - (wq >> 3) + 3) >> 2;
      lf = 8;
      ls = 4 * ld;
      lw = (wq >> 3) * ld + (wq & 7);
      w.gnext = 4u * ((wq >> 3) < 3 ? 8u : (unsigned)(32 * nb1 - 24));
    }
  } else {
    b0 = t;
    gf = 1;
    gs = n1;
    gw = 0;
    lw = 0;
    if (DIR == 1) {  // fast: samples, slow: lines
      w.nbf = N;
      w.nslow = nl;
      lf = ld;
      ls = 1;
      w.gnext = 4u;
    } else {         // fast: lines, slow: samples
      w.nbf = nl;
      w.nslow = N;
      lf = 1;
      ls = ld;
      w.gnext = 4u * (unsigned)n1;
    }
    w.flim = w.nbf;
    w.slim = w.nslow;
  }
  w.fast = b0 % w.nbf;
  w.slow = b0 / w.nbf;
  w.dF = bd % w.nbf;
  w.dS = bd / w.nbf;
  w.g = 4u * (unsigned)(w.slow * gs + w.fast * gf + gw);
  w.l = 8u * (unsigned)(w.fast * lf + w.slow * ls + lw);
  w.dG = 4u * (unsigned)(w.dS * gs + w.dF * gf);
  w.dL = 8u * (unsigned)(w.dF * lf + w.dS * ls);
  w.wG = 4u * (unsigned)(gs - w.nbf * gf);
  w.wL = 8u * (unsigned)(ls - w.nbf * lf);
  return w;
}

template <int DIR>
__device__ __forceinline__ Walk make_walk(int N, int nl, int ld, int nb1, int n1) {
  return make_walk_t<DIR>(threadIdx.x, blockDim.x, N, nl, ld, nb1, n1);
}

// Element offset of the tile's first stored element from the patch offset.
template <int DIR>
__host__ __device__ __forceinline__ long long tile_first(int line0, int nb1, int n1) {
  if (nb1) return DIR == 1 ? 32LL * nb1 * (line0 >> 2) : 32LL * (line0 >> 3);
  return DIR == 1 ? (long long)line0 * n1 : (long long)line0;
}

// Elements of a patch's storage.
__host__ __device__ __forceinline__ long long patch_storage(int n1, int n2, int nb1) {
  return nb1 ? 32LL * nb1 * ((n2 + 3) >> 2) : (long long)n1 * n2;
}

// Byte offset of element (pos, c) from the tile's first stored element.
template <int DIR>
__host__ __device__ __forceinline__ unsigned tile_goff(int pos, int c, int nb1, int n1) {
  const int i = DIR == 1 ? pos : c, j = DIR == 1 ? c : pos;
  if (nb1) return 4u * (unsigned)(32 * ((j >> 2) * nb1 + (i >> 3)) + 8 * (j & 3) + (i & 7));
  return 4u * (unsigned)(j * n1 + i);
}

template <class T>
__device__ __forceinline__ T& at(T* base, unsigned byte_off) {
  return *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + byte_off);
}
template <class T>
__device__ __forceinline__ const T& at(const T* base, unsigned byte_off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off);
}

// Loads and stores of an LDS element at a byte offset from a pointer into
// LDS, addressed in the LDS address space: 32-bit offset arithmetic and
// ds_read / ds_write (a generic pointer's low 32 bits are its LDS offset;
// through the generic pointer the compiler forms 64-bit addresses, with a
// 64-bit multiply-add per twiddle).
__device__ __forceinline__ float2 ld_lds(const float2* base, unsigned byte_off) {
  typedef __attribute__((address_space(3))) const unsigned long long lU;
  const unsigned long long v = *(lU*)(size_t)((unsigned)(size_t)base + byte_off);
  float2 r;
  __builtin_memcpy(&r, &v, sizeof(r));
  return r;
}
__device__ __forceinline__ void st_lds(float2* base, unsigned byte_off, float2 x) {
  typedef __attribute__((address_space(3))) unsigned long long lU;
  unsigned long long v;
  __builtin_memcpy(&v, &x, sizeof(v));
  *(lU*)(size_t)((unsigned)(size_t)base + byte_off) = v;
}

// Visit the valid elements of a walk: f(g, l).
template <class F>
__device__ __forceinline__ void walk(Walk w, F&& f) {
  for (; w.more(); w.next())
    if (w.valid()) f(w.g, w.l);
}

// Batched walk for memory-latency-bound phases: pre(g) issues the loads of
// U elements of the thread, then post(g, l, value) consumes them.  pre runs
// unconditionally (elements that are not valid read the tile's first
// element and are dropped), so the loads are straight-line code and all U
// are in flight together; pre should only load, and leave arithmetic to post.
template <int U, class Pre, class Post>
__device__ __forceinline__ void walk_b(Walk w, Pre&& pre, Post&& post) {
  using T = decltype(pre(0u));
  while (w.more()) {
    T v[U];
    unsigned gs[U], ls[U];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ok[u] = w.valid();
      gs[u] = ok[u] ? w.g : 0u;
      ls[u] = w.l;
      v[u] = pre(gs[u]);
      w.next();
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (ok[u]) post(gs[u], ls[u], v[u]);
  }
}

// Largest radix whose stage reads all its twiddles before the butterfly
// (larger ones would need more registers than the line kernels have).
constexpr int kTwPre = 12;

// One radix-R stage.  Forward (DIF): block of M points, m = M/R, butterfly j
// reads x_t = z[base + j + t m], y = DFT_R(x), y_q *= w_M^(j q), stores back.
// Inverse (DIT): the exact reverse with conjugate twiddles.  MUL (last
// forward stage, M = R, m = 1, no twiddles): multiply the outputs by
// km[pos] (CONJ: by its conjugate, the transposed operator) and apply the
// first inverse stage, which works on the same R contiguous samples without
// twiddles, before storing: one LDS round trip and one barrier fewer.
template <int R, bool INV, bool MUL, bool CONJ>
__device__ __forceinline__ void fft_stage(const LineCtx& X, int L, int M) {
  if (!X.active) return;
  const int m = M / R;
  const int stride = L / M;
  const int nb = L / R;
  const int ld = X.ld;
  // butterfly b of the thread: block blk = b / m, index j = b % m; every
  // offset below is in bytes and advances by a uniform step per iteration,
  // with one correction when j passes m
  const int dblk = X.BS / m, dj = X.BS - dblk * m;
  const unsigned leg = 8u * (unsigned)(m * ld);                     // between the R legs
  const unsigned da = 8u * (unsigned)((dblk * M + dj) * ld);        // leg 0, per iteration
  const unsigned wa = 8u * (unsigned)((M - m) * ld);                // leg 0, when j wraps
  const unsigned dtw = 8u * (unsigned)(stride * dj), wtw = 8u * (unsigned)(stride * m);
  const unsigned dk = 8u * (unsigned)(X.BS * R);
  int b = X.b0;
  const int blk = b / m;
  int j = b - blk * m;
  unsigned a = 8u * (unsigned)((blk * M + j) * ld + X.c);
  unsigned tq = 8u * (unsigned)(stride * j);  // twiddle w^(j) of leg 1; leg q reads q tq
  unsigned kq = 8u * (unsigned)(b * R);       // MUL (m = 1): multipliers of positions b R ..
  for (; b < nb; b += X.BS) {
    float2 x[R];
#pragma unroll
    for (int t = 0; t < R; ++t) x[t] = ld_lds(X.z, a + t * leg);
    // j = 0 reads twiddle 1 + 0i: the product is exact, so no branch
    if (!INV) {
      // up to radix kTwPre the twiddles (multipliers) are read before the
      // butterfly, so that their LDS latency overlaps it
      constexpr bool kPre = R <= kTwPre;
      float2 w[R];
      if (kPre) {
#pragma unroll
        for (int q = MUL ? 0 : 1; q < R; ++q) w[q] = MUL ? ld_lds(X.km, kq + 8u * q) : ld_lds(X.tw, q * tq);
      }
      Dft<R, false>::run(x);
      if (MUL) {
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const float2 k = kPre ? w[q] : ld_lds(X.km, kq + 8u * q);
          x[q] = CONJ ? cmulc(x[q], k) : cmul(x[q], k);
        }
        Dft<R, true>::run(x);
      } else {
#pragma unroll
        for (int q = 1; q < R; ++q) x[q] = cmul(x[q], kPre ? w[q] : ld_lds(X.tw, q * tq));
      }
    } else {
      if (R <= kTwPre) {
        // every twiddle read before the first product
        float2 w[R];
#pragma unroll
        for (int q = 1; q < R; ++q) w[q] = ld_lds(X.tw, q * tq);
#pragma unroll
        for (int q = 1; q < R; ++q) x[q] = cmulc(x[q], w[q]);
      } else {
#pragma unroll
        for (int q = 1; q < R; ++q) x[q] = cmulc(x[q], ld_lds(X.tw, q * tq));
      }
      Dft<R, true>::run(x);
    }
#pragma unroll
    for (int t = 0; t < R; ++t) st_lds(X.z, a + t * leg, x[t]);
    a += da;
    tq += dtw;
    kq += dk;
    j += dj;
    if (j >= m) {
      j -= m;
      a += wa;
      tq -= wtw;
    }
  }
}

template <bool INV, bool MUL, bool CONJ>
__device__ __forceinline__ void fft_dispatch(int R, const LineCtx& X, int L, int M) {
  switch (R) {
    case 2: fft_stage<2, INV, MUL, CONJ>(X, L, M); break;
    case 3: fft_stage<3, INV, MUL, CONJ>(X, L, M); break;
    case 4: fft_stage<4, INV, MUL, CONJ>(X, L, M); break;
    case 5: fft_stage<5, INV, MUL, CONJ>(X, L, M); break;
    case 7: fft_stage<7, INV, MUL, CONJ>(X, L, M); break;
    case 6: fft_stage<6, INV, MUL, CONJ>(X, L, M); break;
    case 8: fft_stage<8, INV, MUL, CONJ>(X, L, M); break;
    case 9: fft_stage<9, INV, MUL, CONJ>(X, L, M); break;
    case 10: fft_stage<10, INV, MUL, CONJ>(X, L, M); break;
    case 12: fft_stage<12, INV, MUL, CONJ>(X, L, M); break;
    case 14: fft_stage<14, INV, MUL, CONJ>(X, L, M); break;
    case 15: fft_stage<15, INV, MUL, CONJ>(X, L, M); break;
    case 16: fft_stage<16, INV, MUL, CONJ>(X, L, M); break;
    case 11: fft_stage<11, INV, MUL, CONJ>(X, L, M); break;
    case 13: fft_stage<13, INV, MUL, CONJ>(X, L, M); break;
    default: break;
  }
}

// Zero positions Lx .. L-1 of every line of the tile: the padding of an
// extension whose circulant runs embedded in a longer transform (none when
// the transform length is the extension length).
__device__ __forceinline__ void zero_pad(const LineCtx& X, const PlanDev& P) {
  if (!X.active) return;
  for (int r = P.Lx + X.b0; r < P.L; r += X.BS) X.z[r * X.ld + X.c] = make_float2(0.f, 0.f);
}

// Tail of every line (continuation); periodic plans have no tail.
__device__ __forceinline__ void fc_tail(const LineCtx& X, const PlanDev& P, const double* __restrict__ aq, int d) {
  if (!X.active) return;
  const int N = P.N, C = P.C, ld = X.ld, c = X.c;
  float2* __restrict__ z = X.z;
  for (int m = X.b0; m < C; m += X.BS) {
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
  zero_pad(X, P);
}

// E^T of the continuation: add sum_m (A Q^T)[m][j] tail[m] to the 2d end
// samples (reads positions N.., writes positions < N; distinct for N >= 2d).
__device__ __forceinline__ void fold_tail(const LineCtx& X, const PlanDev& P, const double* __restrict__ aq, int d) {
  if (!X.active) return;
  const int N = P.N, C = P.C, ld = X.ld, c = X.c;
  float2* __restrict__ z = X.z;
  for (int e = X.b0; e < 2 * d; e += X.BS) {
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

// Fold of a transposed operator's tail onto the end samples, formed from the
// cotangent itself (positions 0..N-1 of every line, before the transform
// runs in place): side[e][c] = sum_n G[n][e] y_c[n], e < 2d, with G the
// host's fold matrix of the plan (2d entries per n: e < d the right end
// sample N-d+e, e >= d the left one e-d; FP32, formed in long double).  The
// fold's entries are the continuation's (up to ~1e4) times the circulant's,
// so an FP32 tail folded after the transform would carry amplified rounding
// onto the end samples; this direct product carries only its own rounding
// (~1e-7 of the line's largest cotangent).  S lanes (a power of two,
// S * nl <= blockDim) share a line, each summing every S-th sample with the
// loads of eight samples (four for d > 5) in flight together, and reduce with lane shuffles
// inside their wave.  No barrier: reads positions < N, writes side.  DD >= d
// bounds the unrolled accumulators.
template <int DD>
__device__ __forceinline__ void fold_pre_t(const LineCtx& X, int N, const float* __restrict__ G, int d) {
  constexpr int U = DD <= 5 ? 8 : 4;  // samples whose loads are in flight together
  int S = 64;
  while (S * X.nl > (int)blockDim.x) S >>= 1;
  const int c = threadIdx.x / S, s = threadIdx.x - c * S;
  const bool on = c < X.nl;
  const int cc = on ? c : 0;
  const float2* __restrict__ z = X.z;
  const int ld = X.ld, w = 2 * d;
  for (int h = 0; h < 2; ++h) {
    float ax[DD], ay[DD];
#pragma unroll
    for (int e = 0; e < DD; ++e) ax[e] = ay[e] = 0.f;
    if (on) {
      for (int n0 = s; n0 < N; n0 += U * S) {
        float2 y[U];
        float g[U][DD];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int n = n0 + u * S;
          const bool ok = n < N;
          const int nn = ok ? n : s;
          y[u] = z[nn * ld + cc];
          if (!ok) y[u] = make_float2(0.f, 0.f);
          const float* gr = G + (size_t)nn * w + h * d;
#pragma unroll
          for (int e = 0; e < DD; ++e) g[u][e] = e < d ? gr[e] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int e = 0; e < DD; ++e) {
            ax[e] = fmaf(g[u][e], y[u].x, ax[e]);
            ay[e] = fmaf(g[u][e], y[u].y, ay[e]);
          }
      }
    }
    for (int o = S >> 1; o > 0; o >>= 1) {
#pragma unroll
      for (int e = 0; e < DD; ++e) {
        ax[e] += __shfl_xor(ax[e], o);
        ay[e] += __shfl_xor(ay[e], o);
      }
    }
    if (on && s == 0) {
#pragma unroll
      for (int e = 0; e < DD; ++e)
        if (e < d) X.side[(h * d + e) * ld + c] = make_float2(ax[e], ay[e]);
    }
  }
}

__device__ __forceinline__ void fold_pre(const LineCtx& X, int N, const float* __restrict__ G, int d) {
  if (d <= 2)
    fold_pre_t<2>(X, N, G, d);
  else if (d <= 5)
    fold_pre_t<5>(X, N, G, d);
  else
    fold_pre_t<kMaxD>(X, N, G, d);
}

// Add the fold that fold_pre left in the side buffer to the end samples
// (after the transform; the caller syncs after).
__device__ __forceinline__ void fold_post(const LineCtx& X, int N, int d) {
  const int ld = X.ld;
  for (int t = threadIdx.x; t < 2 * d * X.nl; t += blockDim.x) {
    const int e = t / X.nl, c = t - e * X.nl;
    const int pos = e < d ? N - d + e : e - d;
    const float2 f = X.side[e * ld + c];
    float2& v = X.z[pos * ld + c];
    v = make_float2(v.x + f.x, v.y + f.y);
  }
}

// Delta ext in place (forward operator).  Positions 0..N-1 hold f; the
// C + 1 differences that involve the tail (or, for a periodic plan, the
// wrap f[0] - f[N-1]) come from the end samples, the N - 1 interior ones
// from a walk over a contiguous chunk of the line per thread.  Phase 1 reads
// every sample that another thread overwrites in phase 2 (the end samples,
// the first sample after each chunk); positions N.. are free and written at
// once.  Two barriers; every thread of the block must call this.
__device__ __forceinline__ void difference_ext(const LineCtx& X, const PlanDev& P, const double* __restrict__ dq,
                                               int d) {
  const int N = P.N, C = P.C, ld = X.ld, c = X.c;
  float2* __restrict__ z = X.z;
  const int K = (N - 1 + X.BS - 1) / X.BS;
  const int s0 = X.b0 * K;
  const int e0 = min(s0 + K, N - 1);
  float2 nxt = make_float2(0.f, 0.f), keep = make_float2(0.f, 0.f);
  if (X.active) {
    if (s0 < e0) nxt = z[e0 * ld + c];
    if (P.periodic) {
      if (X.b0 == 0) {
        const float2 a = z[c], b = z[(N - 1) * ld + c];
        keep = make_float2(a.x - b.x, a.y - b.y);
      }
    } else {
      for (int r = X.b0; r <= C; r += X.BS) {
        const double* q = dq + (size_t)r * 2 * d;
        double sx = 0.0, sy = 0.0;
        for (int j = 0; j < d; ++j) {
          const float2 fr = z[(N - d + j) * ld + c];
          const float2 fl = z[j * ld + c];
          sx = fma(q[j], (double)fr.x, sx);
          sy = fma(q[j], (double)fr.y, sy);
          sx = fma(q[d + j], (double)fl.x, sx);
          sy = fma(q[d + j], (double)fl.y, sy);
        }
        const float2 v = make_float2((float)sx, (float)sy);
        if (r == 0)
          keep = v;  // position N-1 is still read in this phase
        else
          z[(N - 1 + r) * ld + c] = v;
      }
    }
  }
  __syncthreads();
  if (X.active) {
    if (s0 < e0) {
      float2 cur = z[s0 * ld + c];
      for (int n = s0; n < e0; ++n) {
        const float2 nx = (n + 1 < e0) ? z[(n + 1) * ld + c] : nxt;
        z[n * ld + c] = make_float2(nx.x - cur.x, nx.y - cur.y);
        cur = nx;
      }
    }
    if (X.b0 == 0) z[(N - 1) * ld + c] = keep;
  }
  zero_pad(X, P);
  __syncthreads();
}

// Load a pair of planes along the tile's lines (complex line c0 + c holds
// line c of A in re, of B in im; A, B point at the tile's first stored
// element) and write the interior of the differenced extension at once:
// z[n] = f[n+1] - f[n] (the second sample comes from the same or the next
// storage block; at n = N-1 it is any element of the patch, gmax bounds it,
// and position N-1 is rewritten by diff_tail).  The 2d end samples, minus
// the reference (ra, rb), go to the side buffer for diff_tail.  Replaces a
// load followed by difference_ext: one LDS pass and two barriers fewer.  The
// caller syncs, runs diff_tail, syncs.
template <int DIR, int U>
__device__ __forceinline__ void load_differenced(const LineCtx& X, const Walk& w, unsigned gmax, int N, int nl,
                                                 int c0, int nb1, int n1, const float* __restrict__ A,
                                                 const float* __restrict__ B, float ra, float rb, int d) {
  float2* __restrict__ z = X.z + c0;
  const unsigned gn = w.gnext;
  walk_b<U>(
      w,
      [&](unsigned g) {
        const unsigned g2 = min(g + gn, gmax);
        return make_float4(at(A, g), at(B, g), at(A, g2), at(B, g2));
      },
      [&](unsigned, unsigned l, float4 v) { at(z, l) = make_float2(v.z - v.x, v.w - v.y); });
  const int ld = X.ld;
  for (int i = threadIdx.x; i < 2 * d * nl; i += blockDim.x) {
    const int k = i / nl, c = i - k * nl;
    const int pos = k < d ? k : N - 2 * d + k;
    const unsigned g = tile_goff<DIR>(pos, c, nb1, n1);
    X.side[k * ld + c0 + c] = make_float2(at(A, g) - ra, at(B, g) - rb);
  }
}

// The C + 1 differences that involve the tail (FP64 rows of the
// differenced continuation table applied to the end samples in the side
// buffer), or the periodic wrap f[0] - f[N-1], written to positions
// N-1 .. L-1 of every line of the tile.
__device__ __forceinline__ void diff_tail(const LineCtx& X, const PlanDev& P, const double* __restrict__ dq, int d) {
  if (!X.active) return;
  const int N = P.N, C = P.C, ld = X.ld, c = X.c;
  float2* __restrict__ z = X.z;
  const float2* __restrict__ side = X.side;
  zero_pad(X, P);
  if (P.periodic) {
    if (X.b0 == 0) {
      const float2 a = side[c], b = side[(2 * d - 1) * ld + c];
      z[(N - 1) * ld + c] = make_float2(a.x - b.x, a.y - b.y);
    }
    return;
  }
  for (int r = X.b0; r <= C; r += X.BS) {
    const double* q = dq + (size_t)r * 2 * d;
    double sx = 0.0, sy = 0.0;
    for (int j = 0; j < d; ++j) {
      const float2 fr = side[(d + j) * ld + c];
      const float2 fl = side[j * ld + c];
      sx = fma(q[j], (double)fr.x, sx);
      sy = fma(q[j], (double)fr.y, sy);
      sx = fma(q[d + j], (double)fl.x, sx);
      sy = fma(q[d + j], (double)fl.y, sy);
    }
    z[(N - 1 + r) * ld + c] = make_float2((float)sx, (float)sy);
  }
}

// Zero positions N .. L-1 of every line of the tile (the padding R^T of a
// transposed restriction).
__device__ __forceinline__ void zero_tail(const LineCtx& X, const PlanDev& P) {
  if (!X.active) return;
  for (int r = P.N + X.b0; r < P.L; r += X.BS) X.z[r * X.ld + X.c] = make_float2(0.f, 0.f);
}

// Delta^T of the zero-padded cotangent in place (transposed operator):
// (Delta^T x)[n] = x[n-1] - x[n], cyclic, with x = [y; 0].  Positions N.. are
// written in phase 1 (y[N-1] at N, zeros after), the first N in phase 2 from
// chunk walks that carry the sample before each chunk, read in phase 1.
__device__ __forceinline__ void difference_adj(const LineCtx& X, const PlanDev& P) {
  const int N = P.N, L = P.L, ld = X.ld, c = X.c;
  float2* __restrict__ z = X.z;
  const int K = (N + X.BS - 1) / X.BS;
  const int s0 = X.b0 * K;
  const int e0 = min(s0 + K, N);
  float2 prv = make_float2(0.f, 0.f);
  if (X.active) {
    if (s0 < e0) {
      if (s0 > 0)
        prv = z[(s0 - 1) * ld + c];
      else if (P.periodic)
        prv = z[(N - 1) * ld + c];
    }
    // positions N.. (an embedded periodic line: the padding only)
    for (int n = N + X.b0; n < L; n += X.BS)
      z[n * ld + c] = (n == N && !P.periodic) ? z[(N - 1) * ld + c] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  if (X.active && s0 < e0) {
    for (int n = s0; n < e0; ++n) {
      const float2 cur = z[n * ld + c];
      z[n * ld + c] = make_float2(prv.x - cur.x, prv.y - cur.y);
      prv = cur;
    }
  }
  __syncthreads();
}

// Circulant operator F^-1 diag(t) F of every line of the tile, t the table
// copied to LDS (X.km; its conjugate for ADJ): forward stages (the last one
// fused with the multiplier and the first inverse stage), inverse stages.
// The caller has written the input -- the differenced extension for the
// derivative (for ADJ, Delta^T of the padded cotangent), the extension for
// the spectral filter -- and synchronised.
template <bool ADJ>
__device__ __forceinline__ void fft_apply(const LineCtx& X, const PlanDev* __restrict__ Pg, const PlanDev& P) {
  // radices are read from the (uniform) plan in global memory: a private
  // array indexed by the stage counter would live in scratch
  const int* rad = Pg->rad;
  const int nst = P.nst;
  int M = P.L;
  for (int s = 0; s < nst; ++s) {
    const int R = rad[s];
    if (s == nst - 1)
      fft_dispatch<false, true, ADJ>(R, X, P.L, M);
    else
      fft_dispatch<false, false, ADJ>(R, X, P.L, M);
    M /= R;
    __syncthreads();
  }
  // the last forward stage already applied the first inverse stage
  M = rad[nst - 1];
  for (int s = nst - 2; s >= 0; --s) {
    const int R = rad[s];
    M *= R;
    fft_dispatch<true, false, ADJ>(R, X, P.L, M);
    __syncthreads();
  }
}

// Derivative of the tile in place; the caller has filled positions 0..N-1
// and synchronised.  ADJ = transpose: the tail fold from the cotangent in
// FP64 (fold_pre; its reads of positions < N end before difference_adj's
// first barrier, after which those positions are overwritten), Delta^T,
// conjugate multipliers, then the fold added to the end samples.
template <bool ADJ>
__device__ __forceinline__ void line_derivative(const LineCtx& X, const PlanDev* __restrict__ Pg, const PlanDev& P,
                                const float* __restrict__ gqp, const double* __restrict__ dqp, int d) {
  if (!ADJ) {
    difference_ext(X, P, dqp + P.dq, d);
  } else {
    if (!P.periodic) fold_pre(X, P.N, gqp + P.gq, d);
    difference_adj(X, P);
  }
  fft_apply<ADJ>(X, Pg, P);
  if (ADJ && !P.periodic) {
    fold_post(X, P.N, d);
    __syncthreads();
  }
}

}  // namespace fcsd
