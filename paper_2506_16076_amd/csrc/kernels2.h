// Pointwise and stencil kernels: SSPRK register update, step size, proxy and
// network classifier, preliminary viscosity, smoothing-blending operator,
// multi-patch glue and the reverse-mode passes of the right-hand side.
#pragma once
#include "kernels.h"

namespace fcsd {

constexpr int kChunk = 256;  // points per chunk of the pointwise kernels

struct PatchDev {
  int n1, n2;
  long long off;
  float hhat, htilde;
  int internal;  // bit s set: side s (q1-, q1+, q2-, q2+) internal
  int nb1;       // 0: row-major patch storage; else 8x4-blocked with nb1 blocks per block row
};

// Plane index of point (i, j) of a patch.  Row-major: off + j n1 + i.
// 8x4-blocked: blocks of 8 points along q1 by 4 along q2 (128 bytes, one
// cache line), block (i/8, j/4) at off + 32 (j/4 nb1 + i/8), row-major
// inside the block.  A column tile of 8 q2 lines and a row tile of 4 q1
// lines then both read whole cache lines.
__host__ __device__ __forceinline__ long long pidx(const PatchDev& P, int i, int j) {
  if (P.nb1 == 0) return P.off + (long long)j * P.n1 + i;
  return P.off + ((((long long)(j >> 2)) * P.nb1 + (i >> 3)) << 5) + ((j & 3) << 3) + (i & 7);
}

// elements of patch storage (padded to whole blocks when blocked)
__device__ __forceinline__ int pstore(const PatchDev& P) {
  return P.nb1 == 0 ? P.n1 * P.n2 : (P.nb1 << 3) * ((P.n2 + 3) & ~3);
}

// ---------------------------------------------------------------- inter-patch interpolation

// A fringe point and its donor stencil: receiver patch and indices, donor
// patch, stencil centre and the point's local donor coordinates.
struct InterpDev {
  int rp, ri, rj;
  int dp, di, dj;
  float s, t;
};

// Quadratic through (-1, ym), (0, y0), (1, yp) at s by Neville's recurrence
// (the two linear interpolants, then their combination).
__device__ __forceinline__ float neville3(float ym, float y0, float yp, float s) {
  const float p01 = (s + 1.0f) * y0 - s * ym;
  const float p12 = (1.0f - s) * y0 + s * yp;
  return 0.5f * ((s + 1.0f) * p12 - (s - 1.0f) * p01);
}

// Fringe values from the donor patches (paper Sec. 3.4.1): iterated
// quadratic interpolation on the 3 x 3 donor stencil, along q1 on its three
// rows, then along q2; one thread per (fringe point, field).  Donor points
// are never receivers, so every thread reads values no thread writes.
__global__ void __launch_bounds__(kBlock) k_interp(const InterpDev* __restrict__ tab, int n,
                                                   const PatchDev* __restrict__ patches, float* u, long long pl) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= 4 * n) return;
  const int f = k / n;
  const InterpDev e = tab[k - f * n];
  const PatchDev D = patches[e.dp];
  const PatchDev R = patches[e.rp];
  const float* v = u + f * pl;
  float x[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) x[3 * r + c] = v[pidx(D, e.di - 1 + c, e.dj - 1 + r)];
  float row[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) row[r] = neville3(x[3 * r], x[3 * r + 1], x[3 * r + 2], e.s);
  u[f * pl + pidx(R, e.ri, e.rj)] = neville3(row[0], row[1], row[2], e.t);
}

// Transpose of k_interp: every fringe point's cotangent goes to its nine
// donor points with the weights of the quadratic Neville's recurrence
// evaluates (Lagrange weights of the nodes -1, 0, 1) and is then zeroed;
// one thread per (fringe point, field).
__global__ void __launch_bounds__(kBlock) k_interp_adj(const InterpDev* __restrict__ tab, int n,
                                                       const PatchDev* __restrict__ patches, float* ub, long long pl) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= 4 * n) return;
  const int f = k / n;
  const InterpDev e = tab[k - f * n];
  const PatchDev D = patches[e.dp];
  const PatchDev R = patches[e.rp];
  float* v = ub + f * pl;
  const long long r = pidx(R, e.ri, e.rj);
  const float g = v[r];
  v[r] = 0.0f;
  const float ws[3] = {0.5f * e.s * (e.s - 1.0f), 1.0f - e.s * e.s, 0.5f * e.s * (e.s + 1.0f)};
  const float wt[3] = {0.5f * e.t * (e.t - 1.0f), 1.0f - e.t * e.t, 0.5f * e.t * (e.t + 1.0f)};
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int a = 0; a < 3; ++a) atomicAdd(v + pidx(D, e.di - 1 + a, e.dj - 1 + b), wt[b] * ws[a] * g);
}

// ---------------------------------------------------------------- walls

// A wall side of a patch: patch index and side (q1-, q1+, q2-, q2+).
// One entry of a patch's wall condition: the non-corner points t in
// [lo, hi) of a wall side (end < 0), or the corner point where the side
// meets the wall at its tangential end `end` (0: t = 0, 1: t = last; the
// q1 side owns a corner it shares with a q2 side).
struct WallDev {
  int patch, side, lo, hi, end;
};

// Grid offset of the point kk steps from wall `side` along its normal and
// tt along the wall (from its t = 0 end).
__device__ __forceinline__ long long wall_at(const PatchDev& P, int side, int kk, int tt) {
  switch (side) {
    case 0: return pidx(P, kk, tt);
    case 1: return pidx(P, P.n1 - 1 - kk, tt);
    case 2: return pidx(P, tt, kk);
    default: return pidx(P, tt, P.n2 - 1 - kk);
  }
}

__device__ __forceinline__ float theta_at(const float* u, long long pl, long long g, float g1) {
  const float rho = u[g], m = u[pl + g], n = u[2 * pl + g], E = u[3 * pl + g];
  return g1 * (E - 0.5f * (m * m + n * n) / rho) / rho;
}

// theta_w of a wall entry's point t: along its normal line (c[k] theta(k)),
// or at a corner the tensor product of the two one-sided Neumann values
// (c[k] c[l] theta(k, l) over the interior points k, l = 1..d-1).
__device__ __forceinline__ float wall_theta(const WallDev& w, const PatchDev& P, int t, const float* u, long long pl,
                                            float g1, int d, const float* __restrict__ c) {
  float th = 0.f;
  if (w.end < 0) {
    for (int kk = 1; kk < d; ++kk) th = fmaf(c[kk], theta_at(u, pl, wall_at(P, w.side, kk, t), g1), th);
  } else {
    const int len = w.side < 2 ? P.n2 : P.n1;
    for (int kk = 1; kk < d; ++kk)
      for (int ll = 1; ll < d; ++ll)
        th = fmaf(c[kk] * c[ll], theta_at(u, pl, wall_at(P, w.side, kk, w.end == 0 ? ll : len - 1 - ll), g1), th);
  }
  return th;
}

// Tangential position of thread t of wall entry w (corner entries: one).
__device__ __forceinline__ int wall_point(const WallDev& w, const PatchDev& P, int t) {
  if (w.end >= 0) return t == 0 ? (w.end == 0 ? 0 : (w.side < 2 ? P.n2 : P.n1) - 1) : -1;
  const int tt = w.lo + t;
  return tt < w.hi ? tt : -1;
}

// No-slip adiabatic wall (paper Remarks adiabatic_th, adiabatic): on every
// wall point, rho u = rho v = 0 and E = rho theta_w / (gamma - 1) with
// theta_w the Neumann FC boundary value of theta = p / rho for a zero
// normal slope (weights c, host-computed).  Every theta read is an interior
// point's, which no thread writes.
__global__ void __launch_bounds__(kBlock) k_wall(const WallDev* __restrict__ walls, int nwall, int maxlen,
                                                 const PatchDev* __restrict__ patches, float* u, long long pl,
                                                 float g1, int d, const float* __restrict__ c) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (long long)nwall * maxlen) return;
  const int wi = (int)(k / maxlen), t = (int)(k - (long long)wi * maxlen);
  const WallDev w = walls[wi];
  const PatchDev P = patches[w.patch];
  const int tt = wall_point(w, P, t);
  if (tt < 0) return;
  const float th = wall_theta(w, P, tt, u, pl, g1, d, c);
  const long long g0 = wall_at(P, w.side, 0, tt);
  u[pl + g0] = 0.f;
  u[2 * pl + g0] = 0.f;
  u[3 * pl + g0] = u[g0] * th / g1;
}

// Transpose of k_wall at the state it produced (eg: the glued state, whose
// wall-point rho and interior points the wall left as it found them): the
// overwritten momenta and energy drop their cotangents, rho_w gets
// theta_w / (gamma - 1) times E_w's cotangent, and every interior source its
// weight times rho_w / (gamma - 1) times E_w's cotangent through
// d theta / d e.  Entries whose sources may coincide (two sides of one
// patch, a side and a corner) run in separate launches: `only` selects the
// side (0..3) or the corners (4).
__global__ void __launch_bounds__(kBlock) k_wall_adj(const WallDev* __restrict__ walls, int nwall, int maxlen,
                                                     const PatchDev* __restrict__ patches, const float* eg, float* ub,
                                                     long long pl, float g1, int d, const float* __restrict__ c,
                                                     int only) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (long long)nwall * maxlen) return;
  const int wi = (int)(k / maxlen), t = (int)(k - (long long)wi * maxlen);
  const WallDev w = walls[wi];
  if (only < 4 ? (w.end >= 0 || w.side != only) : w.end < 0) return;
  const PatchDev P = patches[w.patch];
  const int tt = wall_point(w, P, t);
  if (tt < 0) return;
  const float th = wall_theta(w, P, tt, eg, pl, g1, d, c);
  const long long g0 = wall_at(P, w.side, 0, tt);
  const float Eb = ub[3 * pl + g0];
  const float tb = Eb * eg[g0] / g1;
  ub[g0] += Eb * th / g1;
  ub[pl + g0] = 0.f;
  ub[2 * pl + g0] = 0.f;
  ub[3 * pl + g0] = 0.f;
  auto add = [&](long long g, float wgt) {
    const float rho = eg[g], m = eg[pl + g], n = eg[2 * pl + g], E = eg[3 * pl + g];
    const float tk = wgt * tb * g1, ir = 1.0f / rho, ir2 = ir * ir;
    ub[g] += tk * (-E * ir2 + (m * m + n * n) * ir2 * ir);
    ub[pl + g] -= tk * m * ir2;
    ub[2 * pl + g] -= tk * n * ir2;
    ub[3 * pl + g] += tk * ir;
  };
  if (w.end < 0) {
    for (int kk = 1; kk < d; ++kk) add(wall_at(P, w.side, kk, tt), c[kk]);
  } else {
    const int len = w.side < 2 ? P.n2 : P.n1;
    for (int kk = 1; kk < d; ++kk)
      for (int ll = 1; ll < d; ++ll) add(wall_at(P, w.side, kk, w.end == 0 ? ll : len - 1 - ll), c[kk] * c[ll]);
  }
}

// Blending window of the initial-data smearing (paper Sec. 4.3.2, eq. qf)
// along DIR, one thread per line of one patch (blockIdx.y): a discontinuity
// sits between neighbours whose region labels differ.  A forward sweep
// stores each point's distance to the nearest discontinuity on its left, a
// backward sweep combines it with the one on the right: 1 between two
// discontinuities closer than c + 2r (one window group), else the rise
// 1 / cos^2(pi (s - c/2) / (2r)) / 0 of the nearer one (c2 = c/2).
template <int DIR>
__global__ void __launch_bounds__(kBlock) k_smear_window(const PatchDev* __restrict__ pd,
                                                          const uint8_t* __restrict__ lab, float* __restrict__ win,
                                                          float c2, float r) {
  const PatchDev P = pd[blockIdx.y];
  const int nlines = DIR == 1 ? P.n2 : P.n1;
  const int N = DIR == 1 ? P.n1 : P.n2;
  const int line = blockIdx.x * blockDim.x + threadIdx.x;
  if (line >= nlines) return;
  auto idx = [&](int t) { return DIR == 1 ? pidx(P, t, line) : pidx(P, line, t); };
  const float far = 1e30f;
  float zl = -far;
  unsigned prev = lab[idx(0)];
  for (int t = 0; t < N; ++t) {
    const long long k = idx(t);
    const unsigned cur = lab[k];
    if (cur != prev) zl = (float)t - 0.5f;
    prev = cur;
    win[k] = (float)t - zl;
  }
  float zr = far;
  unsigned next = lab[idx(N - 1)];
  for (int t = N - 1; t >= 0; --t) {
    const long long k = idx(t);
    const unsigned cur = lab[k];
    if (cur != next) zr = (float)t + 0.5f;
    next = cur;
    const float dl = win[k], dr = zr - (float)t;
    float w;
    if (dl + dr < 2.0f * (c2 + r)) {
      w = 1.0f;
    } else {
      const float s = fminf(dl, dr);
      const float cs = cosf(3.14159265358979f * (s - c2) / (2.0f * r));
      w = s < c2 ? 1.0f : (s > c2 + r ? 0.0f : cs * cs);
    }
    win[k] = w;
  }
}

// point (i, j) stored at storage index k of the patch; false for padding
__device__ __forceinline__ bool pdecode(const PatchDev& P, int k, int& i, int& j) {
  if (P.nb1 == 0) {
    j = k / P.n1;
    i = k - j * P.n1;
    return true;
  }
  const int blk = k >> 5, w = k & 31;
  const int bj = blk / P.nb1, bi = blk - bj * P.nb1;
  i = (bi << 3) + (w & 7);
  j = (bj << 2) + (w >> 3);
  return i < P.n1 && j < P.n2;
}

struct ChunkDev {
  int patch;  // patch (or lattice group) index
  int start;  // first storage index within the patch (lattice: row-major)
};

// Chunk kernels run a grid of at most kChunkGrid blocks that stride over the
// chunks (a block per 256-point chunk spends its time being scheduled).
constexpr int kChunkGrid = 2048;
template <class F>
__device__ __forceinline__ void for_chunks(const ChunkDev* chunks, int nchunks, F&& f) {
  for (int cb = blockIdx.x; cb < nchunks; cb += gridDim.x) f(chunks[cb]);
}

// ---- energy derivatives by the product rule on wall patches (Remark
// adiabatic; eqs. p_T, perfect_gas_T): with E = rho theta / (gamma - 1) +
// |m|^2 / (2 rho), dE = A d rho + B d theta + Cx d m_x + Cy d m_y,
// A = E / rho - |m|^2 / rho^2, B = rho / (gamma - 1), C = m / rho.

// theta - theta_ref at every point of the chunks (the wall patches' ones),
// formed in FP64 and rounded once: its rounding is then relative to the
// difference, as that of e - e_ref is on the other lanes, rather than to
// theta itself (two FC derivatives amplify pointwise noise by about n^2).
__global__ void __launch_bounds__(kBlock) k_theta(const ChunkDev* chunks, int nchunks, const PatchDev* patches,
                                                  const float* u, long long pl, double g1, double th_ref, float* th) {
  for_chunks(chunks, nchunks, [&](const ChunkDev ck) {
    const PatchDev P = patches[ck.patch];
    const int k = ck.start + threadIdx.x;
    int i, j;
    if (k >= pstore(P) || !pdecode(P, k, i, j)) return;
    const long long g = P.off + k;
    const double rho = u[g], m = u[pl + g], n = u[2 * pl + g], E = u[3 * pl + g];
    th[g] = (float)(g1 * (E - 0.5 * (m * m + n * n) / rho) / rho - th_ref);
  });
}

// d[3] = A d[0] + B dth + Cx d[1] + Cy d[2] at the chunks' points (d: the
// four derivative planes of one direction).
__global__ void __launch_bounds__(kBlock) k_energy_rule(const ChunkDev* chunks, int nchunks, const PatchDev* patches,
                                                        const float* u, long long pl, float g1, const float* dth,
                                                        float* d) {
  for_chunks(chunks, nchunks, [&](const ChunkDev ck) {
    const PatchDev P = patches[ck.patch];
    const int k = ck.start + threadIdx.x;
    int i, j;
    if (k >= pstore(P) || !pdecode(P, k, i, j)) return;
    const long long g = P.off + k;
    const float rho = u[g], m = u[pl + g], n = u[2 * pl + g], E = u[3 * pl + g];
    const float ir = 1.0f / rho;
    const float A = E * ir - (m * m + n * n) * ir * ir, B = rho / g1;
    d[3 * pl + g] = A * d[g] + B * dth[g] + m * ir * d[pl + g] + n * ir * d[2 * pl + g];
  });
}

// Transpose of k_energy_rule at u with the forward derivatives d (lanes
// 0..2) and dth: G (the four cotangent planes of d) gets A, Cx, Cy times
// G[3] on lanes 0..2 and G[3] = 0, tb = B G[3] (theta's lane), and ub the
// rule's coefficients' derivatives in (rho, m_x, m_y, E) times G[3].
__global__ void __launch_bounds__(kBlock) k_energy_rule_adj(const ChunkDev* chunks, int nchunks,
                                                            const PatchDev* patches, const float* u, long long pl,
                                                            float g1, const float* d, const float* dth, float* G,
                                                            float* tb, float* ub) {
  for_chunks(chunks, nchunks, [&](const ChunkDev ck) {
    const PatchDev P = patches[ck.patch];
    const int k = ck.start + threadIdx.x;
    int i, j;
    if (k >= pstore(P) || !pdecode(P, k, i, j)) return;
    const long long g = P.off + k;
    const float rho = u[g], m = u[pl + g], n = u[2 * pl + g], E = u[3 * pl + g];
    const float ir = 1.0f / rho, ir2 = ir * ir, q = m * m + n * n;
    const float gE = G[3 * pl + g];
    const float dr = d[g], dm = d[pl + g], dn = d[2 * pl + g], dt = dth[g];
    const float A = E * ir - q * ir2, B = rho / g1;
    G[g] += A * gE;
    G[pl + g] += m * ir * gE;
    G[2 * pl + g] += n * ir * gE;
    G[3 * pl + g] = 0.f;
    tb[g] = B * gE;
    // d/d(rho, m, n, E) of A dr + B dt + (m dm + n dn) / rho
    ub[g] += gE * ((-E * ir2 + 2.f * q * ir2 * ir) * dr + dt / g1 - (m * dm + n * dn) * ir2);
    ub[pl + g] += gE * (-2.f * m * ir2 * dr + dm * ir);
    ub[2 * pl + g] += gE * (-2.f * n * ir2 * dr + dn * ir);
    ub[3 * pl + g] += gE * ir * dr;
  });
}

// ub += (d theta / d e)^T thb at the chunks' points.
__global__ void __launch_bounds__(kBlock) k_theta_adj(const ChunkDev* chunks, int nchunks, const PatchDev* patches,
                                                      const float* u, long long pl, float g1, const float* thb,
                                                      float* ub) {
  for_chunks(chunks, nchunks, [&](const ChunkDev ck) {
    const PatchDev P = patches[ck.patch];
    const int k = ck.start + threadIdx.x;
    int i, j;
    if (k >= pstore(P) || !pdecode(P, k, i, j)) return;
    const long long g = P.off + k;
    const float rho = u[g], m = u[pl + g], n = u[2 * pl + g], E = u[3 * pl + g];
    const float tk = thb[g] * g1, ir = 1.0f / rho, ir2 = ir * ir;
    ub[g] += tk * (-E * ir2 + (m * m + n * n) * ir2 * ir);
    ub[pl + g] -= tk * m * ir2;
    ub[2 * pl + g] -= tk * n * ir2;
    ub[3 * pl + g] += tk * ir;
  });
}

// lattice of the smoothing-blending operator: independent patches are their
// own lattice; the index-aligned annulus is one periodic (G, J) lattice
struct LatDev {
  int W, H, periodic, pad;
  long long base;
};

struct AnnulusDev {
  int nsec, nshell, st1, st2;  // sectors, shells, n1 - 19, n2 - 19
  int n1, n2, ring, nJ;
};

constexpr int kNv = 9;      // viscosity fringe width
constexpr int kNf = 5;      // communication fringe width
constexpr int kOvl = 19;    // overlap between neighbouring patches

__device__ __forceinline__ bool in_dtilde(const PatchDev& P, int i, int j) {
  if ((P.internal & 1) && i < kNv) return false;
  if ((P.internal & 2) && i >= P.n1 - kNv) return false;
  if ((P.internal & 4) && j < kNv) return false;
  if ((P.internal & 8) && j >= P.n2 - kNv) return false;
  return true;
}

// ---------------------------------------------------------------- SSPRK

__global__ void __launch_bounds__(kBlock) k_rk(int stage, const float* dtp, const float* rhs,
                                               const float* u0, const float* ui, float* acc,
                                               float* uout, long long n4) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n4) return;
  const RkCoef K = rk_coef(stage);
  const float dr = dtp[0] * rhs[g];
  const float x = ui[g];
  if (stage <= 1) {
    uout[g] = K.a0 * u0[g] + K.ai * x + K.b * dr;
  } else if (stage == 2) {
    uout[g] = K.a0 * u0[g] + K.ai * x + K.b * dr;
    acc[g] = K.acc_i * x;
  } else if (stage == 3) {
    uout[g] = K.a0 * u0[g] + K.ai * x + K.b * dr;
    acc[g] += K.acc_i * x + K.acc_b * dr;
  } else {
    uout[g] = acc[g] + K.ai * x + K.b * dr;
  }
}

// reverse of k_rk; rhs_bar is overwritten (each stage's r is used once)
__global__ void __launch_bounds__(kBlock) k_rk_adj(int stage, const float* dtp, const float* ob,
                                                   float* u0b, float* uib, float* accb, float* rb,
                                                   long long n4, bool fresh = false) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n4) return;
  const RkCoef K = rk_coef(stage);
  const float dt = dtp[0];
  const float y = ob[g];
  if (fresh && stage > 0) {
    // uib starts at zero (written, not accumulated): the same values as
    // accumulating into a zero-filled uib, without the fill and its read
    if (stage == 1) {
      u0b[g] += K.a0 * y;
      uib[g] = K.ai * y;
      rb[g] = K.b * dt * y;
    } else if (stage == 2) {
      const float ab = accb[g];
      u0b[g] += K.a0 * y;
      uib[g] = K.ai * y + K.acc_i * ab;
      rb[g] = K.b * dt * y;
      accb[g] = 0.f;
    } else if (stage == 3) {
      const float ab = accb[g];
      u0b[g] += K.a0 * y;
      uib[g] = K.ai * y + K.acc_i * ab;
      rb[g] = dt * (K.b * y + K.acc_b * ab);
    } else {
      accb[g] += y;
      uib[g] = K.ai * y;
      rb[g] = K.b * dt * y;
    }
    return;
  }
  if (stage == 0) {
    u0b[g] += y;
    rb[g] = K.b * dt * y;
  } else if (stage == 1) {
    u0b[g] += K.a0 * y;
    uib[g] += K.ai * y;
    rb[g] = K.b * dt * y;
  } else if (stage == 2) {
    const float ab = accb[g];
    u0b[g] += K.a0 * y;
    uib[g] += K.ai * y + K.acc_i * ab;
    rb[g] = K.b * dt * y;
    accb[g] = 0.f;
  } else if (stage == 3) {
    const float ab = accb[g];
    u0b[g] += K.a0 * y;
    uib[g] += K.ai * y + K.acc_i * ab;
    rb[g] = dt * (K.b * y + K.acc_b * ab);
  } else {
    accb[g] += y;
    uib[g] += K.ai * y;
    rb[g] = K.b * dt * y;
  }
}

// ---------------------------------------------------------------- proxy, S

// Primitive variables with one IEEE rounding per operation in a fixed order
// (no contraction): the network classes and the 7x7 maximiser are integer
// decisions taken on these FP32 values.
__device__ __forceinline__ void prim(const float* u, long long pl, long long g, float gam, float& rho,
                                     float& vx, float& vy, float& p) {
#pragma clang fp contract(off)
  rho = u[g];
  const float ir = 1.0f / rho;
  vx = u[pl + g] * ir;
  vy = u[2 * pl + g] * ir;
  p = (gam - 1.0f) * (u[3 * pl + g] - 0.5f * rho * (vx * vx + vy * vy));
}

// Phi = |u| sqrt(rho/(gamma p)) and S = |u| + |v| + a on every patch point
__global__ void __launch_bounds__(kBlock) k_proxy(const ChunkDev* chunks, int nchunks, const PatchDev* patches,
                                                  const float* u, long long pl, float gam, float* phi,
                                                  float* S) {
  for_chunks(chunks, nchunks, [&](const ChunkDev ck) {
    const PatchDev P = patches[ck.patch];
    const int k = ck.start + threadIdx.x;
    int i, j;
    if (k >= pstore(P) || !pdecode(P, k, i, j)) return;
    const long long g = P.off + k;
    {
  #pragma clang fp contract(off)
      float rho, vx, vy, p;
      prim(u, pl, g, gam, rho, vx, vy, p);
      const float a = sqrtf((gam * p) / rho);
      if (phi) phi[g] = sqrtf(vx * vx + vy * vy) / a;
      if (S) S[g] = (fabsf(vx) + fabsf(vy)) + a;
    }
  });
}

// ---------------------------------------------------------------- network

struct MlpPtr {
  const float *W1, *b1, *W2, *b2, *W3, *b3;
};

// The 16-64-64-4 classifier on the fp16 matrix cores with FP32 accuracy
// (operands split into fp16 high and 2^11-scaled low parts, products summed
// in FP32; see mlp16x2).  A wavefront evaluates 16 windows at once, as the transposed
// products H1^T = W1^T X^T, H2^T = W2^T relu(H1^T), O^T = W3^T relu(H2^T)
// with windows along the columns.  Lane l = 16 g + r holds column r (window
// r) and, after each product, rows 4 g + v (v = 0..3) of every 16-row tile
// -- exactly the B operand the next product needs when its K step k = 0..3
// is read as unit 16 t + 4 k + v: activations never leave the registers.
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef _Float16 half4 __attribute__((ext_vector_type(4)));
typedef _Float16 half8 __attribute__((ext_vector_type(8)));

// The network's products run on the fp16 matrix cores with FP32 accuracy:
// every operand v is split as v = hi + lo, hi = fp16(v) (round to nearest),
// lo = v - hi (exact in FP32, |lo| <= 2^-11 |v|), and a product sum is
//     sum hi_a hi_b  +  2^-11 sum (lo_a 2^11 hi_b + hi_a lo_b 2^11)
// with the low parts scaled by 2^11 so that they stay normal fp16 numbers;
// the dropped lo lo term is below 2^-22 of each product.  The main and the
// correction sums accumulate in FP32 in two accumulators.
constexpr float kLoScale = 2048.0f;
constexpr float kLoUnscale = 1.0f / 2048.0f;

// Weights in LDS in the operand layout of the fp16 products.  For lane group
// g (lanes 16 g .. 16 g + 15) and row n = lane % 16, a half8 holds the
// contraction slots k = 16 (2 p) + 4 g + e (e = 0..3) followed by
// k = 16 (2 p + 1) + 4 g + e: a 32-unit chunk pair p.  A layer's output tile
// t (rows 16 t + 4 g + v in lane group g, D layout) is, as it stands in the
// registers, half of chunk pair t / 2 of the next layer's contraction.
// Separate arrays hold the high parts and the 2^11-scaled low parts, so the
// main product and the two corrections each read one half8.
struct MlpLds {
  half4 W1h[4][4][16];        // [output tile t][g][n]: hi of W1[4 e + g][16 t + n] (slots: feature 4 e + g)
  half8 W1c[4][4][16];        // {lo * 2^11 (e = 0..3), hi (e = 0..3)} of the same
  half8 W2h[4][2][4][16];     // [output tile mt][pair p][g][n]: hi of W2[k][16 mt + n]
  half8 W2l[4][2][4][16];     // lo * 2^11 of the same
  half8 W3h[2][4][16];        // [pair p][g][n]: hi of W3[k][n] (n < 4), zero rows n >= 4
  half8 W3l[2][4][16];
  float b1[64];
  float b2[64];
  float b3[4];
};

__device__ __forceinline__ void split1(float w, _Float16& h, _Float16& l) {
  h = (_Float16)w;
  // (w - hi) 2^11 in one mixed-precision fma (exact: w - hi is exact in FP32)
  l = (_Float16)__builtin_fmaf((float)h, -kLoScale, w * kLoScale);
}

__device__ __forceinline__ void mlp_load(MlpLds& L, const MlpPtr& w) {
  for (int q = threadIdx.x; q < 4 * 4 * 16 * 4; q += blockDim.x) {
    const int e = q & 3, n = (q >> 2) & 15, g = (q >> 6) & 3, t = q >> 8;
    _Float16 h, l;
    split1(w.W1[(4 * e + g) * 64 + 16 * t + n], h, l);
    ((_Float16*)&L.W1h[t][g][n])[e] = h;
    ((_Float16*)&L.W1c[t][g][n])[e] = l;
    ((_Float16*)&L.W1c[t][g][n])[4 + e] = h;
  }
  for (int q = threadIdx.x; q < 4 * 2 * 4 * 16 * 8; q += blockDim.x) {
    const int e = q & 7, n = (q >> 3) & 15, g = (q >> 7) & 3, pp = (q >> 9) & 1, mt = q >> 10;
    const int k = 16 * (2 * pp + (e >> 2)) + 4 * g + (e & 3);
    _Float16 h, l;
    split1(w.W2[k * 64 + 16 * mt + n], h, l);
    ((_Float16*)&L.W2h[mt][pp][g][n])[e] = h;
    ((_Float16*)&L.W2l[mt][pp][g][n])[e] = l;
  }
  for (int q = threadIdx.x; q < 2 * 4 * 16 * 8; q += blockDim.x) {
    const int e = q & 7, n = (q >> 3) & 15, g = (q >> 7) & 3, pp = q >> 9;
    const int k = 16 * (2 * pp + (e >> 2)) + 4 * g + (e & 3);
    _Float16 h, l;
    split1(n < 4 ? w.W3[k * 4 + n] : 0.f, h, l);
    ((_Float16*)&L.W3h[pp][g][n])[e] = h;
    ((_Float16*)&L.W3l[pp][g][n])[e] = l;
  }
  for (int k = threadIdx.x; k < 64; k += blockDim.x) {
    L.b1[k] = w.b1[k];
    L.b2[k] = w.b2[k];
  }
  if (threadIdx.x < 4) L.b3[threadIdx.x] = w.b3[threadIdx.x];
}

// relu(m + c 2^-11) of two output tiles, split into the hi and scaled-lo
// half8 operands of a chunk pair (tile a in slots 0..3, tile b in 4..7);
// neighbouring slots are converted together (one packed conversion each)
typedef _Float16 half2v __attribute__((ext_vector_type(2)));
typedef float float2v __attribute__((ext_vector_type(2)));
template <bool RELU>
__device__ __forceinline__ void finish_pair(const floatx4 ma, const floatx4 ca, const floatx4 mb,
                                            const floatx4 cb, half8& h, half8& l) {
  float x[8];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    x[v] = ma[v] + ca[v] * kLoUnscale;
    x[4 + v] = mb[v] + cb[v] * kLoUnscale;
  }
  if (RELU) {
#pragma unroll
    for (int v = 0; v < 8; ++v) x[v] = fmaxf(x[v], 0.f);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const half2v hh = __builtin_convertvector(float2v{x[2 * q], x[2 * q + 1]}, half2v);
    h[2 * q] = hh[0];
    h[2 * q + 1] = hh[1];
    // (x - hi) 2^11, exact before its rounding to fp16
    l[2 * q] = (_Float16)__builtin_fmaf((float)hh[0], -kLoScale, x[2 * q] * kLoScale);
    l[2 * q + 1] = (_Float16)__builtin_fmaf((float)hh[1], -kLoScale, x[2 * q + 1] * kLoScale);
  }
}

// Logits of two sets of 16 windows (the two directions at the same 16
// points); lane 16 g + r supplies features 4 s + g (s = 0..3) of window r in
// x0[s] and x1[s]; lanes 0..15 receive the four logits of window r of each.
// Each product is computed transposed (windows along the columns), so the
// D layout of one layer's output is the B layout of the next.  The layers of
// the two evaluations are interleaved (the matrix products of one overlap
// the vector work of the other) and share each read of the weights from
// LDS.
__device__ __forceinline__ void mlp16x2(const MlpLds& L, const float x0[4], const float x1[4], int g, int r,
                                        floatx4& o0, floatx4& o1) {
  half4 xh[2];
  half8 xb[2];
#pragma unroll
  for (int d = 0; d < 2; ++d) {
    const float* x = d ? x1 : x0;
    half4 xl;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      _Float16 t0, t1;
      split1(x[e], t0, t1);
      xh[d][e] = t0;
      xl[e] = t1;
    }
    xb[d] = half8{xh[d][0], xh[d][1], xh[d][2], xh[d][3], xl[0], xl[1], xl[2], xl[3]};
  }
  half8 ah[2][2], al[2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    floatx4 m[2][2], c[2][2];
#pragma unroll
    for (int d = 0; d < 2; ++d)
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int t = 2 * p + u;
        m[d][u] = floatx4{L.b1[16 * t + 4 * g], L.b1[16 * t + 4 * g + 1], L.b1[16 * t + 4 * g + 2],
                          L.b1[16 * t + 4 * g + 3]};
        c[d][u] = floatx4{0.f, 0.f, 0.f, 0.f};
        m[d][u] = __builtin_amdgcn_mfma_f32_16x16x16f16(L.W1h[t][g][r], xh[d], m[d][u], 0, 0, 0);
        c[d][u] = __builtin_amdgcn_mfma_f32_16x16x32_f16(L.W1c[t][g][r], xb[d], c[d][u], 0, 0, 0);
      }
#pragma unroll
    for (int d = 0; d < 2; ++d) finish_pair<true>(m[d][0], c[d][0], m[d][1], c[d][1], ah[d][p], al[d][p]);
  }
  half8 bh[2][2], bl[2][2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    floatx4 m[2][2], c[2][2];
#pragma unroll
    for (int d = 0; d < 2; ++d)
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int mt = 2 * q + u;
        m[d][u] = floatx4{L.b2[16 * mt + 4 * g], L.b2[16 * mt + 4 * g + 1], L.b2[16 * mt + 4 * g + 2],
                          L.b2[16 * mt + 4 * g + 3]};
        c[d][u] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          m[d][u] = __builtin_amdgcn_mfma_f32_16x16x32_f16(L.W2h[mt][p][g][r], ah[d][p], m[d][u], 0, 0, 0);
          c[d][u] = __builtin_amdgcn_mfma_f32_16x16x32_f16(L.W2l[mt][p][g][r], ah[d][p], c[d][u], 0, 0, 0);
          c[d][u] = __builtin_amdgcn_mfma_f32_16x16x32_f16(L.W2h[mt][p][g][r], al[d][p], c[d][u], 0, 0, 0);
        }
      }
#pragma unroll
    for (int d = 0; d < 2; ++d) finish_pair<true>(m[d][0], c[d][0], m[d][1], c[d][1], bh[d][q], bl[d][q]);
  }
  floatx4 m[2], c[2];
#pragma unroll
  for (int d = 0; d < 2; ++d) {
    m[d] = g == 0 ? floatx4{L.b3[0], L.b3[1], L.b3[2], L.b3[3]} : floatx4{0.f, 0.f, 0.f, 0.f};
    c[d] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      m[d] = __builtin_amdgcn_mfma_f32_16x16x32_f16(L.W3h[p][g][r], bh[d][p], m[d], 0, 0, 0);
      c[d] = __builtin_amdgcn_mfma_f32_16x16x32_f16(L.W3l[p][g][r], bh[d][p], c[d], 0, 0, 0);
      c[d] = __builtin_amdgcn_mfma_f32_16x16x32_f16(L.W3h[p][g][r], bl[d][p], c[d], 0, 0, 0);
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    o0[v] = m[0][v] + c[0][v] * kLoUnscale;
    o1[v] = m[1][v] + c[1][v] * kLoUnscale;
  }
}

// min and max of finite values (the window samples) without the NaN
// quieting of the operands that fminf / fmaxf add
__device__ __forceinline__ float fmin2(float a, float b) {
  float r;
  asm("v_min_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ float fmax2(float a, float b) {
  float r;
  asm("v_max_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ float fmin3(float a, float b, float c) {
  float r;
  asm("v_min3_f32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}
__device__ __forceinline__ float fmax3(float a, float b, float c) {
  float r;
  asm("v_max3_f32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}

// Minimum and maximum over the four lanes 16 g + r (g = 0..3) of window r:
// an exchange between neighbouring rows of 16 lanes, then between the two
// halves of the wavefront (min and max are symmetric, so every lane ends
// with the reduction over all four).
__device__ __forceinline__ void window_minmax(float& lo, float& hi) {
  auto a = __builtin_amdgcn_permlane16_swap(__float_as_uint(lo), __float_as_uint(lo), false, false);
  auto b = __builtin_amdgcn_permlane16_swap(__float_as_uint(hi), __float_as_uint(hi), false, false);
  lo = fmin2(__uint_as_float(a[0]), __uint_as_float(a[1]));
  hi = fmax2(__uint_as_float(b[0]), __uint_as_float(b[1]));
  a = __builtin_amdgcn_permlane32_swap(__float_as_uint(lo), __float_as_uint(lo), false, false);
  b = __builtin_amdgcn_permlane32_swap(__float_as_uint(hi), __float_as_uint(hi), false, false);
  lo = fmin2(__uint_as_float(a[0]), __uint_as_float(a[1]));
  hi = fmax2(__uint_as_float(b[0]), __uint_as_float(b[1]));
}

// Element offset of point (i, j) from the patch's first storage element
// (BLK: 8x4-blocked storage, else row-major).
template <bool BLK>
__device__ __forceinline__ unsigned poff(const PatchDev& P, int i, int j) {
  return BLK ? ((__umul24((unsigned)(j >> 2), (unsigned)P.nb1) + (unsigned)(i >> 3)) << 5) +
                   (unsigned)(((j & 3) << 3) + (i & 7))
             : (unsigned)(j * P.n1 + i);
}

// base[o] as the uniform base plus a 32-bit byte offset
__device__ __forceinline__ float ld_off(const float* __restrict__ base, unsigned o) {
  return *(const float*)((const char*)base + (o << 2));
}

// This lane's samples t = g + 4 s (s = 0..3) of the 16-sample window at
// offsets -8..7 (clamped) along a line, rescaled to [-1, 1] with the min and
// max of the whole window.  `base`: the patch's first storage element.
// `edge` (uniform over the wavefront): some window of the wavefront reaches
// past an end of its line; otherwise no sample needs clamping and the four
// are read at fixed distances.
template <int DIR, bool BLK>
__device__ __forceinline__ void window4(const float* __restrict__ base, const PatchDev& P, int i, int j, int g,
                                        bool edge, float x[4]) {
#pragma clang fp contract(off)
  const int pos = DIR == 1 ? i : j, n = DIR == 1 ? P.n1 : P.n2;
  if (edge) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      int k = pos - 8 + g + 4 * s;
      k = k < 0 ? 0 : (k > n - 1 ? n - 1 : k);
      x[s] = ld_off(base, DIR == 1 ? poff<BLK>(P, k, j) : poff<BLK>(P, i, k));
    }
  } else if (DIR == 1) {
    // along q1, samples k and k + 8 lie one block (blocked) or 8 apart
    const int k0 = pos - 8 + g;
    const unsigned o0 = poff<BLK>(P, k0, j), o1 = poff<BLK>(P, k0 + 4, j);
    x[0] = ld_off(base, o0);
    x[1] = ld_off(base, o1);
    x[2] = ld_off(base, o0 + (BLK ? 32u : 8u));
    x[3] = ld_off(base, o1 + (BLK ? 32u : 8u));
  } else {
    // along q2, samples k and k + 4 lie one block row (blocked) or 4 rows apart
    const unsigned o0 = poff<BLK>(P, i, pos - 8 + g);
    const unsigned st = BLK ? (unsigned)P.nb1 << 5 : 4u * (unsigned)P.n1;
#pragma unroll
    for (int s = 0; s < 4; ++s) x[s] = ld_off(base, o0 + s * st);
  }
  float lo = fmin2(fmin3(x[0], x[1], x[2]), x[3]);
  float hi = fmax2(fmax3(x[0], x[1], x[2]), x[3]);
  window_minmax(lo, hi);
  const float rng = hi - lo;
  if (rng <= 1e-6f * fmaxf(1.0f, fabsf(hi))) {
#pragma unroll
    for (int s = 0; s < 4; ++s) x[s] = 0.f;
  } else {
    const float sc = 2.0f * __builtin_amdgcn_rcpf(rng);
#pragma unroll
    for (int s = 0; s < 4; ++s) x[s] = (x[s] - lo) * sc - 1.0f;
  }
}

__device__ __forceinline__ int argmax4(floatx4 o) {
  int best = 0;
  float bv = o[0];
  if (o[1] > bv) { best = 1; bv = o[1]; }
  if (o[2] > bv) { best = 2; bv = o[2]; }
  if (o[3] > bv) { best = 3; bv = o[3]; }
  return best;
}

// Largest magnitude that the split operands take, bounded from the weights:
// the weights themselves and every hidden activation, with the features in
// [-1, 1] (|h1_j| <= |b1_j| + sum_k |W1_kj|, |h2_m| <= |b2_m| +
// sum_j |W2_jm| |h1_j|).  Run by one workgroup; at or above kHalfSafe the
// fp16 high parts could overflow, and bit 1 of *err is set.
constexpr float kHalfSafe = 65000.0f;
__device__ void sdnn_range_check(const MlpPtr& w, unsigned* err) {
  __shared__ float B1[64];
  __shared__ int bad;
  const int t = threadIdx.x;
  if (t == 0) bad = 0;
  if (t < 64) {
    float s = fabsf(w.b1[t]), m = 0.f;
    for (int k = 0; k < 16; ++k) {
      s += fabsf(w.W1[k * 64 + t]);
      m = fmaxf(m, fabsf(w.W1[k * 64 + t]));
    }
    B1[t] = s;
    if (!(fmaxf(m, s) < kHalfSafe)) bad = 1;
  }
  __syncthreads();
  if (t < 64) {
    float s = fabsf(w.b2[t]), m = 0.f;
    for (int k = 0; k < 64; ++k) {
      s += fabsf(w.W2[k * 64 + t]) * B1[k];
      m = fmaxf(m, fabsf(w.W2[k * 64 + t]));
    }
    for (int n = 0; n < 4; ++n) m = fmaxf(m, fabsf(w.W3[t * 4 + n]));
    if (!(fmaxf(m, s) < kHalfSafe)) bad = 1;
  }
  __syncthreads();
  if (t == 0 && bad) atomicOr(err, 2u);
}

// The points of one chunk, 16 consecutive storage elements per wavefront
// at a time (BLK: the patch's storage layout).
template <bool BLK>
__device__ __forceinline__ void sdnn_chunk(const MlpLds& L, const ChunkDev ck, const PatchDev& P,
                                           const float* __restrict__ phi, signed char* tau, float* logits,
                                           long long pl, int wv, int g, int r) {
  const int np = pstore(P);
  const float* base = phi + P.off;
  for (int q = wv; q < kChunk / 16; q += kBlock / 64) {
    const int k0 = ck.start + 16 * q;  // uniform across the wavefront
    if (k0 >= np) break;
    const int kk = k0 + r;
    int i = 0, j = 0;
    bool valid;
    if (BLK) {
      // chunks start at multiples of 16, so the wavefront's points are one
      // half of an 8x4 block, whose position is uniform
      const int blk = k0 >> 5, bj = blk / P.nb1, bi = blk - bj * P.nb1;
      const int e = (k0 & 16) + r;
      i = (bi << 3) + (e & 7);
      j = (bj << 2) + (e >> 3);
      valid = i < P.n1 && j < P.n2;
    } else {
      valid = kk < np && pdecode(P, kk, i, j);
    }
    // lanes without a point evaluate a valid one (every lane takes part
    // in the matrix products) and write nothing
    i = i < P.n1 ? i : P.n1 - 1;
    j = j < P.n2 ? j : P.n2 - 1;
    const long long gi = P.off + kk;
    // 16 points that all lie outside D~ (the strips next to internal
    // sides) have class 0 and zero logits: the products are skipped
    if (!__any(valid && in_dtilde(P, i, j))) {
      if (g == 0 && valid) {
        tau[gi] = (signed char)0;
        if (logits) {
          *(float4*)&logits[4 * gi] = make_float4(0.f, 0.f, 0.f, 0.f);
          *(float4*)&logits[4 * (pl + gi)] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
      }
      continue;
    }
    float x1[4], x2[4];
    window4<1, BLK>(base, P, i, j, g, __any(i < 8 || i > P.n1 - 8), x1);
    window4<2, BLK>(base, P, i, j, g, __any(j < 8 || j > P.n2 - 8), x2);
    floatx4 o1, o2;
    mlp16x2(L, x1, x2, g, r, o1, o2);
    if (g == 0 && valid) {
      const bool in = in_dtilde(P, i, j);
      const int a1 = argmax4(o1), a2 = argmax4(o2);
      tau[gi] = in ? (signed char)(1 + (a1 < a2 ? a1 : a2)) : (signed char)0;
      if (logits) {
        const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
        *(float4*)&logits[4 * gi] = in ? make_float4(o1[0], o1[1], o1[2], o1[3]) : z;
        *(float4*)&logits[4 * (pl + gi)] = in ? make_float4(o2[0], o2[1], o2[2], o2[3]) : z;
      }
    }
  }
}

// Network classes of every point: tau = 1 + min over the two directions of
// the argmax class (0 outside D~).  Blocks stride over the point chunks;
// each wavefront takes 16 consecutive points of a chunk at a time.  Block 0
// also bounds the split operands' range from the weights (bit 1 of *err).
__global__ void __launch_bounds__(kBlock) k_sdnn(const ChunkDev* __restrict__ chunks, int nchunks,
                                                 const PatchDev* __restrict__ patches, const float* phi, MlpPtr w,
                                                 signed char* tau, float* logits, long long pl, unsigned* err) {
  __shared__ MlpLds L;
  mlp_load(L, w);
  if (blockIdx.x == 0) sdnn_range_check(w, err);
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g = lane >> 4, r = lane & 15;
  for (int cb = blockIdx.x; cb < nchunks; cb += gridDim.x) {
    const ChunkDev ck = chunks[cb];
    const PatchDev P = patches[ck.patch];
    if (P.nb1)
      sdnn_chunk<true>(L, ck, P, phi, tau, logits, pl, wv, g, r);
    else
      sdnn_chunk<false>(L, ck, P, phi, tau, logits, pl, wv, g, r);
  }
}

// ---------------------------------------------------------------- 7x7 max

// max over i-3..i+3 (clamped) with the first maximiser.  The seven samples
// are loaded together at clamped indices (32-bit offsets from the patch's
// first storage element; BLK: 8x4-blocked storage); scanning them in order
// with a strict comparison keeps the first maximiser of the clamped range
// i-3..i+3 (a clamped duplicate repeats an end value at the same index).
template <bool BLK>
__device__ __forceinline__ void rowmax_point(const PatchDev& P, int k, const float* __restrict__ S, float* rmax,
                                             int* rarg) {
  int i, j;
  if (k >= pstore(P) || !pdecode(P, k, i, j)) return;
  const float* base = S + P.off;
  float v[7];
#pragma unroll
  for (int q = 0; q < 7; ++q) v[q] = ld_off(base, poff<BLK>(P, min(max(i + q - 3, 0), P.n1 - 1), j));
  float best = v[0];
  int bi = max(i - 3, 0);
#pragma unroll
  for (int q = 1; q < 7; ++q)
    if (v[q] > best) {
      best = v[q];
      bi = min(i + q - 3, P.n1 - 1);
    }
  (rmax + P.off)[k] = best;
  (rarg + P.off)[k] = bi;
}

__global__ void __launch_bounds__(kBlock) k_rowmax(const ChunkDev* __restrict__ chunks, int nchunks,
                                                   const PatchDev* __restrict__ patches, const float* S, float* rmax,
                                                   int* rarg) {
  for_chunks(chunks, nchunks, [&](const ChunkDev ck) {
    const PatchDev P = patches[ck.patch];
    const int k = ck.start + threadIdx.x;
    if (P.nb1)
      rowmax_point<true>(P, k, S, rmax, rarg);
    else
      rowmax_point<false>(P, k, S, rmax, rarg);
  });
}

// column pass of the 7x7 max and mu^ = R(tau) max S h^ on D~ (0 elsewhere)
template <bool BLK>
__device__ __forceinline__ void muhat_point(const PatchDev& P, int k, const float* __restrict__ rmax,
                                            const int* __restrict__ rarg, const signed char* tau, float* muh,
                                            int* argmax) {
  int i, j;
  if (k >= pstore(P) || !pdecode(P, k, i, j)) return;
  const float* base = rmax + P.off;
  float v[7];
#pragma unroll
  for (int q = 0; q < 7; ++q) v[q] = ld_off(base, poff<BLK>(P, i, min(max(j + q - 3, 0), P.n2 - 1)));
  float best = v[0];
  int bj = max(j - 3, 0);
#pragma unroll
  for (int q = 1; q < 7; ++q)
    if (v[q] > best) {
      best = v[q];
      bj = min(j + q - 3, P.n2 - 1);
    }
  if (argmax) (argmax + P.off)[k] = bj * P.n1 + (rarg + P.off)[poff<BLK>(P, i, bj)];
  float m = 0.f;
  if (in_dtilde(P, i, j)) {
    const int t = (tau + P.off)[k];
    const float R = t == 1 ? 1.5f : (t == 2 ? 1.0f : (t == 3 ? 0.5f : 0.0f));
    m = R * best * P.hhat;
  }
  (muh + P.off)[k] = m;
}

__global__ void __launch_bounds__(kBlock) k_muhat(const ChunkDev* __restrict__ chunks, int nchunks,
                                                  const PatchDev* __restrict__ patches, const float* rmax,
                                                  const int* rarg, const signed char* tau, float* muh,
                                                  int* argmax) {
  for_chunks(chunks, nchunks, [&](const ChunkDev ck) {
    const PatchDev P = patches[ck.patch];
    const int k = ck.start + threadIdx.x;
    if (P.nb1)
      muhat_point<true>(P, k, rmax, rarg, tau, muh, argmax);
    else
      muhat_point<false>(P, k, rmax, rarg, tau, muh, argmax);
  });
}

// ---------------------------------------------------------------- Lambda

__device__ __forceinline__ float win(int k) {
  // cos^2(pi k / 18), |k| <= 8 (values in double, rounded once)
  constexpr float w[9] = {
      (float)(1.0),
      (float)(0.96984631039295421),
      (float)(0.88302222155948906),
      (float)(0.75),
      (float)(0.58682408883346517),
      (float)(0.41317591116653483),
      (float)(0.25),
      (float)(0.11697777844051099),
      (float)(0.030153689607045786)};
  return w[k < 0 ? -k : k];
}

// gather mu^ and the D~ indicator into the lattice.  Independent patches:
// the lattice is the patch itself.  Annulus: cell (G, J) collects every
// patch point with that global index (<= 2 sectors x 2 shells).
__global__ void __launch_bounds__(kBlock) k_lat_gather(const ChunkDev* lchunks, int nchunks, const LatDev* lats,
                                                       const PatchDev* patches, AnnulusDev an,
                                                       const float* muh, float* num, float* den,
                                                       int annulus, int transpose_src) {
  for_chunks(lchunks, nchunks, [&](const ChunkDev ck) {
    const LatDev Lt = lats[ck.patch];
    const int k = ck.start + threadIdx.x;
    if (k >= Lt.W * Lt.H) return;
    const long long cell = Lt.base + k;
    if (!annulus) {
      const PatchDev P = patches[ck.patch];
      const int j = k / P.n1, i = k - j * P.n1;
      const bool in = transpose_src ? true : in_dtilde(P, i, j);
      num[cell] = in ? muh[pidx(P, i, j)] : 0.f;
      if (den) den[cell] = in ? 1.f : 0.f;
      return;
    }
    const int J = k / Lt.W, G = k - J * Lt.W;
    float sn = 0.f, sd = 0.f;
    int k0 = J / an.st2;
    if (k0 > an.nshell - 1) k0 = an.nshell - 1;
    for (int kk = k0 - 1; kk <= k0; ++kk) {
      if (kk < 0) continue;
      const int jj = J - kk * an.st2;
      if (jj < 0 || jj >= an.n2) continue;
      const int s0 = G / an.st1;
      for (int ss = s0 - 1; ss <= s0; ++ss) {
        const int s = (ss + an.nsec) % an.nsec;
        int ii = G - ss * an.st1;
        if (ii < 0 || ii >= an.n1) continue;
        const int p = kk * an.nsec + s;
        const PatchDev P = patches[p];
        if (!transpose_src && !in_dtilde(P, ii, jj)) continue;
        sn += muh[pidx(P, ii, jj)];
        sd += 1.f;
      }
    }
    num[cell] = sn;
    if (den) den[cell] = sd;
  });
}

// Separable 17-tap window sums of a lattice (the smoothing operator's
// numerator and denominator, or the transposed sums), in two passes over
// tiles of 256 columns by kLatRows rows.  Along J (zero padded): a thread
// keeps its column's
// kLatRows + 16 values in registers and forms the kLatRows sums from them
// (two loads per output instead of seventeen), the taps summed in the same
// order, a row outside the lattice read as zero.
constexpr int kLatRows = 16;
struct LatTile {
  int lat, g0, j0, pad;
};

__global__ void __launch_bounds__(kBlock) k_lat_conv_j(const LatTile* __restrict__ tiles, int ntiles,
                                                       const LatDev* __restrict__ lats, const float* in0,
                                                       const float* in1, float* out0, float* out1) {
  for (int tb = blockIdx.x; tb < ntiles; tb += gridDim.x) {
    const LatTile tt = tiles[tb];
    const LatDev Lt = lats[tt.lat];
    const int G = tt.g0 + (int)threadIdx.x;
    if (G >= Lt.W) continue;
    const long long col = Lt.base + G;
    float v0[kLatRows + 16], v1[kLatRows + 16];
#pragma unroll
    for (int q = 0; q < kLatRows + 16; ++q) {
      const int j = tt.j0 - 8 + q;
      const bool ok = j >= 0 && j < Lt.H;
      v0[q] = ok ? in0[col + (long long)j * Lt.W] : 0.f;
      v1[q] = (ok && in1) ? in1[col + (long long)j * Lt.W] : 0.f;
    }
#pragma unroll
    for (int r = 0; r < kLatRows; ++r) {
      const int J = tt.j0 + r;
      if (J >= Lt.H) break;
      float s0 = 0.f, s1 = 0.f;
#pragma unroll
      for (int l = -8; l <= 8; ++l) {
        const int jj = J + l;
        if (jj < 0 || jj >= Lt.H) continue;
        s0 = fmaf(win(l), v0[r + 8 + l], s0);
        if (in1) s1 = fmaf(win(l), v1[r + 8 + l], s1);
      }
      out0[col + (long long)J * Lt.W] = s0;
      if (out1) out1[col + (long long)J * Lt.W] = s1;
    }
  }
}

// Along G (periodic or zero padded), the same tiles: the tile's kLatRows
// row segments and their 8-cell halos (wrapped on a periodic
// lattice, zero outside a plain one) are staged in LDS, then each thread
// forms the sums of its column, taps in the same order.
__global__ void __launch_bounds__(kBlock) k_lat_conv_g(const LatTile* __restrict__ tiles, int ntiles,
                                                       const LatDev* __restrict__ lats, const float* in0,
                                                       const float* in1, float* out0, float* out1) {
  constexpr int kW = kBlock + 16;
  __shared__ float s0[kLatRows][kW], s1[kLatRows][kW];
  for (int tb = blockIdx.x; tb < ntiles; tb += gridDim.x) {
    const LatTile tt = tiles[tb];
    const LatDev Lt = lats[tt.lat];
    // every thread's share of the staging loads is issued before any of them
    // is written to LDS (kLatRows * kW is kStage workgroups' worth exactly)
    constexpr int kStage = kLatRows * kW / kBlock;
    static_assert(kStage * kBlock == kLatRows * kW, "staging covers the tile exactly");
    float a[kStage], b[kStage];
#pragma unroll
    for (int it = 0; it < kStage; ++it) {
      const int q = it * kBlock + (int)threadIdx.x;
      const int r = q / kW, c = q - r * kW;
      const int J = tt.j0 + r;
      int g = tt.g0 - 8 + c;
      bool ok = J < Lt.H;
      if (Lt.periodic) {
        g = g < 0 ? g + Lt.W : (g >= Lt.W ? g - Lt.W : g);   // |offset| <= 8 < W
      } else {
        ok = ok && g >= 0 && g < Lt.W;
      }
      const long long cell = Lt.base + (long long)J * Lt.W + g;
      a[it] = ok ? in0[cell] : 0.f;
      b[it] = (ok && in1) ? in1[cell] : 0.f;
    }
#pragma unroll
    for (int it = 0; it < kStage; ++it) {
      const int q = it * kBlock + (int)threadIdx.x;
      const int r = q / kW, c = q - r * kW;
      s0[r][c] = a[it];
      if (in1) s1[r][c] = b[it];
    }
    __syncthreads();
    const int G = tt.g0 + (int)threadIdx.x;
    if (G < Lt.W) {
      for (int r = 0; r < kLatRows; ++r) {
        const int J = tt.j0 + r;
        if (J >= Lt.H) break;
        float a0 = 0.f, a1 = 0.f;
#pragma unroll
        for (int l = -8; l <= 8; ++l) {
          a0 = fmaf(win(l), s0[r][threadIdx.x + 8 + l], a0);
          if (in1) a1 = fmaf(win(l), s1[r][threadIdx.x + 8 + l], a1);
        }
        const long long cell = Lt.base + (long long)J * Lt.W + G;
        out0[cell] = a0;
        if (out1) out1[cell] = a1;
      }
    }
    __syncthreads();   // the staging rows are reused by the next tile
  }
}

__device__ __forceinline__ long long lat_cell(const PatchDev& P, int p, int i, int j, int annulus,
                                              const AnnulusDev& an) {
  if (!annulus) return P.off + (long long)j * P.n1 + i;  // lattice cells are row-major
  const int s = p % an.nsec, kk = p / an.nsec;
  const int G = (s * an.st1 + i) % an.ring;
  const int J = kk * an.st2 + j;
  return (long long)J * an.ring + G;
}

// mu = num / den at every patch point (mode 0), or the transpose
// gather-scatter of Lambda^T: out = mu_bar / den at every point (mode 1)
__global__ void __launch_bounds__(kBlock) k_lat_scatter(const ChunkDev* chunks, int nchunks, const PatchDev* patches,
                                                        AnnulusDev an, int annulus, const float* num,
                                                        const float* den, float* mu) {
  for_chunks(chunks, nchunks, [&](const ChunkDev ck) {
    const PatchDev P = patches[ck.patch];
    const int k = ck.start + threadIdx.x;
    int i, j;
    if (k >= pstore(P) || !pdecode(P, k, i, j)) return;
    const long long c = lat_cell(P, ck.patch, i, j, annulus, an);
    mu[P.off + k] = num[c] / den[c];
  });
}

// Points of patches that overlap other patches without shared grid lines
// (paper eqs. multipatch_W, zeta, multipatch_W_norm): mu = (num + sum of
// the other patches' num at the nearest grid point of the preimage) / (den +
// the same sum of den).  Targets hold the point's plane index and its own
// lattice cell; src[begin..end) the other patches' cells.
struct OvlTarget {
  long long pt, cell;
  int begin, end;
};

__global__ void __launch_bounds__(kBlock) k_lat_overlap(const OvlTarget* __restrict__ tg, int n,
                                                        const long long* __restrict__ src, const float* num,
                                                        const float* den, float* mu) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const OvlTarget t = tg[k];
  float a = num[t.cell], b = den[t.cell];
  for (int q = t.begin; q < t.end; ++q) {
    a += num[src[q]];
    b += den[src[q]];
  }
  mu[t.pt] = a / b;
}

// Transpose of k_lat_overlap, two steps.  First, at each target point,
// t = mu_bar / (its full denominator) replaces mu_bar / den[own cell];
// after t has been gathered into the lattice, every target's t is also
// added at the other patches' cells it read from.
__global__ void __launch_bounds__(kBlock) k_lat_overlap_div(const OvlTarget* __restrict__ tg, int n,
                                                            const long long* __restrict__ src, const float* mub,
                                                            const float* den, float* t) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const OvlTarget q = tg[k];
  float b = den[q.cell];
  for (int i = q.begin; i < q.end; ++i) b += den[src[i]];
  t[q.pt] = mub[q.pt] / b;
}

__global__ void __launch_bounds__(kBlock) k_lat_overlap_scatter(const OvlTarget* __restrict__ tg, int n,
                                                                const long long* __restrict__ src, const float* t,
                                                                float* acc) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const OvlTarget q = tg[k];
  const float v = t[q.pt];
  for (int i = q.begin; i < q.end; ++i) atomicAdd(acc + src[i], v);
}

// Lambda^T first step: t = mu_bar / den (per patch point, into a plane)
__global__ void __launch_bounds__(kBlock) k_lat_divide_pts(const ChunkDev* chunks, int nchunks, const PatchDev* patches,
                                                           AnnulusDev an, int annulus, const float* mub,
                                                           const float* den, float* t) {
  for_chunks(chunks, nchunks, [&](const ChunkDev ck) {
    const PatchDev P = patches[ck.patch];
    const int k = ck.start + threadIdx.x;
    int i, j;
    if (k >= pstore(P) || !pdecode(P, k, i, j)) return;
    const long long c = lat_cell(P, ck.patch, i, j, annulus, an);
    t[P.off + k] = mub[P.off + k] / den[c];
  });
}

// Lambda^T last step + mu^ -> S routing: sbar(x) = sum over points y in
// the 7x7 neighbourhood of x whose maximiser is x of R(tau_y) h^ mu^bar(y),
// with mu^bar(y) = conv(acc)(cell of y) on D~.
__global__ void __launch_bounds__(kBlock) k_route_S(const ChunkDev* chunks, int nchunks, const PatchDev* patches,
                                                    AnnulusDev an, int annulus, const float* accconv,
                                                    const signed char* tau, const int* argmax,
                                                    float* sbar) {
  for_chunks(chunks, nchunks, [&](const ChunkDev ck) {
    const PatchDev P = patches[ck.patch];
    const int k = ck.start + threadIdx.x;
    int i, j;
    if (k >= pstore(P) || !pdecode(P, k, i, j)) return;
    const int kr = j * P.n1 + i;  // patch-local row-major index, as argmax stores it
    float s = 0.f;
    for (int dj = -3; dj <= 3; ++dj) {
      const int yj = j + dj;
      if (yj < 0 || yj >= P.n2) continue;
      for (int di = -3; di <= 3; ++di) {
        const int yi = i + di;
        if (yi < 0 || yi >= P.n1) continue;
        const long long gy = pidx(P, yi, yj);
        if (argmax[gy] != kr || !in_dtilde(P, yi, yj)) continue;
        const int t = tau[gy];
        const float R = t == 1 ? 1.5f : (t == 2 ? 1.0f : (t == 3 ? 0.5f : 0.0f));
        s += R * P.hhat * accconv[lat_cell(P, ck.patch, yi, yj, annulus, an)];
      }
    }
    sbar[P.off + k] = s;
  });
}

// u_bar += (dS/du)^T sbar, S = |u| + |v| + sqrt(gamma p / rho)
__global__ void __launch_bounds__(kBlock) k_speed_vjp(const ChunkDev* chunks, int nchunks, const PatchDev* patches,
                                                      const float* u, long long pl, float gam,
                                                      const float* sbar, float* ub) {
  for_chunks(chunks, nchunks, [&](const ChunkDev ck) {
    const PatchDev P = patches[ck.patch];
    const int k = ck.start + threadIdx.x;
    int i, j;
    if (k >= pstore(P) || !pdecode(P, k, i, j)) return;
    const long long g = P.off + k;
    const float sb = sbar[g];
    if (sb == 0.f) return;
    float rho, vx, vy, p;
    prim(u, pl, g, gam, rho, vx, vy, p);
    const float ir = 1.0f / rho;
    const float a = sqrtf(gam * p / rho);
    const float su = vx > 0.f ? 1.f : (vx < 0.f ? -1.f : 0.f);
    const float sv = vy > 0.f ? 1.f : (vy < 0.f ? -1.f : 0.f);
    // da/dp = gamma/(2 a rho), da/drho|_p = -a/(2 rho)
    const float ap = gam / (2.f * a * rho) * sb;
    const float g1 = gam - 1.f;
    ub[g] += sb * (-(su * vx + sv * vy) * ir - a * 0.5f * ir) + ap * g1 * 0.5f * (vx * vx + vy * vy);
    ub[pl + g] += sb * su * ir - ap * g1 * vx;
    ub[2 * pl + g] += sb * sv * ir - ap * g1 * vy;
    ub[3 * pl + g] += ap * g1;
  });
}

// ---------------------------------------------------------------- state monitor

// flags |= 1 for a non-finite component, 2 for rho <= 0, 4 for p <= 0 at a
// grid point of a patch (padding is not looked at); one OR per block.
__global__ void __launch_bounds__(kBlock) k_check(const ChunkDev* chunks, int nchunks, const PatchDev* patches,
                                                  const float* u, long long pl, float gam, int* flags) {
  __shared__ int red[kBlock / 64];
  int f = 0;
  for (int cb = blockIdx.x; cb < nchunks; cb += gridDim.x) {
    const ChunkDev ck = chunks[cb];
    const PatchDev P = patches[ck.patch];
    const int k = ck.start + threadIdx.x;
    int i, j;
    if (k < pstore(P) && pdecode(P, k, i, j)) {
      const long long g = P.off + k;
      const float e0 = u[g], e1 = u[pl + g], e2 = u[2 * pl + g], e3 = u[3 * pl + g];
      if (!(isfinite(e0) && isfinite(e1) && isfinite(e2) && isfinite(e3))) f |= 1;
      if (!(e0 > 0.f)) f |= 2;
      const float p = (gam - 1.0f) * (e3 - 0.5f * (e1 * e1 + e2 * e2) / e0);
      if (!(p > 0.f)) f |= 4;
    }
  }
  for (int o = 32; o > 0; o >>= 1) f |= __shfl_xor(f, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = f;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBlock / 64; ++w) f |= red[w];
    if (f) atomicOr(flags, f);
  }
}

// ---------------------------------------------------------------- step size

__global__ void __launch_bounds__(kBlock) k_fill(float* p, float v, long long n) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) p[g] = v;
}

__global__ void __launch_bounds__(kBlock) k_dt_reduce(const ChunkDev* chunks, int nchunks, const PatchDev* patches,
                                                      const float* u, const float* mu, long long pl,
                                                      float gam, unsigned* smax, unsigned* mmax) {
  // a block takes a contiguous run of chunks (chunks are ordered by patch)
  // and keeps per-thread maxima until the patch changes (the same chunk for
  // every thread of the block): the block's maxima are posted only then and
  // at the end, one thread per block, and only where they exceed the value
  // already there (posted maxima only grow, so a stale read costs an atomic
  // at most and never loses one).  Few large patches thus do not serialise
  // thousands of atomics on one address; the chunk loop has no barrier.
  __shared__ float red_s[kBlock / 64], red_m[kBlock / 64];
  const int per = (nchunks + (int)gridDim.x - 1) / (int)gridDim.x;
  const int c0 = (int)blockIdx.x * per, c1 = min(c0 + per, nchunks);
  auto post = [&](int patch, float s, float m) {
    for (int o = 32; o > 0; o >>= 1) {
      s = fmaxf(s, __shfl_xor(s, o));
      m = fmaxf(m, __shfl_xor(m, o));
    }
    if ((threadIdx.x & 63) == 0) {
      red_s[threadIdx.x >> 6] = s;
      red_m[threadIdx.x >> 6] = m;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int w = 1; w < kBlock / 64; ++w) {
        s = fmaxf(s, red_s[w]);
        m = fmaxf(m, red_m[w]);
      }
      // non-negative floats order like their bit patterns
      const unsigned sb = __float_as_uint(fmaxf(s, 0.f)), mb = __float_as_uint(fmaxf(m, 0.f));
      if (sb > smax[patch]) atomicMax(smax + patch, sb);
      if (mb > mmax[patch]) atomicMax(mmax + patch, mb);
    }
    __syncthreads();
  };
  if (c0 >= c1) return;
  int cur = chunks[c0].patch;
  float s = 0.f, m = 0.f;
  for (int c = c0; c < c1; ++c) {
    const ChunkDev ck = chunks[c];
    if (ck.patch != cur) {  // the same for every thread of the block
      post(cur, s, m);
      s = m = 0.f;
      cur = ck.patch;
    }
    const PatchDev P = patches[ck.patch];
    const int k = ck.start + threadIdx.x;
    int i, j;
    if (k < pstore(P) && pdecode(P, k, i, j)) {
      const long long g = P.off + k;
      float rho, vx, vy, p;
      prim(u, pl, g, gam, rho, vx, vy, p);
      s = fmaxf(s, fabsf(vx) + fabsf(vy) + sqrtf(gam * p / rho));
      if (mu) m = fmaxf(m, mu[g]);
    }
  }
  post(cur, s, m);
}

__global__ void __launch_bounds__(kBlock) k_dt_final(const PatchDev* patches, int np, const unsigned* smax,
                                                     const unsigned* mmax, float cfl, float* dt) {
  __shared__ float red[kBlock / 64];
  float best = 3.4e38f;
  for (int p = threadIdx.x; p < np; p += blockDim.x) {
    const double h = patches[p].htilde;
    const double den = (double)__uint_as_float(smax[p]) / h + (double)__uint_as_float(mmax[p]) / (h * h);
    best = fminf(best, (float)(cfl / den));
  }
  for (int o = 32; o > 0; o >>= 1) best = fminf(best, __shfl_xor(best, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) best = fminf(best, red[w]);
    dt[0] = (float)((double)best / 3.14159265358979323846);
  }
}

// ---------------------------------------------------------------- glue

// sector pass: receivers i < 5 (from the left neighbour's column i + st1) and
// i >= n1 - 5 (from the right neighbour's column i - st1), all rows, 4 fields
__global__ void __launch_bounds__(kBlock) k_glue_sectors(const PatchDev* patches, AnnulusDev an, float* u,
                                                         long long pl) {
  const long long per = (long long)an.n2 * 2 * kNf;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long total = per * an.nsec * an.nshell;
  if (t >= total) return;
  const int p = (int)(t / per);
  long long r = t - (long long)p * per;
  const int j = (int)(r / (2 * kNf));
  const int q = (int)(r - (long long)j * 2 * kNf);
  const int s = p % an.nsec, kk = p / an.nsec;
  int i, src, si;
  if (q < kNf) {
    i = q;
    src = kk * an.nsec + (s - 1 + an.nsec) % an.nsec;
    si = i + an.st1;
  } else {
    i = an.n1 - 2 * kNf + q;
    src = kk * an.nsec + (s + 1) % an.nsec;
    si = i - an.st1;
  }
  const long long d = pidx(patches[p], i, j);
  const long long sg = pidx(patches[src], si, j);
  for (int f = 0; f < 4; ++f) u[f * pl + d] = u[f * pl + sg];
}

__global__ void __launch_bounds__(kBlock) k_glue_shells(const PatchDev* patches, AnnulusDev an, float* u,
                                                        long long pl) {
  const long long per = (long long)an.n1 * 2 * kNf;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long total = per * an.nsec * an.nshell;
  if (t >= total) return;
  const int p = (int)(t / per);
  long long r = t - (long long)p * per;
  const int q = (int)(r / an.n1);
  const int i = (int)(r - (long long)q * an.n1);
  const int s = p % an.nsec, kk = p / an.nsec;
  int j, src, sj;
  if (q < kNf) {
    if (kk == 0) return;
    j = q;
    src = (kk - 1) * an.nsec + s;
    sj = j + an.st2;
  } else {
    if (kk == an.nshell - 1) return;
    j = an.n2 - 2 * kNf + q;
    src = (kk + 1) * an.nsec + s;
    sj = j - an.st2;
  }
  const long long d = pidx(patches[p], i, j);
  const long long sg = pidx(patches[src], i, sj);
  for (int f = 0; f < 4; ++f) u[f * pl + d] = u[f * pl + sg];
}

__global__ void __launch_bounds__(kBlock) k_dirichlet(const unsigned char* mask, float* u, long long pl,
                                                      float s0, float s1, float s2, float s3) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= pl || !mask[g]) return;
  u[g] = s0;
  u[pl + g] = s1;
  u[2 * pl + g] = s2;
  u[3 * pl + g] = s3;
}

// ---------------------------------------------------------------- glue reverse mode
//
// Transpose of the fringe copies: every receiver's cotangent moves onto its
// donor (donors are never receivers within a pass and have one receiver
// each, so the updates do not race); run in the reverse order of the
// forward (Dirichlet, shells, sectors).

__global__ void __launch_bounds__(kBlock) k_glue_sectors_adj(const PatchDev* patches, AnnulusDev an, float* ub,
                                                             long long pl) {
  const long long per = (long long)an.n2 * 2 * kNf;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long total = per * an.nsec * an.nshell;
  if (t >= total) return;
  const int p = (int)(t / per);
  long long r = t - (long long)p * per;
  const int j = (int)(r / (2 * kNf));
  const int q = (int)(r - (long long)j * 2 * kNf);
  const int s = p % an.nsec, kk = p / an.nsec;
  int i, src, si;
  if (q < kNf) {
    i = q;
    src = kk * an.nsec + (s - 1 + an.nsec) % an.nsec;
    si = i + an.st1;
  } else {
    i = an.n1 - 2 * kNf + q;
    src = kk * an.nsec + (s + 1) % an.nsec;
    si = i - an.st1;
  }
  const long long d = pidx(patches[p], i, j);
  const long long sg = pidx(patches[src], si, j);
  for (int f = 0; f < 4; ++f) {
    ub[f * pl + sg] += ub[f * pl + d];
    ub[f * pl + d] = 0.f;
  }
}

__global__ void __launch_bounds__(kBlock) k_glue_shells_adj(const PatchDev* patches, AnnulusDev an, float* ub,
                                                            long long pl) {
  const long long per = (long long)an.n1 * 2 * kNf;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long total = per * an.nsec * an.nshell;
  if (t >= total) return;
  const int p = (int)(t / per);
  long long r = t - (long long)p * per;
  const int q = (int)(r / an.n1);
  const int i = (int)(r - (long long)q * an.n1);
  const int s = p % an.nsec, kk = p / an.nsec;
  int j, src, sj;
  if (q < kNf) {
    if (kk == 0) return;
    j = q;
    src = (kk - 1) * an.nsec + s;
    sj = j + an.st2;
  } else {
    if (kk == an.nshell - 1) return;
    j = an.n2 - 2 * kNf + q;
    src = (kk + 1) * an.nsec + s;
    sj = j - an.st2;
  }
  const long long d = pidx(patches[p], i, j);
  const long long sg = pidx(patches[src], i, sj);
  for (int f = 0; f < 4; ++f) {
    ub[f * pl + sg] += ub[f * pl + d];
    ub[f * pl + d] = 0.f;
  }
}

// Dirichlet transpose: dparam += sum over flagged points of ub . dstate,
// then ub = 0 there.  Wavefront shuffles reduce each block to one FP64
// atomic add.
__global__ void __launch_bounds__(kBlock) k_dirichlet_adj(const unsigned char* mask, float* ub, long long pl,
                                                          float d0, float d1, float d2, float d3, double* dparam) {
  __shared__ double part[kBlock / 64];
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double v = 0.0;
  if (g < pl && mask[g]) {
    v = (double)ub[g] * d0 + (double)ub[pl + g] * d1 + (double)ub[2 * pl + g] * d2 + (double)ub[3 * pl + g] * d3;
    ub[g] = 0.f;
    ub[pl + g] = 0.f;
    ub[2 * pl + g] = 0.f;
    ub[3 * pl + g] = 0.f;
  }
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < kBlock / 64; ++k) t += part[k];
    if (t != 0.0) atomicAdd(dparam, t);
  }
}

// ub[k] += alpha ubar (k < n), used by the step reverse mode
__global__ void __launch_bounds__(kBlock) k_axpy(float alpha, const float* x, float* y, long long n) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) y[g] += alpha * x[g];
}

// ---------------------------------------------------------------- RHS reverse mode

// (dF/de)^T fb + (dG/de)^T gb at one point (primitive chain rule)
__device__ __forceinline__ void flux_vjp(const float e[4], float gam, const float fb[4], const float gb[4],
                                         float out[4]) {
  const float rho = e[0], ir = 1.0f / rho;
  const float u = e[1] * ir, v = e[2] * ir;
  const float g1 = gam - 1.0f;
  const float p = g1 * (e[3] - 0.5f * rho * (u * u + v * v));
  const float Hh = e[3] + p;
  const float Pb = fb[1] + gb[2] + fb[3] * u + gb[3] * v;
  const float Ub = fb[1] * e[1] + fb[3] * Hh + gb[1] * e[2];
  const float Vb = fb[2] * e[1] + gb[2] * e[2] + gb[3] * Hh;
  const float Mb = fb[0] + fb[1] * u + fb[2] * v;
  const float Nb = gb[0] + gb[1] * u + gb[2] * v;
  const float Eb = fb[3] * u + gb[3] * v;
  out[0] = -(Ub * u + Vb * v) * ir + Pb * g1 * 0.5f * (u * u + v * v);
  out[1] = Mb + Ub * ir - Pb * g1 * u;
  out[2] = Nb + Vb * ir - Pb * g1 * v;
  out[3] = Eb + Pb * g1;
}

// Reverse of pass C: Hb = D_1^T (m_1x rb, m_1y rb) for every state
// component (q1 lines).  The reverse of pass B2, which also finishes H_bar
// and applies the pointwise reverse of H = mu grad e - f', is k_adjHb2p.
__global__ void FCSD_LINE_BOUNDS k_adjHb1(PassArgs a, const float* rb, float* Hb) {
  FCSD_TILE_BEGIN(a)
  const TileMem M = tile_mem<1>(P, T, nl, ld);
  const long long pl = a.plane, bo = M.base;
  const float* mdx = a.metric + bo;
  const float* mdy = a.metric + pl + bo;
  // loads of the element loops are batched (walk_b): one element's loads
  // waited for before the next element's were issued made this kernel
  // latency-bound
  for (int comp = 0; comp < 4; ++comp) {
    const float* rbc = rb + comp * pl + bo;
    walk_b<kLoadBatch>(
        M.w, [&](unsigned g) { return make_float4(at(rbc, g), at(mdx, g), at(mdy, g), 0.f); },
        [&](unsigned, unsigned l, float4 v) { at(z, l) = make_float2(v.y * v.x, v.z * v.x); });
    __syncthreads();
    line_derivative<true>(X, Pg, P, a.gq, a.dq, a.d);
    float* hbx = Hb + (2 * comp) * pl + bo;
    float* hby = Hb + (2 * comp + 1) * pl + bo;
    walk(M.w, [&](unsigned g, unsigned l) {
      const float2 v = at(z, l);
      at(hbx, g) = v.x;
      at(hby, g) = v.y;
    });
    __syncthreads();
  }
}

// Reverse of pass B2 with two state components per transform (H_bar x,y of
// component c at z[pos][l], of c + 1 at z[pos][nl + l]; tiles of the set
// with two complex lines per grid line): the metric rows, mu and mu_bar are
// read and written once per component pair instead of once per component,
// which is what bounds this reverse pass (HBM traffic).  Hb (+)= D_2^T
// (m_2x rb, m_2y rb), then G1/G2 = mu-weighted metric products (for D^T
// later), mu_bar += H_bar . grad e, u_bar += flux VJP of -H_bar.
template <bool VISC>
__global__ void FCSD_LINE_BOUNDS k_adjHb2p(PassArgs a, const float* rb, float* Hb, const float* d1e,
                                            const float* d2e, float* G1, float* G2, float* mub, float* ub) {
  const TileDev T = a.tiles[blockIdx.x];
  if (T.nl == 0) return;
  const PlanDev P = a.plans[T.plan];
  const PlanDev* Pg = a.plans + T.plan;
  TileDev T2 = T;
  T2.nl = 2 * T.nl;
  const LineCtx X = line_setup(lds_z, T2, P, a.tw, a.km);
  float2* __restrict__ z = X.z;
  const int nl = T.nl, ld = T.ld;
  __syncthreads();
  const TileMem M = tile_mem<2>(P, T, nl, ld);
  const long long pl = a.plane, bo = M.base;
  const float* m1x = a.metric + bo;
  const float* m1y = a.metric + pl + bo;
  const float* m2x = a.metric + 2 * pl + bo;
  const float* m2y = a.metric + 3 * pl + bo;
  float2* __restrict__ zb = z + nl;
  for (int comp = 0; comp < 4; comp += 2) {
    const float* rb0 = rb + comp * pl + bo;
    const float* rb1 = rb0 + pl;
    struct RIn {
      float r0, r1, mx, my;
    };
    walk_b<kEpiBatch>(
        M.w, [&](unsigned g) { return RIn{at(rb0, g), at(rb1, g), at(m2x, g), at(m2y, g)}; },
        [&](unsigned, unsigned l, const RIn& q) {
          at(z, l) = make_float2(q.mx * q.r0, q.my * q.r0);
          at(zb, l) = make_float2(q.mx * q.r1, q.my * q.r1);
        });
    __syncthreads();
    line_derivative<true>(X, Pg, P, a.gq, a.dq, a.d);
    float* hb0 = Hb + (2 * comp) * pl + bo;   // x, y of comp; then of comp + 1
    const long long fo = comp * pl + bo;
    if (!VISC) {
      walk_b<4>(
          M.w, [&](unsigned g) { return make_float4(at(hb0, g), at(hb0 + pl, g), at(hb0 + 2 * pl, g), at(hb0 + 3 * pl, g)); },
          [&](unsigned g, unsigned l, float4 h) {
            const float2 v = at(z, l), w = at(zb, l);
            at(hb0, g) = h.x + v.x;
            at(hb0 + pl, g) = h.y + v.y;
            at(hb0 + 2 * pl, g) = h.z + w.x;
            at(hb0 + 3 * pl, g) = h.w + w.y;
          });
    } else {
      struct VIn2 {
        float h[4], m1x, m1y, m2x, m2y, mu, d1[2], d2[2], mb;
      };
      float* mubp = mub ? mub + bo : nullptr;
      walk_b<kEpiBatchH>(
          M.w,
          [&](unsigned g) {
            VIn2 q;
#pragma unroll
            for (int k = 0; k < 4; ++k) q.h[k] = at(hb0 + k * pl, g);
            q.m1x = at(m1x, g);
            q.m1y = at(m1y, g);
            q.m2x = at(m2x, g);
            q.m2y = at(m2y, g);
            q.mu = at(a.mu + bo, g);
#pragma unroll
            for (int k = 0; k < 2; ++k) {
              q.d1[k] = mubp ? at(d1e + fo + k * pl, g) : 0.f;
              q.d2[k] = mubp ? at(d2e + fo + k * pl, g) : 0.f;
            }
            q.mb = mubp ? at(mubp, g) : 0.f;
            return q;
          },
          [&](unsigned g, unsigned l, const VIn2& q) {
            const float2 v0 = at(z, l), v1 = at(zb, l);
            const float hx[2] = {q.h[0] + v0.x, q.h[2] + v1.x}, hy[2] = {q.h[1] + v0.y, q.h[3] + v1.y};
            float mb = q.mb;
#pragma unroll
            for (int k = 0; k < 2; ++k) {
              at(hb0 + (2 * k) * pl, g) = hx[k];
              at(hb0 + (2 * k + 1) * pl, g) = hy[k];
              at(G1 + fo + k * pl, g) = q.mu * (q.m1x * hx[k] + q.m1y * hy[k]);
              at(G2 + fo + k * pl, g) = q.mu * (q.m2x * hx[k] + q.m2y * hy[k]);
              const float ex = q.m1x * q.d1[k] + q.m2x * q.d2[k];
              const float ey = q.m1y * q.d1[k] + q.m2y * q.d2[k];
              mb = mb + hx[k] * ex + hy[k] * ey;
            }
            if (mubp) at(mubp, g) = mb;
          });
    }
    __syncthreads();
  }
  if (a.mode != FLUX_VISC) {
    struct FIn {
      float e[4], fb[4], gb[4], ub[4];
    };
    walk_b<2>(
        M.w,
        [&](unsigned g) {
          FIn q;
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            q.e[k] = at(a.u + k * pl + bo, g);
            q.fb[k] = at(Hb + (2 * k) * pl + bo, g);
            q.gb[k] = at(Hb + (2 * k + 1) * pl + bo, g);
            q.ub[k] = at(ub + k * pl + bo, g);
          }
          return q;
        },
        [&](unsigned g, unsigned, const FIn& q) {
          float fb[4], gb[4], o[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            fb[k] = -q.fb[k];
            gb[k] = -q.gb[k];
          }
          flux_vjp(q.e, a.gamma, fb, gb, o);
#pragma unroll
          for (int k = 0; k < 4; ++k) at(ub + k * pl + bo, g) = q.ub[k] + o[k];
        });
  }
}

// The viscous reverse of pass B2 on q2 tiles that hold all four state
// components (tile set of four complex lines per grid line), fused with the
// transposed q2 derivative of G2: one transform gives Hb = Hb1 + D_2^T
// (m_2x rb, m_2y rb) of the four components; at every point the epilogue
// forms G1 (stored for the q1 transpose), G2 (kept in LDS as two complex
// lines per grid line), mu_bar and, unless mode is FLUX_VISC, the flux VJP
// of -Hb into u_bar, so that Hb itself is never stored; then u_bar +=
// D_2^T G2.  The same FP32 operations as k_adjHb2p followed by fc_diff_adj
// of G2 along q2, up to the order of the tail folds' sums (fold_pre splits
// a line over a number of lanes that depends on the tile's line count).
__global__ void FCSD_LINE_BOUNDS k_adjHb2w(PassArgs a, const float* rb, const float* Hb, const float* d1e,
                                          const float* d2e, float* G1, float* mub, float* ub) {
  const TileDev T = a.tiles[blockIdx.x];
  if (T.nl == 0) return;
  const PlanDev P = a.plans[T.plan];
  const PlanDev* Pg = a.plans + T.plan;
  TileDev T4 = T;
  T4.nl = 4 * T.nl;
  const LineCtx X4 = line_setup(lds_z, T4, P, a.tw, a.km);
  const LineCtx X2 = line_view(X4, 2 * T.nl);
  float2* __restrict__ z = X4.z;
  const int nl = T.nl, ld = T.ld;
  __syncthreads();
  const TileMem M = tile_mem<2>(P, T, nl, ld);
  const long long pl = a.plane, bo = M.base;
  const float* m1x = a.metric + bo;
  const float* m1y = a.metric + pl + bo;
  const float* m2x = a.metric + 2 * pl + bo;
  const float* m2y = a.metric + 3 * pl + bo;
  float2* __restrict__ z1 = z + nl;
  float2* __restrict__ z2 = z + 2 * nl;
  float2* __restrict__ z3 = z + 3 * nl;
  struct RIn4 {
    float r[4], mx, my;
  };
  walk_b<kEpiBatch>(
      M.w,
      [&](unsigned g) {
        RIn4 q;
#pragma unroll
        for (int k = 0; k < 4; ++k) q.r[k] = at(rb + k * pl + bo, g);
        q.mx = at(m2x, g);
        q.my = at(m2y, g);
        return q;
      },
      [&](unsigned, unsigned l, const RIn4& q) {
        at(z, l) = make_float2(q.mx * q.r[0], q.my * q.r[0]);
        at(z1, l) = make_float2(q.mx * q.r[1], q.my * q.r[1]);
        at(z2, l) = make_float2(q.mx * q.r[2], q.my * q.r[2]);
        at(z3, l) = make_float2(q.mx * q.r[3], q.my * q.r[3]);
      });
  __syncthreads();
  line_derivative<true>(X4, Pg, P, a.gq, a.dq, a.d);
  const bool flux = a.mode != FLUX_VISC;
  float* mubp = mub ? mub + bo : nullptr;
  struct VIn4 {
    float h[8], m1x, m1y, m2x, m2y, mu, d1[4], d2[4], mb, e[4], u[4];
  };
  walk_b<2>(
      M.w,
      [&](unsigned g) {
        VIn4 q;
#pragma unroll
        for (int k = 0; k < 8; ++k) q.h[k] = at(Hb + k * pl + bo, g);
        q.m1x = at(m1x, g);
        q.m1y = at(m1y, g);
        q.m2x = at(m2x, g);
        q.m2y = at(m2y, g);
        q.mu = at(a.mu + bo, g);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          q.d1[k] = mubp ? at(d1e + k * pl + bo, g) : 0.f;
          q.d2[k] = mubp ? at(d2e + k * pl + bo, g) : 0.f;
          q.e[k] = flux ? at(a.u + k * pl + bo, g) : 0.f;
          q.u[k] = flux ? at(ub + k * pl + bo, g) : 0.f;
        }
        q.mb = mubp ? at(mubp, g) : 0.f;
        return q;
      },
      [&](unsigned g, unsigned l, const VIn4& q) {
        const float2 v[4] = {at(z, l), at(z1, l), at(z2, l), at(z3, l)};
        float hx[4], hy[4], g2[4];
        float mb = q.mb;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          hx[k] = q.h[2 * k] + v[k].x;
          hy[k] = q.h[2 * k + 1] + v[k].y;
          at(G1 + k * pl + bo, g) = q.mu * (q.m1x * hx[k] + q.m1y * hy[k]);
          g2[k] = q.mu * (q.m2x * hx[k] + q.m2y * hy[k]);
          const float ex = q.m1x * q.d1[k] + q.m2x * q.d2[k];
          const float ey = q.m1y * q.d1[k] + q.m2y * q.d2[k];
          mb = mb + hx[k] * ex + hy[k] * ey;
        }
        if (mubp) at(mubp, g) = mb;
        at(z, l) = make_float2(g2[0], g2[1]);
        at(z1, l) = make_float2(g2[2], g2[3]);
        if (flux) {
          float fb[4], gb[4], o[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            fb[k] = -hx[k];
            gb[k] = -hy[k];
          }
          flux_vjp(q.e, a.gamma, fb, gb, o);
#pragma unroll
          for (int k = 0; k < 4; ++k) at(ub + k * pl + bo, g) = q.u[k] + o[k];
        }
      });
  __syncthreads();
  // u_bar += D_2^T G2 (G2 of components 0, 1 and 2, 3 as two complex lines)
  line_derivative<true>(X2, Pg, P, a.gq, a.dq, a.d);
  walk_b<kLoadBatch>(
      M.w,
      [&](unsigned g) {
        return make_float4(at(ub + bo, g), at(ub + pl + bo, g), at(ub + 2 * pl + bo, g), at(ub + 3 * pl + bo, g));
      },
      [&](unsigned g, unsigned l, float4 o) {
        const float2 v0 = at(z, l), v1 = at(z1, l);
        at(ub + bo, g) = o.x + v0.x;
        at(ub + pl + bo, g) = o.y + v0.y;
        at(ub + 2 * pl + bo, g) = o.z + v1.x;
        at(ub + 3 * pl + bo, g) = o.w + v1.y;
      });
}

// ---------------------------------------------------------------- network reverse mode

// Reverse mode of the classifier network (Sec. 5.1) at the features of the
// state: for every point of D~ and each direction, the cotangent of the 16
// window features given that of the four logits,
//   feat_bar = W1 (m1 .* W2 (m2 .* W3 logit_bar)),
// m1, m2 the ReLU masks of the forward pass at the window (row-vector
// convention y = x W + b, so the transposes act from the left here); zero
// outside D~.  One thread per (point, direction), FP32; the weights and, per
// thread, the 64 hidden activations and their cotangents live in LDS
// (column tid of a [64][kBlock] array: conflict-free), so that no loop
// keeps 64-entry arrays or the weights in registers.  The features are
// formed as in the forward kernel (window4): offsets -8..7, clamped,
// rescaled to [-1, 1], zero for a flat window.  logit_bar / feat_bar:
// [2][plane][4] / [2][plane][16] at the point's storage index.  Dynamic LDS:
// sdnn_adj_lds_bytes().
struct MlpAdjLds {
  float W1[16 * 64], b1[64], W2[64 * 64], b2[64], W3[64 * 4];
};

__host__ __device__ constexpr size_t sdnn_adj_lds_bytes() {
  return sizeof(MlpAdjLds) + 2 * 64 * kBlock * sizeof(float);
}

__global__ void __launch_bounds__(kBlock) k_sdnn_adj(const ChunkDev* chunks, int nchunks, const PatchDev* patches,
                                                     const float* phi, MlpPtr w, const float* lbar, float* fbar,
                                                     long long pl) {
  MlpAdjLds& L = *reinterpret_cast<MlpAdjLds*>(lds_z);
  float* H = reinterpret_cast<float*>(&L + 1);   // [64][kBlock] hidden activations of layer 1
  float* Gb = H + 64 * kBlock;                    // [64][kBlock] their cotangents
  for (int q = threadIdx.x; q < 16 * 64; q += blockDim.x) L.W1[q] = w.W1[q];
  for (int q = threadIdx.x; q < 64 * 64; q += blockDim.x) L.W2[q] = w.W2[q];
  for (int q = threadIdx.x; q < 64 * 4; q += blockDim.x) L.W3[q] = w.W3[q];
  for (int q = threadIdx.x; q < 64; q += blockDim.x) {
    L.b1[q] = w.b1[q];
    L.b2[q] = w.b2[q];
  }
  __syncthreads();
  const int t = threadIdx.x;
  for (int cb = blockIdx.x; cb < nchunks; cb += gridDim.x) {
    const ChunkDev ck = chunks[cb];
    const PatchDev P = patches[ck.patch];
    const int kk = ck.start + t;
    int i = 0, j = 0;
    if (kk >= pstore(P) || !pdecode(P, kk, i, j)) continue;
    const long long gi = P.off + kk;
    const bool in = in_dtilde(P, i, j);
#pragma unroll 1
    for (int dir = 0; dir < 2; ++dir) {
      float* fo = fbar + 16 * (dir * pl + gi);
      if (!in) {
        for (int f = 0; f < 16; ++f) fo[f] = 0.f;
        continue;
      }
      float x[16];
      {
#pragma clang fp contract(off)
        const int pos = dir == 0 ? i : j, n = dir == 0 ? P.n1 : P.n2;
        float lo = 3.4e38f, hi = -3.4e38f;
#pragma unroll
        for (int f = 0; f < 16; ++f) {
          int k = pos - 8 + f;
          k = k < 0 ? 0 : (k > n - 1 ? n - 1 : k);
          x[f] = phi[dir == 0 ? pidx(P, k, j) : pidx(P, i, k)];
          lo = fminf(lo, x[f]);
          hi = fmaxf(hi, x[f]);
        }
        const float rng = hi - lo;
        const bool flat = rng <= 1e-6f * fmaxf(1.0f, fabsf(hi));
        const float sc = flat ? 0.f : 2.0f / rng;
#pragma unroll
        for (int f = 0; f < 16; ++f) x[f] = flat ? 0.f : (x[f] - lo) * sc - 1.0f;
      }
#pragma unroll 1
      for (int u = 0; u < 64; ++u) {
        float z = L.b1[u];
#pragma unroll
        for (int f = 0; f < 16; ++f) z = fmaf(x[f], L.W1[f * 64 + u], z);
        H[u * kBlock + t] = fmaxf(z, 0.f);
        Gb[u * kBlock + t] = 0.f;
      }
      const float* lb = lbar + 4 * (dir * pl + gi);
      const float l0 = lb[0], l1 = lb[1], l2 = lb[2], l3 = lb[3];
#pragma unroll 1
      for (int k = 0; k < 64; ++k) {
        float z = L.b2[k];
#pragma unroll 8
        for (int u = 0; u < 64; ++u) z = fmaf(H[u * kBlock + t], L.W2[u * 64 + k], z);
        if (z > 0.f) {
          const float* w3 = L.W3 + 4 * k;
          const float g2 = w3[0] * l0 + w3[1] * l1 + w3[2] * l2 + w3[3] * l3;
#pragma unroll 8
          for (int u = 0; u < 64; ++u) Gb[u * kBlock + t] = fmaf(L.W2[u * 64 + k], g2, Gb[u * kBlock + t]);
        }
      }
#pragma unroll 1
      for (int f = 0; f < 16; ++f) {
        float acc = 0.f;
#pragma unroll 8
        for (int u = 0; u < 64; ++u)
          acc = H[u * kBlock + t] > 0.f ? fmaf(L.W1[f * 64 + u], Gb[u * kBlock + t], acc) : acc;
        fo[f] = acc;
      }
    }
  }
}

}  // namespace fcsd
