// Batched pass kernels of the FC-SDNN right-hand side and stage update.
//
// Right-hand side (paper eq. general_curvilinear with the viscous flux of
// eq. f_visc, chain-rule reading):
//     r = sum_{m,a} m[m,a] d/dq^m ( mu d/dx_a e - f_a(e) )
// with d/dx_a e = sum_m m[m,a] d/dq^m e.  Writing H_a = mu d/dx_a e - f'_a
// (f' = f(e) - f(e_ref), the deviation flux; the derivative of the constant
// f(e_ref) is the FC derivative of a constant, ~1e-11) the inviscid and
// viscous divergences share their derivatives, so one stage needs
//   A  (q1 lines): d1 e                                  4 derivatives
//   B1 (q2 lines): d2 e -> H_x, H_y (8 fields)          4 derivatives
//   B2 (q2 lines): r2 = m2x d2 H_x + m2y d2 H_y          8 derivatives
//   C  (q1 lines): r = m1x d1 H_x + m1y d1 H_y + r2, then the SSPRK update
//                                                        8 derivatives
// Every pass is one launch over a tile list covering all patches.
#pragma once
#include "engine.h"

namespace fcsd {

struct PassArgs {
  const PlanDev* plans;
  const TileDev* tiles;
  const float2* tw;
  const float2* km;
  const float2* kf;           // spectral filter factors (null until configured)
  const int* koff;            // per plan: offset of its factors in kf (when not the plan's own)
  const float* win;           // blending window plane (initial-data smearing)
  float* d2out;               // pass B1: also store d2 (e - e_ref) here when not null
  const float* d2th;          // pass B1 on wall patches: d2 theta, for the energy's product rule
  const double* aq;
  const double* dq;
  const float* gq;            // fold matrices of the transposed derivative (per plan, P.gq)
  const float* gf;            // fold matrices of the transposed filter (per plan, P.gf)
  int d;
  long long plane;
  int nf;
  int mode;
  // generic line operator
  const float* in;
  float* out;
  long long ext_plane;
  const long long* ext_off;   // per plan: offset of the plan's first line in ext
  // right-hand side
  const float* u;
  const float* metric;
  const float* mu;
  const float* d1e;
  float* H;
  float* r2;
  float* rhs;
  // stage update
  const float* u0;
  const float* ui;
  float* acc;
  float* uout;
  const float* dt;
  int stage;
  float eref[4];   // reference conserved state
  float pref[4];   // reference primitive state (rho, u, v, p)
  float gamma;
};

enum { MODE_SET = 0, MODE_ADD = 1, MODE_RK = 2 };

// Line kernels: 256 threads, registers capped for five waves per SIMD (the
// butterflies fit in ~96 VGPRs without spilling; five 32 KB tiles fill the LDS)
#define FCSD_LINE_BOUNDS __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(4)))

// elements per thread whose loads are in flight together
constexpr int kLoadBatch = 12;  // load phases (two floats each)
constexpr int kEpiBatch = 8;    // epilogues (point inputs)
constexpr int kEpiBatchH = 4;   // H epilogue (thirteen inputs per point)
constexpr int kEpiBatchC = 8;   // stage-update epilogue (six inputs per point)
constexpr int kDiffBatch = 8;   // differencing loads (four floats each)
enum { FLUX_FULL = 0, FLUX_VISC = 1, FLUX_INVISCID = 2 };

// SSPRK(5,4) Shu-Osher coefficients (five stages, fourth order)
struct RkCoef {
  float a0, ai, b, acc_i, acc_b;
};
__device__ __forceinline__ RkCoef rk_coef(int s) {
  switch (s) {
    case 0: return RkCoef{1.0f, 0.0f, 0.391752226571890f, 0.f, 0.f};
    case 1: return RkCoef{0.444370493651235f, 0.555629506348765f, 0.368410593050371f, 0.f, 0.f};
    case 2: return RkCoef{0.620101851488403f, 0.379898148511597f, 0.251891774271694f, 0.517231671970585f, 0.f};
    case 3: return RkCoef{0.178079954393132f, 0.821920045606868f, 0.544974750228521f, 0.096059710526147f, 0.063692468666290f};
    default: return RkCoef{0.0f, 0.386708617503269f, 0.226007483236906f, 0.f, 0.f};
  }
}

// Deviation fluxes f(e) - f(e_ref), free of cancellation: every term is a
// product with a deviation (de, du, dv, dp).
__device__ __forceinline__ void dev_flux(const float e[4], const float er[4], const float pr[4],
                                         float g, float dF[4], float dG[4]) {
  const float dr = e[0] - er[0], dm = e[1] - er[1], dn = e[2] - er[2], dE = e[3] - er[3];
  const float irho = 1.0f / e[0];
  const float u = e[1] * irho, v = e[2] * irho;
  const float du = (dm - pr[1] * dr) * irho;
  const float dv = (dn - pr[2] * dr) * irho;
  const float mr = er[1], nr = er[2];
  const float dp = (g - 1.0f) * (dE - 0.5f * (dm * u + mr * du + dn * v + nr * dv));
  const float H = e[3] + pr[3] + dp;  // E + p
  dF[0] = dm;
  dF[1] = dm * u + mr * du + dp;
  dF[2] = dm * v + mr * dv;
  dF[3] = du * H + pr[1] * (dE + dp);
  dG[0] = dn;
  dG[1] = dn * u + nr * du;
  dG[2] = dn * v + nr * dv + dp;
  dG[3] = dv * H + pr[2] * (dE + dp);
}

// Global side of a tile: its element walk, the element offset of its first
// stored element in a plane, and the byte offset (from that element) of the
// last element of the patch's storage.
struct TileMem {
  Walk w;
  long long base;
  unsigned gmax;
};

template <int DIR>
__device__ __forceinline__ TileMem tile_mem(const PlanDev& P, const TileDev& T, int nl, int ld) {
  TileMem m;
  m.w = make_walk<DIR>(P.N, nl, ld, P.nb1, P.n1);
  const long long first = tile_first<DIR>(T.line0, P.nb1, P.n1);
  m.base = P.off + first;
  m.gmax = 4u * (unsigned)(patch_storage(P.n1, P.n2, P.nb1) - 1 - first);
  return m;
}

extern __shared__ float2 lds_z[];

// tile prologue common to every line body: tile Tin (nl > 0), plan, LDS
// tables at lds
#define FCSD_TILE_AT(a, Tin, lds)                                            \
  const TileDev T = (Tin);                                                   \
  const PlanDev P = (a).plans[T.plan];                                       \
  const PlanDev* Pg = (a).plans + T.plan;                                    \
  const LineCtx X = line_setup((lds), T, P, (a).tw, (a).km);                 \
  float2* __restrict__ z = X.z;                                              \
  const int N = P.N, nl = T.nl, ld = T.ld;                                   \
  (void)Pg;                                                                  \
  (void)nl;                                                                  \
  (void)N;                                                                   \
  __syncthreads();

// the same for the tile of this workgroup in a one-tile-per-workgroup launch
#define FCSD_TILE_BEGIN(a)                                                   \
  const TileDev T_wg = (a).tiles[blockIdx.x];                                \
  if (T_wg.nl == 0) return; /* padding slot of the launch order */           \
  FCSD_TILE_AT(a, T_wg, lds_z)

// Forward derivative of pairs already loaded by load_differenced: tail
// differences, then the FFT part.
#define FCSD_DIFF_AND_TRANSFORM(a)                                           \
  __syncthreads();                                                           \
  diff_tail(X, P, (a).dq + P.dq, (a).d);                                     \
  __syncthreads();                                                           \
  fft_apply<false>(X, Pg, P);

// ---------------------------------------------------------------- generic line ops

// fc_diff / fc_diff_adj on nf fields, packed two per complex line.
template <int DIR, bool ADJ>
__global__ void FCSD_LINE_BOUNDS k_fcdiff(PassArgs a) {
  FCSD_TILE_BEGIN(a)
  const TileMem M = tile_mem<DIR>(P, T, nl, ld);
  for (int f = 0; f < a.nf; f += 2) {
    const bool two = f + 1 < a.nf;
    const float* A = a.in + (long long)f * a.plane + M.base;
    const float* B = two ? a.in + (long long)(f + 1) * a.plane + M.base : A;
    if (!ADJ) {
      load_differenced<DIR, kDiffBatch>(X, M.w, M.gmax, N, nl, 0, P.nb1, P.n1, A, B, 0.f, 0.f, a.d);
      FCSD_DIFF_AND_TRANSFORM(a)
    } else {
      walk_b<8>(
          M.w, [&](unsigned g) { return make_float2(at(A, g), at(B, g)); },
          [&](unsigned, unsigned l, float2 v) { at(z, l) = make_float2(v.x, two ? v.y : 0.f); });
      __syncthreads();
      line_derivative<true>(X, Pg, P, a.gq, a.dq, a.d);
    }
    float* OA = a.out + (long long)f * a.plane + M.base;
    float* OB = two ? a.out + (long long)(f + 1) * a.plane + M.base : OA;
    if (ADJ) {
      walk_b<kLoadBatch>(
          M.w, [&](unsigned g) { return make_float2(at(OA, g), two ? at(OB, g) : 0.f); },
          [&](unsigned g, unsigned l, float2 o) {
            const float2 v = at(z, l);
            at(OA, g) = o.x + v.x;
            if (two) at(OB, g) = o.y + v.y;
          });
    } else {
      walk(M.w, [&](unsigned g, unsigned l) {
        const float2 v = at(z, l);
        at(OA, g) = v.x;
        if (two) at(OB, g) = v.y;
      });
    }
    __syncthreads();
  }
}

// fc_continue (FWD) and its transpose: ext lines of length L per plan
// (line c of the tile at ext offset e0 + c L, row-major).
template <int DIR, bool ADJ>
__global__ void FCSD_LINE_BOUNDS k_fccont(PassArgs a) {
  FCSD_TILE_BEGIN(a)
  const int L = P.Lx;  // ext lines: the extension, without the padding of an embedded transform
  const TileMem M = tile_mem<DIR>(P, T, nl, ld);
  const Walk we = make_walk<1>(L, nl, ld, 0, L);
  const long long e0 = a.ext_off[T.plan] + (long long)T.line0 * L;
  for (int f = 0; f < a.nf; f += 2) {
    const bool two = f + 1 < a.nf;
    if (!ADJ) {
      const float* A = a.in + (long long)f * a.plane + M.base;
      const float* B = two ? a.in + (long long)(f + 1) * a.plane + M.base : A;
      walk(M.w, [&](unsigned g, unsigned l) { at(z, l) = make_float2(at(A, g), two ? at(B, g) : 0.f); });
      __syncthreads();
      if (!P.periodic) fc_tail(X, P, a.aq + P.aq, a.d);
      __syncthreads();
      float* OA = a.out + (long long)f * a.ext_plane + e0;
      float* OB = two ? a.out + (long long)(f + 1) * a.ext_plane + e0 : OA;
      walk(we, [&](unsigned g, unsigned l) {
        const float2 v = at(z, l);
        at(OA, g) = v.x;
        if (two) at(OB, g) = v.y;
      });
    } else {
      const float* A = a.in + (long long)f * a.ext_plane + e0;
      const float* B = two ? a.in + (long long)(f + 1) * a.ext_plane + e0 : A;
      walk(we, [&](unsigned g, unsigned l) { at(z, l) = make_float2(at(A, g), two ? at(B, g) : 0.f); });
      __syncthreads();
      if (!P.periodic) fold_tail(X, P, a.aq + P.aq, a.d);
      __syncthreads();
      float* OA = a.out + (long long)f * a.plane + M.base;
      float* OB = two ? a.out + (long long)(f + 1) * a.plane + M.base : OA;
      walk(M.w, [&](unsigned g, unsigned l) {
        const float2 v = at(z, l);
        at(OA, g) += v.x;
        if (two) at(OB, g) += v.y;
      });
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- RHS passes

// d_DIR (e - e_ref) of the four state fields into out (pass A for DIR 1),
// on tile Tin with its LDS at lds.
template <int DIR>
__device__ __forceinline__ void dev_diff_tile(const PassArgs& a, const TileDev& Tin, float2* lds) {
  FCSD_TILE_AT(a, Tin, lds)
  const TileMem M = tile_mem<DIR>(P, T, nl, ld);
  const long long pl = a.plane;
  for (int f = 0; f < 4; f += 2) {
    const float* A = a.u + f * pl + M.base;
    const float* B = a.u + (f + 1) * pl + M.base;
    // constant indices: a runtime index into the argument array would live in scratch
    const float ra = f == 0 ? a.eref[0] : a.eref[2], rb = f == 0 ? a.eref[1] : a.eref[3];
    load_differenced<DIR, kDiffBatch>(X, M.w, M.gmax, N, nl, 0, P.nb1, P.n1, A, B, ra, rb, a.d);
    FCSD_DIFF_AND_TRANSFORM(a)
    float* OA = a.out + f * pl + M.base;
    float* OB = a.out + (f + 1) * pl + M.base;
    walk(M.w, [&](unsigned g, unsigned l) {
      const float2 v = at(z, l);
      at(OA, g) = v.x;
      at(OB, g) = v.y;
    });
    __syncthreads();
  }
}

template <int DIR>
__global__ void FCSD_LINE_BOUNDS k_dev_diff(PassArgs a) {
  const TileDev T = a.tiles[blockIdx.x];
  if (T.nl == 0) return;
  dev_diff_tile<DIR>(a, T, lds_z);
}

// Plain load of a pair of planes into complex line c0 + c of the tile (the
// differences then come from difference_ext in LDS: two floats per element
// in flight instead of four, for fields without a reference to subtract).
__device__ __forceinline__ void load_plain(const LineCtx& X, const Walk& w, int c0, const float* __restrict__ A,
                                           const float* __restrict__ B) {
  float2* __restrict__ z = X.z + c0;
  walk_b<kLoadBatch>(
      w, [&](unsigned g) { return make_float2(at(A, g), at(B, g)); },
      [&](unsigned, unsigned l, float2 v) { at(z, l) = v; });
}

// d_DIR (e - e_ref) of the four state fields into out on a tile that holds
// two complex lines per grid line: (e0, e1) and (e2, e3) are loaded
// together, transformed together and stored in one walk.
template <int DIR>
__device__ __forceinline__ void dev_diff2_tile(const PassArgs& a, const TileDev& T, float2* lds) {
  const PlanDev P = a.plans[T.plan];
  const PlanDev* Pg = a.plans + T.plan;
  TileDev T2 = T;
  T2.nl = 2 * T.nl;
  const LineCtx X = line_setup(lds, T2, P, a.tw, a.km);
  float2* __restrict__ z = X.z;
  const int N = P.N, nl = T.nl, ld = T.ld;
  const long long pl = a.plane;
  const TileMem M = tile_mem<DIR>(P, T, nl, ld);
  __syncthreads();
  const float* u = a.u + M.base;
  load_differenced<DIR, kDiffBatch>(X, M.w, M.gmax, N, nl, 0, P.nb1, P.n1, u, u + pl, a.eref[0], a.eref[1], a.d);
  load_differenced<DIR, kDiffBatch>(X, M.w, M.gmax, N, nl, nl, P.nb1, P.n1, u + 2 * pl, u + 3 * pl, a.eref[2],
                                    a.eref[3], a.d);
  FCSD_DIFF_AND_TRANSFORM(a)
  float2* zb = z + nl;
  float* o = a.out + M.base;
  walk(M.w, [&](unsigned g, unsigned l) {
    const float2 v = at(z, l), w = at(zb, l);
    at(o, g) = v.x;
    at(o + pl, g) = v.y;
    at(o + 2 * pl, g) = w.x;
    at(o + 3 * pl, g) = w.y;
  });
}

template <int DIR>
__global__ void FCSD_LINE_BOUNDS k_dev_diff2(PassArgs a) {
  const TileDev T = a.tiles[blockIdx.x];
  if (T.nl == 0) return;
  dev_diff2_tile<DIR>(a, T, lds_z);
}

// Point inputs of all eight H fields (loaded once per point; inputs a flux
// mode does not use read the metric instead, so every load is issued).
struct HIn4 {
  float m1x, m1y, m2x, m2y, mu;
  float d1[4];
  float e[4];
};

// Tile base pointers of those inputs (uniform).
struct HSrc {
  const float *m1x, *m1y, *m2x, *m2y, *mu;
  const float *d10, *d11, *d12, *d13;
  const float *e0, *e1, *e2, *e3;
};

__device__ __forceinline__ HSrc h_sources(const PassArgs& a, long long base, int flux) {
  const long long pl = a.plane;
  const bool visc = flux != FLUX_INVISCID, inv = flux != FLUX_VISC;
  const float* mt = a.metric + base;
  const float* d1 = (visc ? a.d1e : a.metric) + base;
  const long long ds = visc ? pl : 0;
  // the state: for the fluxes, and on wall patches for the energy's product rule
  const bool need_e = inv || a.d2th != nullptr;
  const float* e = (need_e ? a.u : a.metric) + base;
  const long long es = need_e ? pl : 0;
  HSrc h;
  h.m1x = mt;
  h.m1y = mt + pl;
  h.m2x = mt + 2 * pl;
  h.m2y = mt + 3 * pl;
  h.mu = (visc ? a.mu : a.metric) + base;
  h.d10 = d1;
  h.d11 = d1 + ds;
  h.d12 = d1 + 2 * ds;
  h.d13 = d1 + 3 * ds;
  h.e0 = e;
  h.e1 = e + es;
  h.e2 = e + 2 * es;
  h.e3 = e + 3 * es;
  return h;
}

__device__ __forceinline__ HIn4 load_H4_inputs(const HSrc& h, unsigned g) {
  HIn4 q;
  q.m1x = at(h.m1x, g);
  q.m1y = at(h.m1y, g);
  q.m2x = at(h.m2x, g);
  q.m2y = at(h.m2y, g);
  q.mu = at(h.mu, g);
  q.d1[0] = at(h.d10, g);
  q.d1[1] = at(h.d11, g);
  q.d1[2] = at(h.d12, g);
  q.d1[3] = at(h.d13, g);
  q.e[0] = at(h.e0, g);
  q.e[1] = at(h.e1, g);
  q.e[2] = at(h.e2, g);
  q.e[3] = at(h.e3, g);
  return q;
}

// Pass B1 (q2 lines): d2 e of all four components at once (two complex
// lines per grid line: components 0,1 at z[pos][c], 2,3 at z[pos][nl + c]),
// then H = mu grad_x e - f' (mode FLUX_FULL / FLUX_VISC).  H layout: field
// 2c = H_x component c, 2c+1 = H_y component c.
// FUSED: passes B1 and B2 on one tile.  The H epilogue also leaves
// (H_x, H_y) of components 0 and 1 in LDS as the two complex lines of every
// grid line, which are differenced and transformed in place; components 2
// and 3 are then read back from the H this workgroup has just stored (the
// barrier orders the stores before the loads), and r2_c = m2x d2 H_x,c +
// m2y d2 H_y,c is stored for all four.  The result equals passes B1 and B2
// bit for bit (the same FP32 operations on every line).  With FLUX_INVISCID
// the first transform is skipped and H = -f'.
template <bool FUSED>
__device__ __forceinline__ void passB_tile(const PassArgs& a, const TileDev& T, float2* lds) {
  const PlanDev P = a.plans[T.plan];
  const PlanDev* Pg = a.plans + T.plan;
  TileDev T2 = T;
  T2.nl = 2 * T.nl;
  const LineCtx X = line_setup(lds, T2, P, a.tw, a.km);
  float2* __restrict__ z = X.z;
  const int N = P.N, nl = T.nl, ld = T.ld;
  const long long pl = a.plane;
  const TileMem M = tile_mem<2>(P, T, nl, ld);
  __syncthreads();
  const int flux = a.mode;
  if (!FUSED || flux != FLUX_INVISCID) {
    const float* u = a.u + M.base;
    load_differenced<2, kDiffBatch>(X, M.w, M.gmax, N, nl, 0, P.nb1, P.n1, u, u + pl, a.eref[0], a.eref[1], a.d);
    load_differenced<2, kDiffBatch>(X, M.w, M.gmax, N, nl, nl, P.nb1, P.n1, u + 2 * pl, u + 3 * pl, a.eref[2],
                                    a.eref[3], a.d);
    FCSD_DIFF_AND_TRANSFORM(a)
  }
  const HSrc hs = h_sources(a, M.base, flux);
  float* H = a.H + M.base;
  float* d2o = a.d2out ? a.d2out + M.base : nullptr;
  float2* zb = z + nl;
  walk_b<kEpiBatchH>(
      M.w, [&](unsigned g) { return load_H4_inputs(hs, g); },
      [&](unsigned g, unsigned l, const HIn4& q) {
        const float2 za = at(z, l), zq = at(zb, l);
        float d2[4] = {za.x, za.y, zq.x, zq.y};
        if (a.d2th && P.wallp) {
          // the energy's derivative by the product rule from rho, m and theta's
          // (Remark adiabatic): dE = A d rho + B d theta + (m . dm) / rho
          const float ir = 1.0f / q.e[0], mq = q.e[1] * q.e[1] + q.e[2] * q.e[2];
          const float A = q.e[3] * ir - mq * ir * ir, B = q.e[0] / (a.gamma - 1.0f);
          d2[3] = A * d2[0] + B * at(a.d2th + M.base, g) + (q.e[1] * d2[1] + q.e[2] * d2[2]) * ir;
        }
        if (d2o) {
#pragma unroll
          for (int k = 0; k < 4; ++k) at(d2o + k * pl, g) = d2[k];
        }
        float dF[4] = {0.f, 0.f, 0.f, 0.f}, dG[4] = {0.f, 0.f, 0.f, 0.f};
        if (flux != FLUX_VISC) dev_flux(q.e, a.eref, a.pref, a.gamma, dF, dG);
        float h[8];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          float vx = 0.f, vy = 0.f;
          if (flux != FLUX_INVISCID) {
            vx = q.mu * (q.m1x * q.d1[k] + q.m2x * d2[k]);
            vy = q.mu * (q.m1y * q.d1[k] + q.m2y * d2[k]);
          }
          h[2 * k] = vx - dF[k];
          h[2 * k + 1] = vy - dG[k];
          at(H + (2 * k) * pl, g) = h[2 * k];
          at(H + (2 * k + 1) * pl, g) = h[2 * k + 1];
        }
        if (FUSED) {
          at(z, l) = make_float2(h[0], h[1]);
          at(zb, l) = make_float2(h[2], h[3]);
        }
      });
  if (!FUSED) return;
  const float* m2x = a.metric + 2 * pl + M.base;
  const float* m2y = a.metric + 3 * pl + M.base;
  float* r2 = a.r2 + M.base;
  __syncthreads();
  // components 0 and 1: differences of the LDS lines, transform
  difference_ext(X, P, a.dq + P.dq, a.d);
  fft_apply<false>(X, Pg, P);
  for (int half = 0; half < 2; ++half) {
    float* ra = r2 + (2 * half) * pl;
    float* rb = r2 + (2 * half + 1) * pl;
    walk_b<kLoadBatch>(
        M.w, [&](unsigned g) { return make_float2(at(m2x, g), at(m2y, g)); },
        [&](unsigned g, unsigned l, float2 m) {
          const float2 v = at(z, l), w = at(zb, l);
          at(ra, g) = m.x * v.x + m.y * v.y;
          at(rb, g) = m.x * w.x + m.y * w.y;
        });
    __syncthreads();
    if (half == 1) break;
    // components 2 and 3 from the stored H
    load_plain(X, M.w, 0, H + 4 * pl, H + 5 * pl);
    load_plain(X, M.w, nl, H + 6 * pl, H + 7 * pl);
    __syncthreads();
    difference_ext(X, P, a.dq + P.dq, a.d);
    fft_apply<false>(X, Pg, P);
  }
}

// Passes B1 and B2 on a q2 tile that holds all eight H fields in LDS (tile
// set of four complex lines per grid line, row stride >= 4 nl): d2 e of the
// four components in slots 0, 1 (two complex lines per grid line), the H
// epilogue stores H (for pass C) and writes (H_x, H_y) of component c into
// slot c, then one transform of the four slots and r2 of all components from
// one read of the q2 metric rows.  The same FP32 operations on every line as
// passes B1 and B2 (bit-identical results).
__device__ __forceinline__ void passB4_tile(const PassArgs& a, const TileDev& T, float2* lds) {
  const PlanDev P = a.plans[T.plan];
  const PlanDev* Pg = a.plans + T.plan;
  TileDev T2 = T;
  T2.nl = 2 * T.nl;
  const LineCtx X = line_setup(lds, T2, P, a.tw, a.km);
  const LineCtx X4 = line_view(X, 4 * T.nl);
  float2* __restrict__ z = X.z;
  const int N = P.N, nl = T.nl, ld = T.ld;
  const long long pl = a.plane;
  const TileMem M = tile_mem<2>(P, T, nl, ld);
  __syncthreads();
  const int flux = a.mode;
  if (flux != FLUX_INVISCID) {
    const float* u = a.u + M.base;
    load_differenced<2, kDiffBatch>(X, M.w, M.gmax, N, nl, 0, P.nb1, P.n1, u, u + pl, a.eref[0], a.eref[1], a.d);
    load_differenced<2, kDiffBatch>(X, M.w, M.gmax, N, nl, nl, P.nb1, P.n1, u + 2 * pl, u + 3 * pl, a.eref[2],
                                    a.eref[3], a.d);
    FCSD_DIFF_AND_TRANSFORM(a)
  }
  const HSrc hs = h_sources(a, M.base, flux);
  float* H = a.H + M.base;
  float* d2o = a.d2out ? a.d2out + M.base : nullptr;
  float2* zb = z + nl;
  float2* zc = z + 2 * nl;
  float2* zd = z + 3 * nl;
  walk_b<kEpiBatchH>(
      M.w, [&](unsigned g) { return load_H4_inputs(hs, g); },
      [&](unsigned g, unsigned l, const HIn4& q) {
        const float2 za = at(z, l), zq = at(zb, l);
        float d2[4] = {za.x, za.y, zq.x, zq.y};
        if (a.d2th && P.wallp) {
          // the energy's derivative by the product rule (Remark adiabatic)
          const float ir = 1.0f / q.e[0], mq = q.e[1] * q.e[1] + q.e[2] * q.e[2];
          const float A = q.e[3] * ir - mq * ir * ir, B = q.e[0] / (a.gamma - 1.0f);
          d2[3] = A * d2[0] + B * at(a.d2th + M.base, g) + (q.e[1] * d2[1] + q.e[2] * d2[2]) * ir;
        }
        if (d2o) {
#pragma unroll
          for (int k = 0; k < 4; ++k) at(d2o + k * pl, g) = d2[k];
        }
        float dF[4] = {0.f, 0.f, 0.f, 0.f}, dG[4] = {0.f, 0.f, 0.f, 0.f};
        if (flux != FLUX_VISC) dev_flux(q.e, a.eref, a.pref, a.gamma, dF, dG);
        float h[8];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          float vx = 0.f, vy = 0.f;
          if (flux != FLUX_INVISCID) {
            vx = q.mu * (q.m1x * q.d1[k] + q.m2x * d2[k]);
            vy = q.mu * (q.m1y * q.d1[k] + q.m2y * d2[k]);
          }
          h[2 * k] = vx - dF[k];
          h[2 * k + 1] = vy - dG[k];
          at(H + (2 * k) * pl, g) = h[2 * k];
          at(H + (2 * k + 1) * pl, g) = h[2 * k + 1];
        }
        at(z, l) = make_float2(h[0], h[1]);
        at(zb, l) = make_float2(h[2], h[3]);
        at(zc, l) = make_float2(h[4], h[5]);
        at(zd, l) = make_float2(h[6], h[7]);
      });
  __syncthreads();
  difference_ext(X4, P, a.dq + P.dq, a.d);
  fft_apply<false>(X4, Pg, P);
  const float* m2x = a.metric + 2 * pl + M.base;
  const float* m2y = a.metric + 3 * pl + M.base;
  float* r2 = a.r2 + M.base;
  walk_b<kLoadBatch>(
      M.w, [&](unsigned g) { return make_float2(at(m2x, g), at(m2y, g)); },
      [&](unsigned g, unsigned l, float2 m) {
        const float2 v0 = at(z, l), v1 = at(zb, l), v2 = at(zc, l), v3 = at(zd, l);
        at(r2, g) = m.x * v0.x + m.y * v0.y;
        at(r2 + pl, g) = m.x * v1.x + m.y * v1.y;
        at(r2 + 2 * pl, g) = m.x * v2.x + m.y * v2.y;
        at(r2 + 3 * pl, g) = m.x * v3.x + m.y * v3.y;
      });
}

__global__ void FCSD_LINE_BOUNDS k_passB1(PassArgs a) {
  const TileDev T = a.tiles[blockIdx.x];
  if (T.nl == 0) return;
  passB_tile<false>(a, T, lds_z);
}

// Passes B1 and B2 in one launch (see passB_tile).
__global__ void FCSD_LINE_BOUNDS k_passB(PassArgs a) {
  const TileDev T = a.tiles[blockIdx.x];
  if (T.nl == 0) return;
  passB_tile<true>(a, T, lds_z);
}

// The same with all eight H fields in LDS (see passB4_tile).
__global__ void FCSD_LINE_BOUNDS k_passB4(PassArgs a) {
  const TileDev T = a.tiles[blockIdx.x];
  if (T.nl == 0) return;
  passB4_tile(a, T, lds_z);
}

// Spectral filter of the state (paper Sec. 4.3.1, eq. filtering) along
// DIR: two complex lines per grid line, (rho, rho u) at z[pos][c] and
// (rho v, theta) at z[pos][nl + c], extended by the continuation (fc_tail),
// transformed with the filter factors as multipliers.  DIR 1 reads the
// conserved state and forms theta = p / rho (eqs. perfect_gas, p_T), and
// writes theta in place of E; DIR 2 reads that and writes the state with E
// rebuilt from the filtered fields (eq. perfect_gas_T).  A tile reads all of
// its lines before it writes them, so in may equal out.
template <int DIR>
__global__ void FCSD_LINE_BOUNDS k_filter(PassArgs a) {
  const TileDev T = a.tiles[blockIdx.x];
  if (T.nl == 0) return;
  const PlanDev P = a.plans[T.plan];
  const PlanDev* Pg = a.plans + T.plan;
  TileDev T2 = T;
  T2.nl = 2 * T.nl;
  const LineCtx X = line_setup(lds_z, T2, P, a.tw, a.kf, P.kf);
  float2* __restrict__ z = X.z;
  const int nl = T.nl, ld = T.ld;
  const long long pl = a.plane;
  const TileMem M = tile_mem<DIR>(P, T, nl, ld);
  const float g1 = a.gamma - 1.0f;
  const float* in = a.in + M.base;
  float* out = a.out + M.base;
  float2* __restrict__ zb = z + nl;
  __syncthreads();
  walk_b<kEpiBatch>(
      M.w, [&](unsigned g) { return make_float4(at(in, g), at(in + pl, g), at(in + 2 * pl, g), at(in + 3 * pl, g)); },
      [&](unsigned, unsigned l, float4 v) {
        float th = v.w;
        if (DIR == 1) th = g1 * (v.w - 0.5f * (v.y * v.y + v.z * v.z) / v.x) / v.x;
        at(z, l) = make_float2(v.x, v.y);
        at(zb, l) = make_float2(v.z, th);
      });
  __syncthreads();
  if (!P.periodic)
    fc_tail(X, P, a.aq + P.aq, a.d);
  else
    zero_pad(X, P);
  __syncthreads();
  fft_apply<false>(X, Pg, P);
  walk(M.w, [&](unsigned g, unsigned l) {
    const float2 p = at(z, l), q = at(zb, l);
    at(out, g) = p.x;
    at(out + pl, g) = p.y;
    at(out + 2 * pl, g) = q.x;
    at(out + 3 * pl, g) = DIR == 1 ? q.y : p.x * q.y / g1 + 0.5f * (p.y * p.y + q.x * q.x) / p.x;
  });
}

// Localized smearing of initial data (paper Sec. 4.3.2, eq. q) along DIR:
// every line is filtered as in k_filter, with the smearing filter's factors
// (table a.kf at offset a.koff[plan]), and blended with its unfiltered values
// by the window plane a.win, F + w (F~ - F), for rho, rho u, rho v and theta.
// DIR 1 reads the state and writes theta in place of E; DIR 2 reads that
// and writes the state with E rebuilt (eq. perfect_gas_T).  in may equal out.
template <int DIR>
__global__ void FCSD_LINE_BOUNDS k_smear(PassArgs a) {
  const TileDev T = a.tiles[blockIdx.x];
  if (T.nl == 0) return;
  const PlanDev P = a.plans[T.plan];
  const PlanDev* Pg = a.plans + T.plan;
  TileDev T2 = T;
  T2.nl = 2 * T.nl;
  const LineCtx X = line_setup(lds_z, T2, P, a.tw, a.kf, a.koff[T.plan]);
  float2* __restrict__ z = X.z;
  const int nl = T.nl, ld = T.ld;
  const long long pl = a.plane;
  const TileMem M = tile_mem<DIR>(P, T, nl, ld);
  const float g1 = a.gamma - 1.0f;
  const float* in = a.in + M.base;
  const float* win = a.win + M.base;
  float* out = a.out + M.base;
  float2* __restrict__ zb = z + nl;
  auto theta = [&](float4 v) { return DIR == 1 ? g1 * (v.w - 0.5f * (v.y * v.y + v.z * v.z) / v.x) / v.x : v.w; };
  __syncthreads();
  walk_b<kEpiBatch>(
      M.w, [&](unsigned g) { return make_float4(at(in, g), at(in + pl, g), at(in + 2 * pl, g), at(in + 3 * pl, g)); },
      [&](unsigned, unsigned l, float4 v) {
        at(z, l) = make_float2(v.x, v.y);
        at(zb, l) = make_float2(v.z, theta(v));
      });
  __syncthreads();
  if (!P.periodic)
    fc_tail(X, P, a.aq + P.aq, a.d);
  else
    zero_pad(X, P);
  __syncthreads();
  fft_apply<false>(X, Pg, P);
  struct In5 {
    float4 v;
    float w;
  };
  walk_b<kEpiBatch>(
      M.w,
      [&](unsigned g) {
        In5 q;
        q.v = make_float4(at(in, g), at(in + pl, g), at(in + 2 * pl, g), at(in + 3 * pl, g));
        q.w = at(win, g);
        return q;
      },
      [&](unsigned g, unsigned l, const In5& q) {
        const float2 p = at(z, l), r = at(zb, l);
        const float th = theta(q.v);
        const float f0 = q.v.x + q.w * (p.x - q.v.x), f1 = q.v.y + q.w * (p.y - q.v.y);
        const float f2 = q.v.z + q.w * (r.x - q.v.z), f3 = th + q.w * (r.y - th);
        at(out, g) = f0;
        at(out + pl, g) = f1;
        at(out + 2 * pl, g) = f2;
        at(out + 3 * pl, g) = DIR == 1 ? f3 : f0 * f3 / g1 + 0.5f * (f1 * f1 + f2 * f2) / f0;
      });
}

// Reverse mode of k_filter along DIR (transpose E^T S R^T of each line
// filter, S symmetric: zero-pad, the same factors, fold the tail), two
// complex lines per grid line as in the forward pass.  DIR 2 runs first:
// a.in holds the cotangent of the filtered state, a.u the filtered state
// (for the vector-Jacobian product of the rebuilt E), out the cotangent of
// (rho, rho u, rho v, theta) after the transposed q2 filter.  DIR 1: a.in
// holds that, a.u the filter's input state (for the product of theta), out
// the cotangent of the input state.  in may equal out.
template <int DIR>
__global__ void FCSD_LINE_BOUNDS k_filter_adj(PassArgs a) {
  const TileDev T = a.tiles[blockIdx.x];
  if (T.nl == 0) return;
  const PlanDev P = a.plans[T.plan];
  const PlanDev* Pg = a.plans + T.plan;
  TileDev T2 = T;
  T2.nl = 2 * T.nl;
  const LineCtx X = line_setup(lds_z, T2, P, a.tw, a.kf, P.kf);
  float2* __restrict__ z = X.z;
  const int nl = T.nl, ld = T.ld;
  const long long pl = a.plane;
  const TileMem M = tile_mem<DIR>(P, T, nl, ld);
  const float g1 = a.gamma - 1.0f;
  const float* in = a.in + M.base;
  const float* st = a.u + M.base;
  float* out = a.out + M.base;
  float2* __restrict__ zb = z + nl;
  __syncthreads();
  if (DIR == 2) {
    struct In8 {
      float b[4], e[4];
    };
    walk_b<kEpiBatchH>(
        M.w,
        [&](unsigned g) {
          In8 q;
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            q.b[k] = at(in + k * pl, g);
            q.e[k] = at(st + k * pl, g);
          }
          return q;
        },
        [&](unsigned, unsigned l, const In8& q) {
          // E' = rho' theta' / (gamma - 1) + (m'^2 + n'^2) / (2 rho')
          const float r = q.e[0], m = q.e[1], n = q.e[2];
          const float ir = 1.0f / r, ke = 0.5f * (m * m + n * n) * ir;
          const float th = g1 * (q.e[3] - ke) * ir;
          const float Eb = q.b[3];
          at(z, l) = make_float2(q.b[0] + Eb * (th / g1 - ke * ir), q.b[1] + Eb * m * ir);
          at(zb, l) = make_float2(q.b[2] + Eb * n * ir, Eb * r / g1);
        });
  } else {
    walk_b<kEpiBatch>(
        M.w, [&](unsigned g) { return make_float4(at(in, g), at(in + pl, g), at(in + 2 * pl, g), at(in + 3 * pl, g)); },
        [&](unsigned, unsigned l, float4 v) {
          at(z, l) = make_float2(v.x, v.y);
          at(zb, l) = make_float2(v.z, v.w);
        });
  }
  zero_tail(X, P);
  __syncthreads();
  if (!P.periodic) {
    fold_pre(X, P.N, a.gf + P.gf, a.d);
    __syncthreads();
  }
  fft_apply<true>(X, Pg, P);
  if (!P.periodic) {
    fold_post(X, P.N, a.d);
    __syncthreads();
  }
  if (DIR == 2) {
    walk(M.w, [&](unsigned g, unsigned l) {
      const float2 p = at(z, l), q = at(zb, l);
      at(out, g) = p.x;
      at(out + pl, g) = p.y;
      at(out + 2 * pl, g) = q.x;
      at(out + 3 * pl, g) = q.y;
    });
  } else {
    // theta = (gamma - 1) (E / rho - (m^2 + n^2) / (2 rho^2))
    walk_b<kEpiBatch>(
        M.w, [&](unsigned g) { return make_float4(at(st, g), at(st + pl, g), at(st + 2 * pl, g), at(st + 3 * pl, g)); },
        [&](unsigned g, unsigned l, float4 e) {
          const float2 p = at(z, l), q = at(zb, l);
          const float ir = 1.0f / e.x, ir2 = ir * ir, tb = q.y * g1;
          at(out, g) = p.x + tb * (-e.w * ir2 + (e.y * e.y + e.z * e.z) * ir2 * ir);
          at(out + pl, g) = p.y - tb * e.y * ir2;
          at(out + 2 * pl, g) = q.x - tb * e.z * ir2;
          at(out + 3 * pl, g) = tb * ir;
        });
  }
}

// Inviscid H = -f' (pointwise, no derivative needed).
__global__ void __launch_bounds__(kBlock) k_passH(PassArgs a, long long n) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  float e[4], dF[4], dG[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) e[k] = a.u[(long long)k * a.plane + g];
  if (!(e[0] > 0.f)) {  // padding between patches: leave H at zero
#pragma unroll
    for (int k = 0; k < 8; ++k) a.H[(long long)k * a.plane + g] = 0.f;
    return;
  }
  dev_flux(e, a.eref, a.pref, a.gamma, dF, dG);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    a.H[(long long)(2 * k) * a.plane + g] = -dF[k];
    a.H[(long long)(2 * k + 1) * a.plane + g] = -dG[k];
  }
}

// Pass B2 (q2 lines): r2_c = m2x d2 H_x,c + m2y d2 H_y,c.
__global__ void FCSD_LINE_BOUNDS k_passB2(PassArgs a) {
  FCSD_TILE_BEGIN(a)
  const TileMem M = tile_mem<2>(P, T, nl, ld);
  const long long pl = a.plane;
  const float* m2x = a.metric + 2 * pl + M.base;
  const float* m2y = a.metric + 3 * pl + M.base;
  for (int comp = 0; comp < 4; ++comp) {
    const float* A = a.H + (2 * comp) * pl + M.base;
    const float* B = a.H + (2 * comp + 1) * pl + M.base;
    load_differenced<2, kDiffBatch>(X, M.w, M.gmax, N, nl, 0, P.nb1, P.n1, A, B, 0.f, 0.f, a.d);
    FCSD_DIFF_AND_TRANSFORM(a)
    float* r2 = a.r2 + comp * pl + M.base;
    walk_b<kLoadBatch>(
        M.w, [&](unsigned g) { return make_float2(at(m2x, g), at(m2y, g)); },
        [&](unsigned g, unsigned l, float2 m) {
          const float2 v = at(z, l);
          at(r2, g) = m.x * v.x + m.y * v.y;
        });
    __syncthreads();
  }
}

// Pass C (q1 lines): r = m1x d1 H_x + m1y d1 H_y + r2, then store (SET/ADD)
// or the SSPRK register update (RK), on tile Tin with its LDS at lds.
__device__ __forceinline__ void passC_tile(const PassArgs& a, const TileDev& Tin, float2* lds) {
  FCSD_TILE_AT(a, Tin, lds)
  const TileMem M = tile_mem<1>(P, T, nl, ld);
  const long long pl = a.plane;
  float dt = 0.f;
  const RkCoef K = rk_coef(a.stage);
  if (a.mode == MODE_RK) dt = a.dt[0];
  const float* m1x = a.metric + M.base;
  const float* m1y = a.metric + pl + M.base;
  for (int comp = 0; comp < 4; ++comp) {
    const float* A = a.H + (2 * comp) * pl + M.base;
    const float* B = a.H + (2 * comp + 1) * pl + M.base;
    load_plain(X, M.w, 0, A, B);
    __syncthreads();
    difference_ext(X, P, a.dq + P.dq, a.d);
    fft_apply<false>(X, Pg, P);
    const long long fo = comp * pl + M.base;
    // point inputs: the q1 metric row, r2 and the SSPRK registers of the
    // stage; every load is issued (registers the stage does not use read r2)
    const float* r2c = a.r2 + fo;
    const bool rk = a.mode == MODE_RK;
    const float* uic = rk ? a.ui + fo : r2c;
    const float* wc = a.mode == MODE_ADD ? a.rhs + fo : ((rk && a.stage >= 3) ? a.acc + fo : r2c);
    const float* u0c = (rk && a.stage <= 3) ? a.u0 + fo : r2c;
    float* rhs = a.rhs + fo;
    float* uout = a.uout + fo;
    float* acc = a.acc + fo;
    struct CIn {
      float m1x, m1y, r2, ui, w, u0;
    };
    walk_b<kEpiBatchC>(
        M.w,
        [&](unsigned g) {
          CIn q;
          q.m1x = at(m1x, g);
          q.m1y = at(m1y, g);
          q.r2 = at(r2c, g);
          q.ui = at(uic, g);
          q.w = at(wc, g);
          q.u0 = at(u0c, g);
          return q;
        },
        [&](unsigned g, unsigned l, const CIn& q) {
          const float2 v = at(z, l);
          const float r = q.m1x * v.x + q.m1y * v.y + q.r2;
          if (a.mode == MODE_SET) {
            at(rhs, g) = r;
          } else if (a.mode == MODE_ADD) {
            at(rhs, g) = q.w + r;
          } else {
            const float ui = q.ui;
            const float dr = dt * r;
            if (a.stage <= 1) {
              at(uout, g) = K.a0 * q.u0 + K.ai * ui + K.b * dr;
            } else if (a.stage == 2) {
              at(uout, g) = K.a0 * q.u0 + K.ai * ui + K.b * dr;
              at(acc, g) = K.acc_i * ui;
            } else if (a.stage == 3) {
              at(uout, g) = K.a0 * q.u0 + K.ai * ui + K.b * dr;
              at(acc, g) = q.w + (K.acc_i * ui + K.acc_b * dr);
            } else {
              at(uout, g) = q.w + K.ai * ui + K.b * dr;
            }
          }
        });
    __syncthreads();
  }
}

__global__ void FCSD_LINE_BOUNDS k_passC(PassArgs a) {
  const TileDev T = a.tiles[blockIdx.x];
  if (T.nl == 0) return;
  passC_tile(a, T, lds_z);
}

// ---------------------------------------------------------------- one launch per stage

// Task kinds of the persistent stage kernel: pass A on a q1 tile, passes
// B1 + B2 on a q2 tile (two complex lines per grid line), pass C on a q1
// tile.
enum { TASK_A = 0, TASK_B = 1, TASK_C = 2 };

struct StageArgs {
  PassArgs A, B, C;         // the passes' arguments (A.tiles, B.tiles: the q1 and q2 tile arrays)
  const int2* tasks;        // (kind, tile index), in queue order
  int ntasks;
  int npatch;
  int skipA;                // inviscid stage: A tasks do nothing
  unsigned* ctr;            // [0] queue head; [1 + p] A tiles done of patch p; [1 + np + p] B tiles done
  const unsigned* need;     // [p] A tiles of patch p; [np + p] B tiles of patch p
  unsigned* err;            // bit 0 set when a wait gave up (results of the launch are then invalid)
};

// Upper bound on the polls of one dependency wait (each poll sleeps ~128
// cycles: about a second in all), after which the workgroup records the
// failure in err and goes on, so that every workgroup ends.
constexpr int kSpinLimit = 1 << 24;

// One RK stage in one launch: every workgroup takes tasks from a global
// queue until it is empty.  The queue holds all A tasks, then every B task,
// then every C task, so a task only depends on tasks taken before it (B on
// its patch's A tiles, C on its patch's B tiles), which are held by running
// workgroups: the earliest unfinished task can always proceed, whatever the
// number of resident workgroups.  A task's completion is published by a
// release increment of its patch's counter after a workgroup barrier (every
// thread's stores are then complete); a dependent task starts after an
// acquire poll of that counter.  Phases of different patches overlap, and no
// workgroup idles at the end of a pass.  The counters start at zero (the
// host clears them before the launch).
__global__ void FCSD_LINE_BOUNDS k_stage(StageArgs s) {
  // the first 16 bytes of the dynamic LDS hold the task index; tiles start after
  int* slot = reinterpret_cast<int*>(lds_z);
  float2* lds = lds_z + 2;
  const int np = s.npatch;
  for (;;) {
    __syncthreads();  // the previous task's LDS reads are done; the slot is free
    if (threadIdx.x == 0) slot[0] = (int)atomicAdd(s.ctr, 1u);
    __syncthreads();
    const int t = slot[0];
    if (t >= s.ntasks) return;
    const int2 k = s.tasks[t];
    const TileDev T = (k.x == TASK_B ? s.B.tiles : s.A.tiles)[k.y];
    const int p = T.plan;  // one plan per patch and direction
    if (k.x != TASK_A) {
      if (threadIdx.x == 0) {
        const int dep = (k.x == TASK_B ? 0 : np) + p;
        const unsigned need = s.need[dep];
        unsigned* c = s.ctr + 1 + dep;
        int polls = 0;
        while (__hip_atomic_load(c, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < need) {
          if (++polls > kSpinLimit) {
            atomicOr(s.err, 1u);
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
      }
      __syncthreads();
    }
    if (k.x == TASK_A) {
      if (!s.skipA) dev_diff_tile<1>(s.A, T, lds);
    } else if (k.x == TASK_B) {
      passB_tile<true>(s.B, T, lds);
    } else {
      passC_tile(s.C, T, lds);
    }
    if (k.x != TASK_C) {
      __syncthreads();  // every thread's stores of the task are complete
      if (threadIdx.x == 0)
        __hip_atomic_fetch_add(s.ctr + 1 + (k.x == TASK_A ? 0 : np) + p, 1u, __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

}  // namespace fcsd
