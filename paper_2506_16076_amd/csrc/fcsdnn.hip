// libfcsdnn: host side of the C ABI declared in include/fcsdnn.h.
#include "../../include/fcsdnn.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "kernels2.h"

using namespace fcsd;

extern "C" int fcsd_host_fc_matrix(int d, int C, double* out);
extern "C" int fcsd_host_fc_dmatrix(int d, int C, double* out);
extern "C" void fcsd_host_twiddles(int L, float* out);
extern "C" int fcsd_host_factor(int L, int* rad);
extern "C" int fcsd_host_embed_length(int n);
extern "C" void fcsd_host_kmul_embedded(int N, int L, int M, int nst, const int* rad, float* out, int periodic);
extern "C" void fcsd_host_fmul_embedded(int N, int L, int M, int nst, const int* rad, double alpha, int p,
                                        float* out);
extern "C" void fcsd_host_kmul(int N, int L, int nst, const int* rad, float* out, int periodic);
extern "C" void fcsd_host_fmul(int L, int nst, const int* rad, double alpha, int p, float* out);
extern "C" int fcsd_host_fold_matrix(int N, int C, int d, const double* arq, int kind, double alpha, int p,
                                     double* out);

namespace {

constexpr size_t kLdsBudget = 65536;  // bytes of LDS per line-engine workgroup

struct GraphEntry {
  std::vector<unsigned char> key;
  hipGraphExec_t exec = nullptr;
};
constexpr size_t kMaxGraphs = 8;   // captured steps kept per patch set (distinct argument sets)

}  // namespace

struct fcsd_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  unsigned* scratch = nullptr;  // this device's address of the static scratch array
};

// Scratch of the allocation-free entry point fcsd_cfl_dt_noalloc: the
// per-patch maxima of the step-size reduction, two words per patch, for at
// most kNoAllocPatches patches (128 KiB).  Every device the library runs on
// holds its own copy until the process ends.  Host code never uses the
// name as an address: its device address is looked up once per device
// (hipGetSymbolAddress, with that device current, at context creation) and
// kept in scratch_of_device.
constexpr int kNoAllocPatches = 16384;
static __device__ __align__(256) unsigned scratch[2 * kNoAllocPatches];

namespace {

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
unsigned* scratch_of_device[kMaxDevices] = {};

// Device address of `scratch` on the current device `device`.
hipError_t scratch_address(int device, unsigned** out) {
  std::lock_guard<std::mutex> g(scratch_mu);
  if (!scratch_of_device[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    scratch_of_device[device] = static_cast<unsigned*>(p);
  }
  *out = scratch_of_device[device];
  return hipSuccess;
}

}  // namespace

namespace {

// Tiles of one direction for kernels that hold `fields` complex lines per
// grid line in LDS (1, or 2 for the H pass, which transforms all four state
// components at once).
struct TileSet {
  size_t budget = 0;                      // LDS budget per workgroup (bytes)
  int threads = kBlock;                   // workgroup size
  std::vector<TileDev> tiles;             // launch order (LPT or XCD-grouped)
  std::vector<TileDev> tiles_by_patch;    // patch-contiguous
  std::vector<int> patch_begin;           // npatch + 1
  std::vector<size_t> patch_lds;          // per patch
  size_t lds = 0;
  TileDev* d_tiles = nullptr;
  TileDev* d_tiles_bp = nullptr;
};

struct DirPlan {
  std::vector<PlanDev> plans;             // one per patch
  TileSet ts[3];                          // one / two / four complex lines per grid line
  std::vector<long long> ext_off;         // per plan
  long long ext_plane = 0;
  PlanDev* d_plans = nullptr;
  long long* d_ext_off = nullptr;
};

}  // namespace

struct fcsd_set {
  fcsd_ctx* ctx = nullptr;
  int npatch = 0, d = 0;
  long long plane = 0;
  long long npoints = 0;
  std::vector<fcsd_patch_desc> desc;
  DirPlan dir[2];
  float2* d_tw = nullptr;
  float2* d_km = nullptr;
  float2* d_kf = nullptr;                 // spectral filter factors (fcsd_set_filter)
  int filter_on = 0;
  double filter_alpha = 0.0;
  int filter_p = 0;
  WallDev* d_walls = nullptr;             // no-slip adiabatic wall entries (fcsd_set_walls)
  int nwalls = 0, wall_len = 0;
  std::vector<uint8_t> wall_patch;        // per patch: has a wall side
  ChunkDev* d_wchunks = nullptr;          // point chunks of the wall patches
  int nwchunks = 0;
  TileDev* d_wtiles[2] = {nullptr, nullptr};  // per direction: line tiles (single-field set) of the wall patches
  int nwtiles[2] = {0, 0};
  float* d_wplanes = nullptr;             // 6 planes: theta, d1 theta, d2 theta, and reverse-mode scratch
  float* d_wall_c = nullptr;              // Neumann boundary-value weights c[0..d-1]
  float wall_g1 = 0.4f;
  InterpDev* d_interp = nullptr;          // inter-patch interpolation table (fcsd_set_interp)
  int ninterp = 0;
  OvlTarget* d_ovl = nullptr;             // smoothing operator across those patches
  long long* d_ovl_src = nullptr;
  int novl = 0;
  float2* d_ks = nullptr;                 // initial-data smearing filter factors (fcsd_smear)
  int* d_ksoff[2] = {nullptr, nullptr};   // per direction and plan: offset of the plan's factors
  double ks_alpha = -1.0;
  int ks_p = -1;
  double* d_aq = nullptr;
  double* d_dq = nullptr;
  float* d_gq = nullptr;                  // fold matrices of the transposed derivatives, per (N, C)
  float* d_gf = nullptr;                  // fold matrices of the transposed filter (fcsd_set_filter)
  PatchDev* d_patches = nullptr;
  ChunkDev* d_chunks = nullptr;
  int nchunks = 0;
  std::vector<int> patch_chunk_begin;
  LatDev* d_lats = nullptr;
  ChunkDev* d_lchunks = nullptr;
  int nlchunks = 0;
  LatTile* d_ltiles = nullptr;            // column tiles of the lattices (J-direction window sums)
  int nltiles = 0;
  long long lat_size = 0;
  int annulus = 0;
  AnnulusDev an{};
  std::vector<GraphEntry> graphs;

  int layout = FCSD_LAYOUT_ROWS;

  int tile_order = FCSD_ORDER_XCD;

  // schedule of a stage's line passes (FCSD_SCHED_*) and the persistent
  // stage kernel's task queue
  int schedule = FCSD_SCHED_FUSED;
  int2* d_tasks = nullptr;
  int ntasks = 0;
  unsigned* d_ctr = nullptr;              // queue head, 2 npatch counters, then the error word
  unsigned* d_need = nullptr;             // 2 npatch: A tiles, B tiles per patch
  unsigned stage_grid = 0;                // resident workgroups of the persistent launch
  size_t stage_lds = 0;
  int stage_threads = 0;
  bool wide_ok = false;                   // the q2 tiles of four complex lines per grid line fit the LDS
  bool a_wide = false;                    // pass A on the q1 tiles of two complex lines per grid line
};

namespace {

fcsd_status rebuild_wall_tiles(fcsd_set* s);

fcsd_status fail(fcsd_ctx* c, fcsd_status s, const std::string& m) {
  if (c) c->err = m;
  return s;
}

#define HIPCHK(ctx, call)                                                               \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(ctx, FCSD_EHIP, std::string(#call ": ") + hipGetErrorString(e_));    \
  } while (0)

template <class T>
fcsd_status upload(fcsd_ctx* ctx, T** dst, const std::vector<T>& v) {
  *dst = nullptr;
  if (v.empty()) return FCSD_OK;
  HIPCHK(ctx, hipMalloc((void**)dst, v.size() * sizeof(T)));
  HIPCHK(ctx, hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return FCSD_OK;
}

fcsd_status launch_check(fcsd_ctx* ctx, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(ctx, FCSD_EHIP, std::string(what) + ": " + hipGetErrorString(e));
  return FCSD_OK;
}

PassArgs base_args(const fcsd_set* s, int dir) {
  PassArgs a;
  memset(&a, 0, sizeof(a));
  a.plans = s->dir[dir - 1].d_plans;
  a.tiles = s->dir[dir - 1].ts[0].d_tiles;
  a.tw = s->d_tw;
  a.km = s->d_km;
  a.kf = s->d_kf;
  a.aq = s->d_aq;
  a.dq = s->d_dq;
  a.gq = s->d_gq;
  a.gf = s->d_gf;
  a.d = s->d;
  a.plane = s->plane;
  return a;
}

void set_ref(PassArgs& a, const float ref[4], float gamma) {
  a.gamma = gamma;
  for (int k = 0; k < 4; ++k) a.pref[k] = ref[k];
  const double r = ref[0], u = ref[1], v = ref[2], p = ref[3];
  a.eref[0] = (float)r;
  a.eref[1] = (float)(r * u);
  a.eref[2] = (float)(r * v);
  a.eref[3] = (float)(p / (gamma - 1.0) + 0.5 * r * (u * u + v * v));
}

unsigned blocks_for(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }
unsigned chunk_grid(int nchunks) { return (unsigned)std::max(1, std::min(nchunks, kChunkGrid)); }

// launch a line-engine kernel over the batched tile list or one patch's tiles
template <class K>
fcsd_status launch_lines(const fcsd_set* s, int dir, K kern, PassArgs a, int patch = -1, int fields = 1) {
  const TileSet& D = s->dir[dir - 1].ts[fields == 4 ? 2 : fields - 1];
  unsigned grid;
  size_t lds;
  if (patch < 0) {
    a.tiles = D.d_tiles;
    grid = (unsigned)D.tiles.size();
    lds = D.lds;
  } else {
    a.tiles = D.d_tiles_bp + D.patch_begin[patch];
    grid = (unsigned)(D.patch_begin[patch + 1] - D.patch_begin[patch]);
    lds = D.patch_lds[patch];
  }
  if (grid == 0) return FCSD_OK;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(D.threads), lds, s->ctx->stream, a);
  return launch_check(s->ctx, "line kernel");
}

fcsd_status check_set(fcsd_ctx* ctx, const fcsd_set* s, int64_t plane) {
  if (!ctx) return FCSD_EINVAL;
  if (!s) return fail(ctx, FCSD_EINVAL, "null patch set");
  if (s->ctx != ctx) return fail(ctx, FCSD_EINVAL, "patch set belongs to another context");
  if (plane != s->plane) return fail(ctx, FCSD_EINVAL, "plane size differs from the patch set's");
  return FCSD_OK;
}

// elements of a patch's storage (blocked: padded to whole 8x4 blocks)
long long patch_storage(int n1, int n2, int layout) {
  if (layout == FCSD_LAYOUT_B8X4) return (long long)((n1 + 7) & ~7) * ((n2 + 3) & ~3);
  return (long long)n1 * n2;
}

// step reverse mode: 5 stage inputs (20), forward registers (8), cotangents
// of the stage output, stage input, step input, acc and rhs (20), mu_bar (1),
// the right-hand-side reverse workspace (24) and the viscosity one (11)
constexpr size_t kStepAdjPlanes = 20 + 8 + 20 + 1 + 24 + 11;

size_t ws_planes(const fcsd_set* s, int op) {
  switch (op) {
    case FCSD_WS_RHS: return 16;
    case FCSD_WS_AV: return 11;
    case FCSD_WS_STEP: return 16 + 12 + 11;
    case FCSD_WS_RHS_ADJ: return 24;
    case FCSD_WS_STEP_ADJ: return kStepAdjPlanes;
    case FCSD_WS_FILTER_ADJ: return 8;
    case FCSD_WS_SMEAR: return 2;
    case FCSD_WS_STAGE_ADJ: return 24 + 4;   // right-hand-side reverse workspace, rhs_bar
    default: return 0;
  }
}

size_t ws_bytes_of(const fcsd_set* s, int op) {
  size_t b = ws_planes(s, op) * (size_t)s->plane * sizeof(float);
  if (op == FCSD_WS_AV || op == FCSD_WS_STEP || op == FCSD_WS_STEP_ADJ)
    b += 2 * sizeof(unsigned) * (size_t)(s->npatch + 64);
  return b;
}

}  // namespace

// ======================================================================== context

extern "C" fcsd_status fcsd_ctx_create(int device, void* stream, fcsd_ctx** out) {
  if (!out) return FCSD_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return FCSD_EDEVICE;
  if (device < 0 || device >= n) return FCSD_EINVAL;
  std::unique_ptr<fcsd_ctx> c(new fcsd_ctx);
  c->device = device;
  if (device >= kMaxDevices) return FCSD_EUNSUPPORTED;
  if (hipSetDevice(device) != hipSuccess) return FCSD_EDEVICE;
  if (scratch_address(device, &c->scratch) != hipSuccess) return FCSD_EHIP;
  if (stream) {
    c->stream = (hipStream_t)stream;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) return FCSD_EHIP;
    c->own_stream = true;
  }
  if (hipDeviceSynchronize() != hipSuccess) return FCSD_EHIP;
  *out = c.release();
  return FCSD_OK;
}

extern "C" fcsd_status fcsd_ctx_destroy(fcsd_ctx* ctx) {
  if (!ctx) return FCSD_EINVAL;
  if (ctx->own_stream) hipStreamDestroy(ctx->stream);
  delete ctx;
  return FCSD_OK;
}

extern "C" fcsd_status fcsd_ctx_set_stream(fcsd_ctx* ctx, void* stream) {
  if (!ctx) return FCSD_EINVAL;
  if (ctx->own_stream) hipStreamDestroy(ctx->stream);
  ctx->own_stream = false;
  ctx->stream = (hipStream_t)stream;
  return FCSD_OK;
}

extern "C" void* fcsd_ctx_stream(fcsd_ctx* ctx) { return ctx ? (void*)ctx->stream : nullptr; }

extern "C" fcsd_status fcsd_ctx_sync(fcsd_ctx* ctx) {
  if (!ctx) return FCSD_EINVAL;
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  return FCSD_OK;
}

extern "C" const char* fcsd_last_error(const fcsd_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

extern "C" const char* fcsd_version(void) { return "fcsdnn 0.1 gfx950"; }

// ======================================================================== host-only helpers

extern "C" fcsd_status fcsd_fc_matrix(int d, int C, double* out) {
  if (!out || d < 1 || d > 8 || C < 1 || C > 256) return FCSD_EINVAL;
  return fcsd_host_fc_matrix(d, C, out) == 0 ? FCSD_OK : FCSD_EUNSUPPORTED;
}

extern "C" fcsd_status fcsd_fft_plan(int L, int* nst, int rad[8]) {
  if (!nst || !rad || L < 2) return FCSD_EINVAL;
  int k = fcsd_host_factor(L, rad);
  *nst = k;
  return k ? FCSD_OK : FCSD_EUNSUPPORTED;
}

// Validate a patch table without a device (also used by fcsd_set_create).
namespace {
// Longest transform of a line (an extension of up to 4096 + 256 points, or
// the embedding of a circulant whose extension length has a prime factor
// above 13).
constexpr int kMaxTransform = 8192;

// Transform length of a line of N points with C continuation points: the
// extension length N + C when it has a radix plan, else the embedding length
// of its circulant (the smallest 13-smooth length >= N + (N + C) with a plan,
// see fcmat.cpp); 0 if none.
int transform_length(int N, int C) {
  int rad[8];
  const int Lx = N + C;
  if (Lx <= kMaxTransform && fcsd_host_factor(Lx, rad) > 0) return Lx;
  return fcsd_host_embed_length(N + Lx);
}
}  // namespace

extern "C" fcsd_status fcsd_validate_patches(int npatch, const fcsd_patch_desc* p, int d, int64_t plane,
                                             int ring_sectors, int ring_shells, int layout, char* msg,
                                             int msglen) {
  auto say = [&](const std::string& m) {
    if (msg && msglen > 0) snprintf(msg, (size_t)msglen, "%s", m.c_str());
  };
  if (npatch <= 0 || !p) return say("no patches"), FCSD_EINVAL;
  if (d < 1 || d > 8) return say("d must be in 1..8"), FCSD_EINVAL;
  if (layout != FCSD_LAYOUT_ROWS && layout != FCSD_LAYOUT_B8X4) return say("unknown layout"), FCSD_EINVAL;
  std::vector<std::pair<long long, long long>> iv;
  for (int i = 0; i < npatch; ++i) {
    const fcsd_patch_desc& q = p[i];
    char b[160];
    if (q.n1 < 2 * d + 1 || q.n2 < 2 * d + 1 || q.n1 > 4096 || q.n2 > 4096) {
      snprintf(b, sizeof b, "patch %d: sides must be in [2d+1, 4096]", i);
      return say(b), FCSD_EINVAL;
    }
    if (q.C1 < 0 || q.C2 < 0 || q.C1 > 256 || q.C2 > 256) {
      snprintf(b, sizeof b, "patch %d: C must be in [0, 256]", i);
      return say(b), FCSD_EINVAL;
    }
    const long long store = patch_storage(q.n1, q.n2, layout);
    if (q.off < 0 || q.off + store > plane) {
      snprintf(b, sizeof b, "patch %d lies outside the plane", i);
      return say(b), FCSD_EINVAL;
    }
    if (layout == FCSD_LAYOUT_B8X4 && q.off % 32 != 0) {
      snprintf(b, sizeof b, "patch %d: blocked storage needs an offset that is a multiple of 32", i);
      return say(b), FCSD_EINVAL;
    }
    if (!(q.htilde > 0) || !(q.hhat > 0)) {
      snprintf(b, sizeof b, "patch %d: spacing bounds must be positive", i);
      return say(b), FCSD_EINVAL;
    }
    for (int dir = 0; dir < 2; ++dir) {
      const int N = dir ? q.n2 : q.n1, C = dir ? q.C2 : q.C1;
      const int L = transform_length(N, C);
      if (L == 0 || L > kMaxTransform) {
        snprintf(b, sizeof b,
                 "patch %d: extension length %d has a prime factor above 13 and no embedding of length <= %d",
                 i, N + C, kMaxTransform);
        return say(b), FCSD_EUNSUPPORTED;
      }
    }
    iv.push_back({q.off, q.off + store});
  }
  std::sort(iv.begin(), iv.end());
  for (size_t i = 1; i < iv.size(); ++i)
    if (iv[i].first < iv[i - 1].second) return say("patches overlap in the plane"), FCSD_EINVAL;
  if (ring_sectors < 0 || ring_shells < 0) return say("negative ring layout"), FCSD_EINVAL;
  if (ring_sectors > 0) {
    if (ring_shells <= 0 || ring_sectors * ring_shells != npatch)
      return say("ring layout must cover all patches"), FCSD_EINVAL;
    for (int i = 0; i < npatch; ++i)
      if (p[i].n1 != p[0].n1 || p[i].n2 != p[0].n2 || p[0].n1 < 2 * kOvl || p[0].n2 < 2 * kOvl)
        return say("ring patches must share n1, n2 >= 38"), FCSD_EINVAL;
  }
  return FCSD_OK;
}

namespace {

size_t default_lds_budget() {
  const char* e = getenv("FCSD_LDS_BUDGET");
  long v = e ? atol(e) : 0;
  return (v >= 8192 && v <= 160 * 1024) ? (size_t)v : kLdsBudget;
}

// Split every patch's lines into tiles that fit `budget` bytes of LDS
// (lines + twiddle and multiplier tables), balanced per patch, and order the
// batched list longest-first.
// Workgroups of a launch go to the accelerator dies (XCDs, each with its own
// L2) round-robin by workgroup index.
constexpr int kXcd = 8;

void build_tileset(const std::vector<PlanDev>& plans, TileSet& D, size_t budget, int order, int fields, int align,
                   int d) {
  D.tiles_by_patch.clear();
  D.patch_begin.assign(1, 0);
  D.patch_lds.clear();
  D.lds = 0;
  std::vector<long long> pcost;
  for (size_t p = 0; p < plans.size(); ++p) {
    const PlanDev& P = plans[p];
    // LDS: lines (L x ld), twiddle and multiplier tables (2 L), end samples (2d x ld)
    const size_t tables = (size_t)P.L * 2 * sizeof(float2);
    const size_t per_ld = sizeof(float2) * ((size_t)P.L + 2 * (size_t)d);
    int nlmax = budget > tables ? (int)((budget - tables) / per_ld) - 1 : 1;
    nlmax = std::max(1, std::min(kMaxTile, nlmax)) / fields;
    nlmax = std::max(align, nlmax / align * align);  // blocked storage: tiles start on block edges
    const int nt = (P.nlines + nlmax - 1) / nlmax;
    const int nl = ((P.nlines + nt - 1) / nt + align - 1) / align * align;
    size_t plds = 0;
    long long cost = 0;
    for (int t = 0; t < nt; ++t) {
      TileDev T;
      T.plan = (int)p;
      T.line0 = t * nl;
      T.nl = std::min(nl, P.nlines - T.line0);
      if (T.nl <= 0) continue;
      // odd row stride (the line-fastest FFT accesses and the position-fastest
      // loads both free of LDS bank conflicts), or the even one when only
      // that keeps the tile within the budget: two workgroups per CU instead
      // of one are worth far more than the conflicts (the q2 tiles of two
      // complex lines per grid line on the longest lines: 83 KB odd, 79 KB even)
      T.ld = (fields * T.nl) | 1;
      if (per_ld * T.ld + tables > budget && per_ld * (fields * T.nl) + tables <= budget) T.ld = fields * T.nl;
      D.tiles_by_patch.push_back(T);
      plds = std::max(plds, per_ld * T.ld + tables);
      cost += (long long)P.L * T.nl;
    }
    D.patch_begin.push_back((int)D.tiles_by_patch.size());
    D.patch_lds.push_back(plds);
    D.lds = std::max(D.lds, plds);
    pcost.push_back(cost);
  }
  if (order == FCSD_ORDER_LPT) {
    // longest tile first over all patches
    D.tiles = D.tiles_by_patch;
    std::stable_sort(D.tiles.begin(), D.tiles.end(), [&](const TileDev& a, const TileDev& b) {
      const PlanDev &pa = plans[a.plan], &pb = plans[b.plan];
      return (long long)pa.L * a.nl > (long long)pb.L * b.nl;
    });
    return;
  }
  // XCD-grouped: patches are dealt to the dies by longest-first greedy
  // balancing of their work, so that the tiles of one patch, which share
  // cache lines at their column edges (q2 lines) and metric rows, run on one
  // L2.  A patch with more work than a die's fair share (few large patches)
  // is first cut into runs of consecutive tiles of about that share, so
  // that every die gets work.  Slot b of the launch belongs to die b % kXcd;
  // dies with fewer tiles get empty tiles (nl = 0, the kernels return at
  // once).
  struct Run {
    int begin, end;
    long long cost;
  };
  long long total = 0;
  for (long long c : pcost) total += c;
  const long long share = std::max(1LL, (total + kXcd - 1) / kXcd);
  std::vector<Run> runs;
  for (int p = 0; p < (int)plans.size(); ++p) {
    const int b = D.patch_begin[p], e = D.patch_begin[p + 1], nt = e - b;
    if (nt == 0) continue;
    const int k = (int)std::min<long long>(nt, (pcost[p] + share - 1) / share);
    for (int i = 0; i < k; ++i) {
      Run r{b + (int)((long long)nt * i / k), b + (int)((long long)nt * (i + 1) / k), 0};
      for (int t = r.begin; t < r.end; ++t) r.cost += (long long)plans[p].L * D.tiles_by_patch[t].nl;
      runs.push_back(r);
    }
  }
  std::stable_sort(runs.begin(), runs.end(), [](const Run& a, const Run& b) { return a.cost > b.cost; });
  std::vector<long long> load(kXcd, 0);
  std::vector<std::vector<TileDev>> lst(kXcd);
  for (const Run& r : runs) {
    const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    load[x] += r.cost;
    for (int t = r.begin; t < r.end; ++t) lst[x].push_back(D.tiles_by_patch[t]);
  }
  size_t mx = 0;
  for (auto& l : lst) mx = std::max(mx, l.size());
  TileDev empty;
  empty.plan = 0;
  empty.line0 = 0;
  empty.nl = 0;
  empty.ld = 1;
  D.tiles.assign(mx * kXcd, empty);
  for (int x = 0; x < kXcd; ++x)
    for (size_t k = 0; k < lst[x].size(); ++k) D.tiles[k * kXcd + x] = lst[x][k];
}

// align: lines per tile a multiple of it (blocked storage: 4 q1 lines, 8 q2 lines)
void build_tiles(DirPlan& D, int order, int align, int d) {
  for (int f = 0; f < 3; ++f) build_tileset(D.plans, D.ts[f], D.ts[f].budget, order, 1 << f, align, d);
}

int tile_align(int layout, int dir) { return layout == FCSD_LAYOUT_B8X4 ? (dir == 0 ? 4 : 8) : 1; }

fcsd_status upload_tiles(fcsd_ctx* ctx, DirPlan& D) {
  for (auto& t : D.ts) {
    (void)hipFree(t.d_tiles);
    (void)hipFree(t.d_tiles_bp);
    t.d_tiles = t.d_tiles_bp = nullptr;
    fcsd_status r;
    if ((r = upload(ctx, &t.d_tiles, t.tiles)) || (r = upload(ctx, &t.d_tiles_bp, t.tiles_by_patch))) return r;
  }
  return FCSD_OK;
}

// Spectral filter factors (alpha, p) of plan P (Sec. 4.3.1, eq. filtering):
// of its extension length, or of its circulant embedded in the longer
// transform (then they also depend on N).
std::tuple<int, int, int> filter_key(const PlanDev& P) {
  return std::make_tuple(P.Lx, P.L, P.L == P.Lx ? 0 : P.N);
}
void filter_table(const PlanDev& P, double alpha, int p, std::vector<float>& t) {
  t.assign(2 * (size_t)P.L, 0.0f);
  if (P.L == P.Lx)
    fcsd_host_fmul(P.L, P.nst, P.rad, alpha, p, t.data());
  else
    fcsd_host_fmul_embedded(P.N, P.Lx, P.L, P.nst, P.rad, alpha, p, t.data());
}

// The set's device error word, after the stage queue's head and per-patch
// counters: bit 0 a persistent stage's dependency wait gave up, bit 1 the
// network's weights let its split fp16 operands leave the fp16 range.
unsigned* set_error_word(const fcsd_set* s) { return s->d_ctr + 1 + 2 * (size_t)s->npatch; }

// Pass A runs on the q1 tiles of two complex lines per grid line (the four
// state fields in one round) when those tiles keep within the q1 tiles' LDS
// (a launch takes its largest tile's LDS; long lines, whose two-line tiles
// need more, would halve the workgroups per CU for the whole pass).
bool pick_a_wide(const fcsd_set* s) {
  const TileSet &one = s->dir[0].ts[0], &two = s->dir[0].ts[1];
  return two.lds <= std::max(one.lds, one.budget);
}

// Task queue of the persistent stage kernel from the current tile sets:
// every A task (q1 tiles in launch order), then the B tasks (q2 tiles with
// two complex lines per grid line) patch by patch in the order in which the
// patches' last A tasks stand in the queue, then the C tasks (q1 tiles)
// patch by patch in the order of the patches' last B tasks, so that the
// tasks taken first are the ones whose inputs are done first.  Also the
// per-patch tile counts, the counters and the launch shape.
fcsd_status build_stage_tasks(fcsd_set* s) {
  fcsd_ctx* ctx = s->ctx;
  const int np = s->npatch;
  const TileSet& TA = s->dir[0].ts[0];
  const TileSet& TB = s->dir[1].ts[1];
  std::vector<int2> tasks;
  std::vector<unsigned> need(2 * (size_t)np, 0u);
  std::vector<long long> lastA(np, -1), lastB(np, -1);
  for (size_t i = 0; i < TA.tiles.size(); ++i) {
    const TileDev& T = TA.tiles[i];
    if (T.nl == 0) continue;
    lastA[T.plan] = (long long)tasks.size();
    ++need[T.plan];
    tasks.push_back(make_int2(TASK_A, (int)i));
  }
  auto by_last = [&](const std::vector<long long>& last) {
    std::vector<int> ord(np);
    for (int p = 0; p < np; ++p) ord[p] = p;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return last[a] < last[b]; });
    return ord;
  };
  std::vector<std::vector<int>> tb(np), ta(np);
  for (size_t i = 0; i < TB.tiles.size(); ++i)
    if (TB.tiles[i].nl > 0) tb[TB.tiles[i].plan].push_back((int)i);
  for (size_t i = 0; i < TA.tiles.size(); ++i)
    if (TA.tiles[i].nl > 0) ta[TA.tiles[i].plan].push_back((int)i);
  for (int p : by_last(lastA))
    for (int i : tb[p]) {
      lastB[p] = (long long)tasks.size();
      ++need[np + p];
      tasks.push_back(make_int2(TASK_B, i));
    }
  for (int p : by_last(lastB))
    for (int i : ta[p]) tasks.push_back(make_int2(TASK_C, i));
  (void)hipFree(s->d_tasks);
  (void)hipFree(s->d_need);
  s->d_tasks = nullptr;
  s->d_need = nullptr;
  fcsd_status r;
  if ((r = upload(ctx, &s->d_tasks, tasks)) || (r = upload(ctx, &s->d_need, need))) return r;
  s->ntasks = (int)tasks.size();
  if (!s->d_ctr) {
    const size_t words = 2 + 2 * (size_t)np;
    HIPCHK(ctx, hipMalloc(&s->d_ctr, words * sizeof(unsigned)));
    HIPCHK(ctx, hipMemset(s->d_ctr, 0, words * sizeof(unsigned)));
  }
  // launch shape: the q1 set's workgroup size, the larger LDS of the two
  // sets plus the queue slot, as many workgroups as can be resident
  s->stage_threads = TA.threads;
  s->stage_lds = std::max(TA.lds, TB.lds) + 16;
  s->stage_grid = 0;
  int maxlds = 0, ncu = 0, per_cu = 0;
  HIPCHK(ctx, hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device));
  if (s->stage_lds > (size_t)maxlds) return FCSD_OK;  // the persistent schedule cannot run with these tiles
  HIPCHK(ctx, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ctx->device));
  HIPCHK(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_stage, s->stage_threads, s->stage_lds));
  s->stage_grid = (unsigned)std::max(0, std::min(s->ntasks, per_cu * ncu));
  return FCSD_OK;
}

}  // namespace

// ======================================================================== patch set

extern "C" fcsd_status fcsd_set_create(fcsd_ctx* ctx, int npatch, const fcsd_patch_desc* patches, int d,
                                       int64_t plane, int ring_sectors, int ring_shells, int layout,
                                       fcsd_set** out) {
  if (!ctx || !out) return FCSD_EINVAL;
  *out = nullptr;
  char msg[256] = {0};
  fcsd_status st = fcsd_validate_patches(npatch, patches, d, plane, ring_sectors, ring_shells, layout, msg, 256);
  if (st != FCSD_OK) return fail(ctx, st, msg);
  HIPCHK(ctx, hipSetDevice(ctx->device));
  std::unique_ptr<fcsd_set> s(new fcsd_set);
  s->ctx = ctx;
  s->npatch = npatch;
  s->d = d;
  s->plane = plane;
  s->layout = layout;
  s->desc.assign(patches, patches + npatch);
  // pools
  std::vector<float2> tw;
  std::vector<float2> km;
  std::vector<double> aq, dq;
  std::vector<float> gq;
  std::map<int, int> tw_of_L, aq_of_C, dq_of_C;
  std::map<std::pair<int, int>, int> gq_of;
  std::map<std::tuple<int, int, int, int>, int> km_of;
  for (int dir = 1; dir <= 2; ++dir) {
    DirPlan& D = s->dir[dir - 1];
    long long eo = 0;
    for (int p = 0; p < npatch; ++p) {
      const fcsd_patch_desc& q = patches[p];
      PlanDev P;
      memset(&P, 0, sizeof(P));
      P.N = dir == 1 ? q.n1 : q.n2;
      P.C = dir == 1 ? q.C1 : q.C2;
      P.Lx = P.N + P.C;
      P.L = transform_length(P.N, P.C);
      P.periodic = P.C == 0;
      P.nst = fcsd_host_factor(P.L, P.rad);
      P.nlines = dir == 1 ? q.n2 : q.n1;
      P.n1 = q.n1;
      P.n2 = q.n2;
      P.patch = p;
      P.nb1 = layout == FCSD_LAYOUT_B8X4 ? (q.n1 + 7) >> 3 : 0;
      P.off = q.off;
      if (!tw_of_L.count(P.L)) {
        tw_of_L[P.L] = (int)tw.size();
        std::vector<float> t(2 * P.L);
        fcsd_host_twiddles(P.L, t.data());
        for (int n = 0; n < P.L; ++n) tw.push_back(make_float2(t[2 * n], t[2 * n + 1]));
      }
      P.tw = tw_of_L[P.L];
      auto key = std::make_tuple(P.N, P.L, P.periodic, P.Lx);
      if (!km_of.count(key)) {
        km_of[key] = (int)km.size();
        std::vector<float> t(2 * P.L);
        if (P.L == P.Lx)
          fcsd_host_kmul(P.N, P.L, P.nst, P.rad, t.data(), P.periodic);
        else  // the circulant of the extension, embedded in the longer transform
          fcsd_host_kmul_embedded(P.N, P.Lx, P.L, P.nst, P.rad, t.data(), P.periodic);
        for (int n = 0; n < P.L; ++n) km.push_back(make_float2(t[2 * n], t[2 * n + 1]));
      }
      P.km = km_of[key];
      if (!P.periodic) {
        if (!aq_of_C.count(P.C)) {
          aq_of_C[P.C] = (int)aq.size();
          std::vector<double> m((size_t)P.C * d);
          if (fcsd_host_fc_matrix(d, P.C, m.data()) != 0)
            return fail(ctx, FCSD_EUNSUPPORTED, "continuation fit failed");
          aq.insert(aq.end(), m.begin(), m.end());
          dq_of_C[P.C] = (int)dq.size();
          std::vector<double> r((size_t)(P.C + 1) * 2 * d);
          if (fcsd_host_fc_dmatrix(d, P.C, r.data()) != 0)
            return fail(ctx, FCSD_EUNSUPPORTED, "continuation fit failed");
          dq.insert(dq.end(), r.begin(), r.end());
        }
        P.aq = aq_of_C[P.C];
        P.dq = dq_of_C[P.C];
        const auto gkey = std::make_pair(P.N, P.C);
        if (!gq_of.count(gkey)) {
          gq_of[gkey] = (int)gq.size();
          std::vector<double> g((size_t)P.N * 2 * d);
          if (fcsd_host_fold_matrix(P.N, P.C, d, aq.data() + P.aq, 0, 0.0, 0, g.data()) != 0)
            return fail(ctx, FCSD_EUNSUPPORTED, "fold matrix of the transposed derivative failed");
          for (double v : g) gq.push_back((float)v);
        }
        P.gq = gq_of[gkey];
      }
      D.plans.push_back(P);
      D.ext_off.push_back(eo);
      eo += (long long)P.nlines * P.Lx;
    }
    D.ext_plane = eo;
  }
  for (int dir = 0; dir < 2; ++dir) {
    for (auto& t : s->dir[dir].ts) t.budget = default_lds_budget();
    build_tiles(s->dir[dir], s->tile_order, tile_align(layout, dir), d);
  }
  {
    // the smallest tiles (one storage-aligned group of lines) must fit the LDS
    int maxlds = 0;
    HIPCHK(ctx, hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device));
    for (int dir = 0; dir < 2; ++dir)
      for (int f = 0; f < 2; ++f)
        if (s->dir[dir].ts[f].lds > (size_t)maxlds)
          return fail(ctx, FCSD_EUNSUPPORTED,
                      "a line tile needs more LDS than a workgroup has (transform length too long for the "
                      "storage's smallest tile)");
    // the wide fused q2 pass (four complex lines per grid line) is optional
    s->wide_ok = s->dir[1].ts[2].lds <= (size_t)maxlds;
    s->a_wide = pick_a_wide(s.get());
  }
  // per-patch descriptors and point chunks
  std::vector<PatchDev> pd;
  std::vector<ChunkDev> ch;
  for (int p = 0; p < npatch; ++p) {
    const fcsd_patch_desc& q = patches[p];
    PatchDev P;
    P.n1 = q.n1;
    P.n2 = q.n2;
    P.off = q.off;
    P.hhat = (float)q.hhat;
    P.htilde = (float)q.htilde;
    P.internal = (q.internal[0] ? 1 : 0) | (q.internal[1] ? 2 : 0) | (q.internal[2] ? 4 : 0) | (q.internal[3] ? 8 : 0);
    P.nb1 = layout == FCSD_LAYOUT_B8X4 ? (q.n1 + 7) >> 3 : 0;
    pd.push_back(P);
    s->patch_chunk_begin.push_back((int)ch.size());
    const long long store = patch_storage(q.n1, q.n2, layout);
    for (long long k = 0; k < store; k += kChunk) ch.push_back(ChunkDev{p, (int)k});
    s->npoints += (long long)q.n1 * q.n2;
  }
  s->patch_chunk_begin.push_back((int)ch.size());
  s->nchunks = (int)ch.size();
  // smoothing-blending lattice
  std::vector<LatDev> lat;
  std::vector<ChunkDev> lch;
  if (ring_sectors > 0) {
    s->annulus = 1;
    AnnulusDev& A = s->an;
    A.nsec = ring_sectors;
    A.nshell = ring_shells;
    A.n1 = patches[0].n1;
    A.n2 = patches[0].n2;
    A.st1 = A.n1 - kOvl;
    A.st2 = A.n2 - kOvl;
    A.ring = A.nsec * A.st1;
    A.nJ = A.nshell * A.st2 + kOvl;
    LatDev Lt{A.ring, A.nJ, 1, 0, 0};
    lat.push_back(Lt);
    for (long long k = 0; k < (long long)A.ring * A.nJ; k += kChunk) lch.push_back(ChunkDev{0, (int)k});
    s->lat_size = (long long)A.ring * A.nJ;
    if (s->lat_size > plane) return fail(ctx, FCSD_EINVAL, "annulus lattice larger than a plane");
  } else {
    for (int p = 0; p < npatch; ++p) {
      LatDev Lt{patches[p].n1, patches[p].n2, 0, 0, patches[p].off};
      lat.push_back(Lt);
    }
    lch = ch;
    s->lat_size = plane;
  }
  s->nlchunks = (int)lch.size();
  std::vector<LatTile> ltiles;
  for (int li = 0; li < (int)lat.size(); ++li)
    for (int j0 = 0; j0 < lat[li].H; j0 += kLatRows)
      for (int g0 = 0; g0 < lat[li].W; g0 += kBlock) ltiles.push_back(LatTile{li, g0, j0, 0});
  s->nltiles = (int)ltiles.size();
  fcsd_status r;
  if ((r = upload(ctx, &s->d_tw, tw)) || (r = upload(ctx, &s->d_km, km)) || (r = upload(ctx, &s->d_aq, aq)) ||
      (r = upload(ctx, &s->d_dq, dq)) || (r = upload(ctx, &s->d_gq, gq)) ||
      (r = upload(ctx, &s->d_patches, pd)) || (r = upload(ctx, &s->d_chunks, ch)) ||
      (r = upload(ctx, &s->d_lats, lat)) || (r = upload(ctx, &s->d_lchunks, lch)) ||
      (r = upload(ctx, &s->d_ltiles, ltiles)))
    return r;
  if (aq.empty()) {  // keep a valid pointer for kernels
    std::vector<double> one(1, 0.0);
    std::vector<float> onef(1, 0.f);
    if ((r = upload(ctx, &s->d_aq, one)) || (r = upload(ctx, &s->d_dq, one)) || (r = upload(ctx, &s->d_gq, onef)))
      return r;
  }
  for (int dir = 0; dir < 2; ++dir) {
    DirPlan& D = s->dir[dir];
    if ((r = upload(ctx, &D.d_plans, D.plans)) || (r = upload_tiles(ctx, D)) ||
        (r = upload(ctx, &D.d_ext_off, D.ext_off)))
      return r;
  }
  if ((r = build_stage_tasks(s.get()))) return r;
  HIPCHK(ctx, hipDeviceSynchronize());
  *out = s.release();
  return FCSD_OK;
}

extern "C" fcsd_status fcsd_set_destroy(fcsd_set* s) {
  if (!s) return FCSD_EINVAL;
  hipStreamSynchronize(s->ctx->stream);
  for (auto& g : s->graphs)
    if (g.exec) hipGraphExecDestroy(g.exec);
  for (int dir = 0; dir < 2; ++dir) {
    (void)hipFree(s->dir[dir].d_plans);
    for (auto& t : s->dir[dir].ts) {
      (void)hipFree(t.d_tiles);
      (void)hipFree(t.d_tiles_bp);
    }
    (void)hipFree(s->dir[dir].d_ext_off);
  }
  hipFree(s->d_tw);
  hipFree(s->d_km);
  hipFree(s->d_kf);
  hipFree(s->d_walls);
  hipFree(s->d_wall_c);
  hipFree(s->d_wchunks);
  hipFree(s->d_wtiles[0]);
  hipFree(s->d_wtiles[1]);
  hipFree(s->d_wplanes);
  hipFree(s->d_interp);
  hipFree(s->d_ovl);
  hipFree(s->d_ovl_src);
  hipFree(s->d_ks);
  hipFree(s->d_ksoff[0]);
  hipFree(s->d_ksoff[1]);
  hipFree(s->d_aq);
  hipFree(s->d_dq);
  hipFree(s->d_gq);
  hipFree(s->d_gf);
  hipFree(s->d_patches);
  hipFree(s->d_chunks);
  hipFree(s->d_lats);
  hipFree(s->d_lchunks);
  hipFree(s->d_ltiles);
  hipFree(s->d_tasks);
  hipFree(s->d_need);
  hipFree(s->d_ctr);
  delete s;
  return FCSD_OK;
}

extern "C" fcsd_status fcsd_set_tune(fcsd_set* s, const int lds_budget[3], const int threads[3], int order) {
  if (!s || !lds_budget || !threads) return FCSD_EINVAL;
  fcsd_ctx* ctx = s->ctx;
  int maxlds = 0;
  HIPCHK(ctx, hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device));
  for (int k = 0; k < 3; ++k) {
    if (lds_budget[k] < 8192 || lds_budget[k] > 160 * 1024)
      return fail(ctx, FCSD_EINVAL, "fcsd_set_tune: budget must be in [8 KB, 160 KB]");
    if (lds_budget[k] > maxlds)
      return fail(ctx, FCSD_EINVAL, "fcsd_set_tune: budget above the device's LDS per workgroup");
    const int t = threads[k];
    if (t != 64 && t != 128 && t != 256 && t != 512 && t != 1024)
      return fail(ctx, FCSD_EINVAL, "fcsd_set_tune: threads must be 64, 128, 256, 512 or 1024");
  }
  if (order != FCSD_ORDER_LPT && order != FCSD_ORDER_XCD) return fail(ctx, FCSD_EINVAL, "fcsd_set_tune: bad order");
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  for (auto& g : s->graphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  s->graphs.clear();
  s->tile_order = order;
  // tile sets: q1 lines; q2 lines; q2 lines with two complex lines per grid line
  s->dir[0].ts[0].budget = (size_t)lds_budget[0];
  s->dir[0].ts[0].threads = threads[0];
  s->dir[0].ts[1].budget = (size_t)lds_budget[0];
  s->dir[0].ts[1].threads = threads[0];
  s->dir[1].ts[0].budget = (size_t)lds_budget[1];
  s->dir[1].ts[0].threads = threads[1];
  s->dir[1].ts[1].budget = (size_t)lds_budget[2];
  s->dir[1].ts[1].threads = threads[2];
  s->dir[0].ts[2].budget = (size_t)lds_budget[0];
  s->dir[0].ts[2].threads = threads[0];
  s->dir[1].ts[2].budget = (size_t)lds_budget[2];
  s->dir[1].ts[2].threads = threads[2];
  fcsd_status r;
  for (int dir = 0; dir < 2; ++dir) {
    DirPlan& D = s->dir[dir];
    build_tiles(D, order, tile_align(s->layout, dir), s->d);
    if (dir == 1) {
      // q2 tiles of four complex lines per grid line (the wide fused pass,
      // the reverse mode's q2 pass): when their tiles exceed the third
      // budget (its smallest storage-aligned tiles do not fit), they are
      // built for the device's whole LDS with 1024-thread workgroups
      TileSet& W = D.ts[2];
      if (W.lds > W.budget && W.budget < (size_t)maxlds) {
        W.budget = (size_t)maxlds;
        W.threads = 1024;
        build_tileset(D.plans, W, W.budget, order, 4, tile_align(s->layout, dir), s->d);
      }
    }
    if ((r = upload_tiles(ctx, D))) return r;
  }
  if ((r = build_stage_tasks(s))) return r;
  s->wide_ok = s->dir[1].ts[2].lds <= (size_t)maxlds;
  s->a_wide = pick_a_wide(s);
  if ((s->schedule == FCSD_SCHED_PERSISTENT && s->stage_grid == 0) ||
      (s->schedule == FCSD_SCHED_FUSED_WIDE && !s->wide_ok))
    s->schedule = FCSD_SCHED_FUSED;
  return rebuild_wall_tiles(s);
}

extern "C" fcsd_status fcsd_set_schedule(fcsd_set* s, int schedule) {
  if (!s) return FCSD_EINVAL;
  fcsd_ctx* ctx = s->ctx;
  if (schedule != FCSD_SCHED_SPLIT && schedule != FCSD_SCHED_FUSED && schedule != FCSD_SCHED_PERSISTENT &&
      schedule != FCSD_SCHED_FUSED_WIDE)
    return fail(ctx, FCSD_EINVAL, "fcsd_set_schedule: unknown schedule");
  if (schedule == FCSD_SCHED_PERSISTENT && s->stage_grid == 0)
    return fail(ctx, FCSD_EINVAL,
                "fcsd_set_schedule: the tile sets leave no room for the persistent kernel's queue slot "
                "(tune LDS budgets to at most 160 KB - 16)");
  if (schedule == FCSD_SCHED_FUSED_WIDE && !s->wide_ok)
    return fail(ctx, FCSD_EINVAL, "fcsd_set_schedule: q2 tiles of four complex lines per grid line do not fit the LDS");
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  for (auto& g : s->graphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  s->graphs.clear();
  s->schedule = schedule;
  return FCSD_OK;
}

extern "C" fcsd_status fcsd_stage_errors(fcsd_set* s, int32_t* flags) {
  if (!s || !flags) return FCSD_EINVAL;
  fcsd_ctx* ctx = s->ctx;
  unsigned* e = set_error_word(s);
  unsigned v = 0;
  HIPCHK(ctx, hipMemcpyAsync(&v, e, sizeof(v), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipMemsetAsync(e, 0, sizeof(v), ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  *flags = (int32_t)v;
  return FCSD_OK;
}

extern "C" fcsd_status fcsd_set_filter(fcsd_set* s, double alpha, int p) {
  if (!s) return FCSD_EINVAL;
  fcsd_ctx* ctx = s->ctx;
  if (!(alpha >= 0.0) || !std::isfinite(alpha) || p < 2 || p > 64 || p % 2)
    return fail(ctx, FCSD_EINVAL, "fcsd_set_filter: need alpha >= 0 finite and an even p in [2, 64]");
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  for (auto& g : s->graphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  s->graphs.clear();
  std::vector<float2> kf;
  std::map<std::tuple<int, int, int>, int> kf_of_L;
  std::vector<float> gf;
  std::map<std::pair<int, int>, int> gf_of;
  std::map<int, std::vector<double>> aq_of_C;
  for (int dir = 0; dir < 2; ++dir)
    for (PlanDev& P : s->dir[dir].plans) {
      const auto fkey = filter_key(P);
      if (!kf_of_L.count(fkey)) {
        kf_of_L[fkey] = (int)kf.size();
        std::vector<float> t;
        filter_table(P, alpha, p, t);
        for (int n = 0; n < P.L; ++n) kf.push_back(make_float2(t[2 * n], t[2 * n + 1]));
      }
      P.kf = kf_of_L[fkey];
      if (P.periodic) continue;
      const auto key = std::make_pair(P.N, P.C);
      if (!gf_of.count(key)) {
        if (!aq_of_C.count(P.C)) {
          std::vector<double> m((size_t)P.C * s->d);
          if (fcsd_host_fc_matrix(s->d, P.C, m.data()) != 0)
            return fail(ctx, FCSD_EUNSUPPORTED, "continuation fit failed");
          aq_of_C[P.C] = m;
        }
        gf_of[key] = (int)gf.size();
        std::vector<double> g((size_t)P.N * 2 * s->d);
        if (fcsd_host_fold_matrix(P.N, P.C, s->d, aq_of_C[P.C].data(), 1, alpha, p, g.data()) != 0)
          return fail(ctx, FCSD_EUNSUPPORTED, "fold matrix of the transposed filter failed");
        for (double v : g) gf.push_back((float)v);
      }
      P.gf = gf_of[key];
    }
  if (gf.empty()) gf.push_back(0.f);
  (void)hipFree(s->d_kf);
  s->d_kf = nullptr;
  (void)hipFree(s->d_gf);
  s->d_gf = nullptr;
  s->filter_on = 0;
  fcsd_status r;
  if ((r = upload(ctx, &s->d_kf, kf)) || (r = upload(ctx, &s->d_gf, gf))) return r;
  for (int dir = 0; dir < 2; ++dir) {
    DirPlan& D = s->dir[dir];
    (void)hipFree(D.d_plans);
    if ((r = upload(ctx, &D.d_plans, D.plans))) return r;
  }
  s->filter_on = 1;
  s->filter_alpha = alpha;
  s->filter_p = p;
  return FCSD_OK;
}

extern "C" fcsd_status fcsd_workspace_size(const fcsd_set* s, int op, size_t* bytes) {
  if (!s || !bytes || op < 0 || op > FCSD_WS_STAGE_ADJ) return FCSD_EINVAL;
  *bytes = ws_bytes_of(s, op);
  return FCSD_OK;
}

extern "C" fcsd_status fcsd_ext_size(const fcsd_set* s, int dir, int64_t* floats) {
  if (!s || !floats || (dir != 1 && dir != 2)) return FCSD_EINVAL;
  *floats = s->dir[dir - 1].ext_plane;
  return FCSD_OK;
}

// ======================================================================== line operators

extern "C" fcsd_status fc_diff(fcsd_ctx* ctx, const fcsd_set* s, int dir, int nf, const float* in, float* out,
                               int64_t plane) {
  fcsd_status st = check_set(ctx, s, plane);
  if (st) return st;
  if ((dir != 1 && dir != 2) || nf < 1 || !in || !out) return fail(ctx, FCSD_EINVAL, "fc_diff: bad arguments");
  if (in == out) return fail(ctx, FCSD_EINVAL, "fc_diff: out aliases in");
  PassArgs a = base_args(s, dir);
  a.nf = nf;
  a.in = in;
  a.out = out;
  return dir == 1 ? launch_lines(s, 1, k_fcdiff<1, false>, a) : launch_lines(s, 2, k_fcdiff<2, false>, a);
}

extern "C" fcsd_status fc_diff_adj(fcsd_ctx* ctx, const fcsd_set* s, int dir, int nf, const float* out_bar,
                                   float* in_bar, int64_t plane) {
  fcsd_status st = check_set(ctx, s, plane);
  if (st) return st;
  if ((dir != 1 && dir != 2) || nf < 1 || !out_bar || !in_bar)
    return fail(ctx, FCSD_EINVAL, "fc_diff_adj: bad arguments");
  if (out_bar == in_bar) return fail(ctx, FCSD_EINVAL, "fc_diff_adj: in_bar aliases out_bar");
  PassArgs a = base_args(s, dir);
  a.nf = nf;
  a.in = out_bar;
  a.out = in_bar;
  return dir == 1 ? launch_lines(s, 1, k_fcdiff<1, true>, a) : launch_lines(s, 2, k_fcdiff<2, true>, a);
}

extern "C" fcsd_status fc_continue(fcsd_ctx* ctx, const fcsd_set* s, int dir, int nf, const float* in,
                                   int64_t plane, float* ext, int64_t ext_plane) {
  fcsd_status st = check_set(ctx, s, plane);
  if (st) return st;
  if ((dir != 1 && dir != 2) || nf < 1 || !in || !ext) return fail(ctx, FCSD_EINVAL, "fc_continue: bad arguments");
  if (ext_plane < s->dir[dir - 1].ext_plane) return fail(ctx, FCSD_EINVAL, "fc_continue: ext_plane too small");
  PassArgs a = base_args(s, dir);
  a.nf = nf;
  a.in = in;
  a.out = ext;
  a.ext_plane = ext_plane;
  a.ext_off = s->dir[dir - 1].d_ext_off;
  return dir == 1 ? launch_lines(s, 1, k_fccont<1, false>, a) : launch_lines(s, 2, k_fccont<2, false>, a);
}

extern "C" fcsd_status fc_continue_adj(fcsd_ctx* ctx, const fcsd_set* s, int dir, int nf, const float* ext_bar,
                                       int64_t ext_plane, float* in_bar, int64_t plane) {
  fcsd_status st = check_set(ctx, s, plane);
  if (st) return st;
  if ((dir != 1 && dir != 2) || nf < 1 || !in_bar || !ext_bar)
    return fail(ctx, FCSD_EINVAL, "fc_continue_adj: bad arguments");
  if (ext_plane < s->dir[dir - 1].ext_plane) return fail(ctx, FCSD_EINVAL, "fc_continue_adj: ext_plane too small");
  PassArgs a = base_args(s, dir);
  a.nf = nf;
  a.in = ext_bar;
  a.out = in_bar;
  a.ext_plane = ext_plane;
  a.ext_off = s->dir[dir - 1].d_ext_off;
  return dir == 1 ? launch_lines(s, 1, k_fccont<1, true>, a) : launch_lines(s, 2, k_fccont<2, true>, a);
}

// ======================================================================== right-hand side

namespace {

struct RhsWs {
  float *d1e, *H, *r2;
};

RhsWs carve_rhs(const fcsd_set* s, void* ws) {
  float* w = (float*)ws;
  const long long pl = s->plane;
  return RhsWs{w, w + 4 * pl, w + 12 * pl};
}

// flux: FLUX_FULL, FLUX_VISC, FLUX_INVISCID ; out: MODE_SET / MODE_ADD / MODE_RK
// Launch a line kernel over an explicit list of n tiles of the
// single-field tile set of direction dir.
template <class K>
fcsd_status launch_tiles(const fcsd_set* s, int dir, K kern, PassArgs a, const TileDev* tiles, int n) {
  if (n == 0) return FCSD_OK;
  const TileSet& D = s->dir[dir - 1].ts[0];
  a.tiles = tiles;
  hipLaunchKernelGGL(kern, dim3((unsigned)n), dim3(D.threads), D.lds, s->ctx->stream, a);
  return launch_check(s->ctx, "line kernel");
}

// The chunks of the wall patches (patch < 0) or of wall patch `patch`.
void wall_chunks(const fcsd_set* s, int patch, const ChunkDev** ch, int* n) {
  if (patch < 0) {
    *ch = s->d_wchunks;
    *n = s->nwchunks;
  } else {
    *ch = s->d_chunks + s->patch_chunk_begin[patch];
    *n = s->patch_chunk_begin[patch + 1] - s->patch_chunk_begin[patch];
  }
}

// theta - theta_ref on the wall patches (or wall patch `patch`) and its FC
// derivatives along q1 and q2, into the set's planes 0, 1, 2 (the energy's
// product rule, Remark adiabatic; ref = (rho, u, v, p) of the reference).
fcsd_status wall_theta_derivs(fcsd_ctx* ctx, const fcsd_set* s, const float* u, const float ref[4], float gamma,
                              int patch) {
  const long long pl = s->plane;
  float* TH = s->d_wplanes;
  const ChunkDev* ch;
  int n;
  wall_chunks(s, patch, &ch, &n);
  hipLaunchKernelGGL(k_theta, dim3(chunk_grid(n)), dim3(kBlock), 0, ctx->stream, ch, n, s->d_patches, u, pl,
                     (double)gamma - 1.0, (double)ref[3] / (double)ref[0], TH);
  fcsd_status st;
  for (int dir = 1; dir <= 2; ++dir) {
    PassArgs a = base_args(s, dir);
    a.in = TH;
    a.out = TH + dir * pl;
    a.nf = 1;
    auto kern = dir == 1 ? k_fcdiff<1, false> : k_fcdiff<2, false>;
    st = patch < 0 ? launch_tiles(s, dir, kern, a, s->d_wtiles[dir - 1], s->nwtiles[dir - 1])
                   : launch_lines(s, dir, kern, a, patch);
    if (st) return st;
  }
  return launch_check(ctx, "wall theta derivatives");
}

fcsd_status rhs_passes(fcsd_ctx* ctx, const fcsd_set* s, const float* u, const float* metric, const float* mu,
                       const float ref[4], float gamma, int flux, int outmode, float* rhs, int stage,
                       const float* u0, float* acc, float* uout, const float* dtp, void* ws, int patch,
                       unsigned passes = 15u, float* d1e_rec = nullptr, float* d2e_rec = nullptr) {
  RhsWs W = carve_rhs(s, ws);
  if (d1e_rec) W.d1e = d1e_rec;  // q1 derivatives of e - e_ref kept for the reverse mode
  PassArgs a = base_args(s, 1);
  set_ref(a, ref, gamma);
  a.u = u;
  a.metric = metric;
  a.mu = mu;
  a.d1e = W.d1e;
  a.H = W.H;
  a.r2 = W.r2;
  fcsd_status st;
  // patches with a wall side: the energy's derivatives by the product rule
  // from those of rho, m and theta (after pass A for q1, inside B1 for q2)
  const bool walls = flux != FLUX_INVISCID && s->nwchunks > 0 && (patch < 0 || s->wall_patch[patch]);
  // passes B1 and B2 in one launch (a whole-set call of the fused or
  // persistent schedule)
  // (bit 4 of passes asks for it whatever the schedule)
  const bool fuse = patch < 0 && (s->schedule != FCSD_SCHED_SPLIT || (passes & 48u)) && (passes & 6u) == 6u;
  // the fused pass with all eight H fields in LDS (bit 5 of passes asks for it)
  const bool wide = fuse && !(passes & 16u) && s->wide_ok &&
                    (s->schedule == FCSD_SCHED_FUSED_WIDE || (passes & 32u));
  const bool persistent = fuse && passes == 15u && !walls && s->schedule == FCSD_SCHED_PERSISTENT;
  a.out = W.d1e;
  PassArgs b = a;
  b.plans = s->dir[1].d_plans;
  b.mode = flux;
  b.d2out = d2e_rec;
  b.d2th = walls ? s->d_wplanes + 2 * s->plane : nullptr;
  PassArgs e = a;
  e.plans = s->dir[0].d_plans;
  e.mode = outmode;
  e.rhs = rhs;
  e.stage = stage;
  e.u0 = u0;
  e.ui = u;
  e.acc = acc;
  e.uout = uout;
  e.dt = dtp;
  if (persistent) {
    const int np = s->npatch;
    StageArgs g;
    g.A = a;
    g.A.tiles = s->dir[0].ts[0].d_tiles;
    g.B = b;
    g.B.tiles = s->dir[1].ts[1].d_tiles;
    g.C = e;
    g.C.tiles = s->dir[0].ts[0].d_tiles;
    g.tasks = s->d_tasks;
    g.ntasks = s->ntasks;
    g.npatch = np;
    g.skipA = flux == FLUX_INVISCID;
    g.ctr = s->d_ctr;
    g.need = s->d_need;
    g.err = set_error_word(s);
    // counters to zero with a fill kernel (no memset node in a captured step)
    const long long nw = 1 + 2 * (long long)np;
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(nw)), dim3(kBlock), 0, ctx->stream, (float*)s->d_ctr, 0.0f, nw);
    if ((st = launch_check(ctx, "stage counters"))) return st;
    hipLaunchKernelGGL(k_stage, dim3(s->stage_grid), dim3(s->stage_threads), s->stage_lds, ctx->stream, g);
    return launch_check(ctx, "persistent stage");
  }
  if (flux == FLUX_INVISCID) {
    if (!fuse && (passes & 3u)) {
      if (patch < 0) {
        hipLaunchKernelGGL(k_passH, dim3(blocks_for(s->plane)), dim3(kBlock), 0, ctx->stream, a,
                           (long long)s->plane);
      } else {
        const fcsd_patch_desc& q = s->desc[patch];
        PassArgs h = a;
        h.u = u + q.off;
        h.H = W.H + q.off;
        const long long n = (long long)q.n1 * q.n2;
        hipLaunchKernelGGL(k_passH, dim3(blocks_for(n)), dim3(kBlock), 0, ctx->stream, h, n);
      }
      if ((st = launch_check(ctx, "pass H"))) return st;
    }
  } else {
    if (walls && (passes & 3u))
      if ((st = wall_theta_derivs(ctx, s, u, ref, gamma, patch))) return st;
    if (passes & 1u) {
      st = s->a_wide ? launch_lines(s, 1, k_dev_diff2<1>, a, patch, 2) : launch_lines(s, 1, k_dev_diff<1>, a, patch);
      if (st) return st;
      if (walls) {
        const ChunkDev* ch;
        int n;
        wall_chunks(s, patch, &ch, &n);
        hipLaunchKernelGGL(k_energy_rule, dim3(chunk_grid(n)), dim3(kBlock), 0, ctx->stream, ch, n, s->d_patches, u,
                           (long long)s->plane, gamma - 1.0f, (const float*)(s->d_wplanes + s->plane), W.d1e);
        if ((st = launch_check(ctx, "energy rule q1"))) return st;
      }
    }
    if ((passes & 2u) && !fuse)
      if ((st = launch_lines(s, 2, k_passB1, b, patch, 2))) return st;
  }
  if (fuse) {
    if ((st = wide ? launch_lines(s, 2, k_passB4, b, patch, 4) : launch_lines(s, 2, k_passB, b, patch, 2)))
      return st;
  } else if (passes & 4u) {
    PassArgs c = a;
    c.plans = s->dir[1].d_plans;
    if ((st = launch_lines(s, 2, k_passB2, c, patch))) return st;
  }
  if (!(passes & 8u)) return FCSD_OK;
  return launch_lines(s, 1, k_passC, e, patch);
}

}  // namespace

extern "C" fcsd_status fcsd_rhs(fcsd_ctx* ctx, const fcsd_set* s, const float* u, const float* metric,
                                const float* mu, const float ref[4], float gamma, float* rhs, int64_t plane,
                                void* ws, size_t ws_bytes) {
  fcsd_status st = check_set(ctx, s, plane);
  if (st) return st;
  if (!u || !metric || !ref || !rhs || !ws) return fail(ctx, FCSD_EINVAL, "fcsd_rhs: null argument");
  if (ws_bytes < ws_bytes_of(s, FCSD_WS_RHS)) return fail(ctx, FCSD_EINVAL, "fcsd_rhs: workspace too small");
  return rhs_passes(ctx, s, u, metric, mu, ref, gamma, mu ? FLUX_FULL : FLUX_INVISCID, MODE_SET, rhs, 0, nullptr,
                    nullptr, nullptr, nullptr, ws, -1);
}

extern "C" fcsd_status euler_rhs(fcsd_ctx* ctx, const fcsd_set* s, const float* u, const float* metric,
                                 const float ref[4], float gamma, float* rhs, int64_t plane, void* ws,
                                 size_t ws_bytes) {
  return fcsd_rhs(ctx, s, u, metric, nullptr, ref, gamma, rhs, plane, ws, ws_bytes);
}

extern "C" fcsd_status av_apply(fcsd_ctx* ctx, const fcsd_set* s, const float* u, const float* metric,
                                const float* mu, const float ref[4], float* rhs, int64_t plane, void* ws,
                                size_t ws_bytes) {
  fcsd_status st = check_set(ctx, s, plane);
  if (st) return st;
  if (!u || !metric || !mu || !ref || !rhs || !ws) return fail(ctx, FCSD_EINVAL, "av_apply: null argument");
  if (ws_bytes < ws_bytes_of(s, FCSD_WS_RHS)) return fail(ctx, FCSD_EINVAL, "av_apply: workspace too small");
  return rhs_passes(ctx, s, u, metric, mu, ref, 1.4f, FLUX_VISC, MODE_ADD, rhs, 0, nullptr, nullptr, nullptr,
                    nullptr, ws, -1);
}

// ======================================================================== stepping

extern "C" fcsd_status rk_stage(fcsd_ctx* ctx, const fcsd_set* s, int stage, const float* dt_dev, const float* rhs,
                                const float* u0, const float* ui, float* acc, float* uout, int64_t plane) {
  fcsd_status st = check_set(ctx, s, plane);
  if (st) return st;
  if (stage < 0 || stage > 4 || !dt_dev || !rhs || !u0 || !ui || !uout || (stage >= 2 && !acc))
    return fail(ctx, FCSD_EINVAL, "rk_stage: bad arguments");
  if (uout == u0 && stage != 4) return fail(ctx, FCSD_EINVAL, "rk_stage: uout may alias u0 only at stage 4");
  const long long n4 = 4 * (long long)s->plane;
  hipLaunchKernelGGL(k_rk, dim3(blocks_for(n4)), dim3(kBlock), 0, ctx->stream, stage, dt_dev, rhs, u0, ui, acc,
                     uout, n4);
  return launch_check(ctx, "rk_stage");
}

extern "C" fcsd_status rk_stage_adj(fcsd_ctx* ctx, const fcsd_set* s, int stage, const float* dt_dev,
                                    const float* uout_bar, float* u0_bar, float* ui_bar, float* acc_bar,
                                    float* rhs_bar, int64_t plane) {
  fcsd_status st = check_set(ctx, s, plane);
  if (st) return st;
  if (stage < 0 || stage > 4 || !dt_dev || !uout_bar || !u0_bar || !rhs_bar || (stage > 0 && !ui_bar) ||
      (stage >= 2 && !acc_bar))
    return fail(ctx, FCSD_EINVAL, "rk_stage_adj: bad arguments");
  const long long n4 = 4 * (long long)s->plane;
  hipLaunchKernelGGL(k_rk_adj, dim3(blocks_for(n4)), dim3(kBlock), 0, ctx->stream, stage, dt_dev, uout_bar, u0_bar,
                     ui_bar, acc_bar, rhs_bar, n4);
  return launch_check(ctx, "rk_stage_adj");
}

namespace {

fcsd_status cfl_dt_impl(fcsd_ctx* ctx, const fcsd_set* s, const float* u, const float* mu, float cfl, float gamma,
                        float* dt_dev, unsigned* red) {
  const int np = s->npatch;
  unsigned* smax = red;
  unsigned* mmax = red + np;
  hipLaunchKernelGGL(k_fill, dim3(blocks_for(2 * np)), dim3(kBlock), 0, ctx->stream, (float*)red, 0.f,
                     (long long)(2 * np));
  hipLaunchKernelGGL(k_dt_reduce, dim3(chunk_grid(s->nchunks)), dim3(kBlock), 0, ctx->stream, s->d_chunks, s->nchunks, s->d_patches, u, mu,
                     (long long)s->plane, gamma, smax, mmax);
  hipLaunchKernelGGL(k_dt_final, dim3(1), dim3(kBlock), 0, ctx->stream, s->d_patches, np, smax, mmax, cfl, dt_dev);
  return launch_check(ctx, "cfl_dt");
}

}  // namespace

extern "C" fcsd_status fcsd_cfl_dt(fcsd_ctx* ctx, const fcsd_set* s, const float* u, const float* mu, float cfl,
                                   float gamma, float* dt_dev, int64_t plane, void* ws, size_t ws_bytes) {
  fcsd_status st = check_set(ctx, s, plane);
  if (st) return st;
  if (!u || !dt_dev || !ws || !(cfl > 0)) return fail(ctx, FCSD_EINVAL, "fcsd_cfl_dt: bad arguments");
  if (ws_bytes < 2 * sizeof(unsigned) * (size_t)s->npatch)
    return fail(ctx, FCSD_EINVAL, "fcsd_cfl_dt: workspace too small");
  return cfl_dt_impl(ctx, s, u, mu, cfl, gamma, dt_dev, (unsigned*)ws);
}

extern "C" fcsd_status fcsd_cfl_dt_noalloc(fcsd_ctx* ctx, const fcsd_set* s, const float* u, const float* mu,
                                           float cfl, float gamma, float* dt_dev, int64_t plane) {
  fcsd_status st = check_set(ctx, s, plane);
  if (st) return st;
  if (!u || !dt_dev || !(cfl > 0)) return fail(ctx, FCSD_EINVAL, "fcsd_cfl_dt_noalloc: bad arguments");
  if (s->npatch > kNoAllocPatches)
    return fail(ctx, FCSD_EINVAL, "fcsd_cfl_dt_noalloc: more than " + std::to_string(kNoAllocPatches) +
                                      " patches (the static scratch holds two words per patch)");
  if (!ctx->scratch) return fail(ctx, FCSD_EHIP, "fcsd_cfl_dt_noalloc: no scratch address for this device");
  return cfl_dt_impl(ctx, s, u, mu, cfl, gamma, dt_dev, ctx->scratch);
}

extern "C" fcsd_status fcsd_check(fcsd_ctx* ctx, const fcsd_set* s, const float* u, float gamma, int32_t* flags_dev,
                                  int64_t plane) {
  fcsd_status st = check_set(ctx, s, plane);
  if (st) return st;
  if (!u || !flags_dev || !(gamma > 1.0f)) return fail(ctx, FCSD_EINVAL, "fcsd_check: bad arguments");
  hipLaunchKernelGGL(k_fill, dim3(1), dim3(kBlock), 0, ctx->stream, (float*)flags_dev, 0.f, 1LL);
  hipLaunchKernelGGL(k_check, dim3(chunk_grid(s->nchunks)), dim3(kBlock), 0, ctx->stream, s->d_chunks, s->nchunks,
                     s->d_patches, u, (long long)s->plane, gamma, (int*)flags_dev);
  return launch_check(ctx, "fcsd_check");
}

// ======================================================================== viscosity

namespace {

struct AvWs {
  float *phi, *S, *rmax, *muh, *num, *den, *t0, *t1, *tp;
  int* rarg;
  unsigned* red;
};

AvWs carve_av(const fcsd_set* s, void* ws) {
  float* w = (float*)ws;
  const long long pl = s->plane;
  AvWs A;
  A.phi = w;
  A.S = w + pl;
  A.rmax = w + 2 * pl;
  A.rarg = (int*)(w + 3 * pl);
  A.muh = w + 4 * pl;
  A.num = w + 5 * pl;
  A.den = w + 6 * pl;
  A.t0 = w + 7 * pl;
  A.t1 = w + 8 * pl;
  A.tp = w + 9 * pl;
  A.red = (unsigned*)(w + 11 * pl);
  return A;
}

fcsd_status sdnn_impl(fcsd_ctx* ctx, const fcsd_set* s, const float* u, float gamma, const fcsd_mlp* w,
                      int8_t* tau, float* logits, float* phi) {
  hipLaunchKernelGGL(k_proxy, dim3(chunk_grid(s->nchunks)), dim3(kBlock), 0, ctx->stream, s->d_chunks, s->nchunks, s->d_patches, u,
                     (long long)s->plane, gamma, phi, (float*)nullptr);
  MlpPtr m{w->W1, w->b1, w->W2, w->b2, w->W3, w->b3};
  // blocks stride over the chunks so each loads the weights into LDS once
  const int grid = std::min(s->nchunks, 2048);
  hipLaunchKernelGGL(k_sdnn, dim3(grid), dim3(kBlock), 0, ctx->stream, s->d_chunks, s->nchunks, s->d_patches,
                     (const float*)phi, m, (signed char*)tau, logits, (long long)s->plane, set_error_word(s));
  return launch_check(ctx, "sdnn_infer");
}

// forward Lambda denominators (den = conv of the D~ indicator) into A.t1
fcsd_status lambda_forward(fcsd_ctx* ctx, const fcsd_set* s, const AvWs& A, const float* muh, float* mu) {
  hipStream_t st = ctx->stream;
  hipLaunchKernelGGL(k_lat_gather, dim3(chunk_grid(s->nlchunks)), dim3(kBlock), 0, st, s->d_lchunks, s->nlchunks, s->d_lats, s->d_patches,
                     s->an, muh, A.num, A.den, s->annulus, 0);
  hipLaunchKernelGGL(k_lat_conv_g, dim3(chunk_grid(s->nltiles)), dim3(kBlock), 0, st, s->d_ltiles, s->nltiles, s->d_lats,
                     (const float*)A.num, (const float*)A.den, A.t0, A.t1);
  hipLaunchKernelGGL(k_lat_conv_j, dim3(chunk_grid(s->nltiles)), dim3(kBlock), 0, st, s->d_ltiles, s->nltiles, s->d_lats,
                     (const float*)A.t0, (const float*)A.t1, A.num, A.den);
  if (mu) {
    hipLaunchKernelGGL(k_lat_scatter, dim3(chunk_grid(s->nchunks)), dim3(kBlock), 0, st, s->d_chunks, s->nchunks, s->d_patches, s->an,
                       s->annulus, (const float*)A.num, (const float*)A.den, mu);
    if (s->novl > 0)
      hipLaunchKernelGGL(k_lat_overlap, dim3(blocks_for(s->novl)), dim3(kBlock), 0, st, s->d_ovl, s->novl,
                         s->d_ovl_src, (const float*)A.num, (const float*)A.den, mu);
  }
  return launch_check(ctx, "lambda");
}

fcsd_status viscosity_impl(fcsd_ctx* ctx, const fcsd_set* s, const float* u, const int8_t* tau, float gamma,
                           float* mu, int32_t* argmax, const AvWs& A) {
  hipStream_t st = ctx->stream;
  hipLaunchKernelGGL(k_proxy, dim3(chunk_grid(s->nchunks)), dim3(kBlock), 0, st, s->d_chunks, s->nchunks, s->d_patches, u,
                     (long long)s->plane, gamma, (float*)nullptr, A.S);
  hipLaunchKernelGGL(k_rowmax, dim3(chunk_grid(s->nchunks)), dim3(kBlock), 0, st, s->d_chunks, s->nchunks, s->d_patches, (const float*)A.S,
                     A.rmax, A.rarg);
  hipLaunchKernelGGL(k_muhat, dim3(chunk_grid(s->nchunks)), dim3(kBlock), 0, st, s->d_chunks, s->nchunks, s->d_patches,
                     (const float*)A.rmax, (const int*)A.rarg, (const signed char*)tau, A.muh, (int*)argmax);
  fcsd_status r = launch_check(ctx, "mu hat");
  if (r) return r;
  return lambda_forward(ctx, s, A, A.muh, mu);
}

}  // namespace

extern "C" fcsd_status sdnn_infer(fcsd_ctx* ctx, const fcsd_set* s, const float* u, float gamma, const fcsd_mlp* w,
                                  int8_t* tau, float* logits, int64_t plane, void* ws, size_t ws_bytes) {
  fcsd_status st = check_set(ctx, s, plane);
  if (st) return st;
  if (!u || !w || !tau || !ws || !w->W1 || !w->b1 || !w->W2 || !w->b2 || !w->W3 || !w->b3)
    return fail(ctx, FCSD_EINVAL, "sdnn_infer: null argument");
  if (ws_bytes < ws_bytes_of(s, FCSD_WS_AV)) return fail(ctx, FCSD_EINVAL, "sdnn_infer: workspace too small");
  return sdnn_impl(ctx, s, u, gamma, w, tau, logits, carve_av(s, ws).phi);
}

extern "C" fcsd_status av_viscosity(fcsd_ctx* ctx, const fcsd_set* s, const float* u, const int8_t* tau, float gamma,
                                    float* mu, int32_t* argmax, int64_t plane, void* ws, size_t ws_bytes) {
  fcsd_status st = check_set(ctx, s, plane);
  if (st) return st;
  if (!u || !tau || !mu || !ws) return fail(ctx, FCSD_EINVAL, "av_viscosity: null argument");
  if (ws_bytes < ws_bytes_of(s, FCSD_WS_AV)) return fail(ctx, FCSD_EINVAL, "av_viscosity: workspace too small");
  return viscosity_impl(ctx, s, u, tau, gamma, mu, argmax, carve_av(s, ws));
}

extern "C" fcsd_status av_viscosity_adj(fcsd_ctx* ctx, const fcsd_set* s, const float* u, const int8_t* tau,
                                        const int32_t* argmax, float gamma, const float* mu_bar, float* u_bar,
                                        int64_t plane, void* ws, size_t ws_bytes) {
  fcsd_status st = check_set(ctx, s, plane);
  if (st) return st;
  if (!u || !tau || !argmax || !mu_bar || !u_bar || !ws) return fail(ctx, FCSD_EINVAL, "av_viscosity_adj: null argument");
  if (ws_bytes < ws_bytes_of(s, FCSD_WS_AV)) return fail(ctx, FCSD_EINVAL, "av_viscosity_adj: workspace too small");
  AvWs A = carve_av(s, ws);
  hipStream_t sm = ctx->stream;
  // denominators of the forward operator (indicator only; num unused)
  hipLaunchKernelGGL(k_fill, dim3(blocks_for(s->plane)), dim3(kBlock), 0, sm, A.muh, 0.f, (long long)s->plane);
  if ((st = lambda_forward(ctx, s, A, A.muh, nullptr))) return st;
  // t = mu_bar / den at every point, gathered into the lattice, window sum
  hipLaunchKernelGGL(k_lat_divide_pts, dim3(chunk_grid(s->nchunks)), dim3(kBlock), 0, sm, s->d_chunks, s->nchunks, s->d_patches, s->an,
                     s->annulus, mu_bar, (const float*)A.den, A.tp);
  if (s->novl > 0)
    hipLaunchKernelGGL(k_lat_overlap_div, dim3(blocks_for(s->novl)), dim3(kBlock), 0, sm, s->d_ovl, s->novl,
                       s->d_ovl_src, mu_bar, (const float*)A.den, A.tp);
  hipLaunchKernelGGL(k_lat_gather, dim3(chunk_grid(s->nlchunks)), dim3(kBlock), 0, sm, s->d_lchunks, s->nlchunks, s->d_lats, s->d_patches,
                     s->an, (const float*)A.tp, A.t0, (float*)nullptr, s->annulus, 1);
  if (s->novl > 0)
    hipLaunchKernelGGL(k_lat_overlap_scatter, dim3(blocks_for(s->novl)), dim3(kBlock), 0, sm, s->d_ovl, s->novl,
                       s->d_ovl_src, (const float*)A.tp, A.t0);
  hipLaunchKernelGGL(k_lat_conv_g, dim3(chunk_grid(s->nltiles)), dim3(kBlock), 0, sm, s->d_ltiles, s->nltiles, s->d_lats,
                     (const float*)A.t0, (const float*)nullptr, A.t1, (float*)nullptr);
  hipLaunchKernelGGL(k_lat_conv_j, dim3(chunk_grid(s->nltiles)), dim3(kBlock), 0, sm, s->d_ltiles, s->nltiles, s->d_lats,
                     (const float*)A.t1, (const float*)nullptr, A.t0, (float*)nullptr);
  hipLaunchKernelGGL(k_route_S, dim3(chunk_grid(s->nchunks)), dim3(kBlock), 0, sm, s->d_chunks, s->nchunks, s->d_patches, s->an, s->annulus,
                     (const float*)A.t0, (const signed char*)tau, argmax, A.S);
  hipLaunchKernelGGL(k_speed_vjp, dim3(chunk_grid(s->nchunks)), dim3(kBlock), 0, sm, s->d_chunks, s->nchunks, s->d_patches, u,
                     (long long)s->plane, gamma, (const float*)A.S, u_bar);
  return launch_check(ctx, "av_viscosity_adj");
}

// ======================================================================== glue

namespace {

fcsd_status glue_impl(fcsd_ctx* ctx, const fcsd_set* s, float* u, const uint8_t* mask, const float* st4) {
  if (s->annulus) {
    const AnnulusDev& A = s->an;
    if (A.nsec > 1) {
      const long long n = (long long)A.n2 * 2 * kNf * A.nsec * A.nshell;
      hipLaunchKernelGGL(k_glue_sectors, dim3(blocks_for(n)), dim3(kBlock), 0, ctx->stream, s->d_patches, A, u,
                         (long long)s->plane);
    }
    if (A.nshell > 1) {
      const long long n = (long long)A.n1 * 2 * kNf * A.nsec * A.nshell;
      hipLaunchKernelGGL(k_glue_shells, dim3(blocks_for(n)), dim3(kBlock), 0, ctx->stream, s->d_patches, A, u,
                         (long long)s->plane);
    }
  }
  if (s->ninterp > 0)
    hipLaunchKernelGGL(k_interp, dim3(blocks_for(4LL * s->ninterp)), dim3(kBlock), 0, ctx->stream, s->d_interp,
                       s->ninterp, s->d_patches, u, (long long)s->plane);
  if (mask)
    hipLaunchKernelGGL(k_dirichlet, dim3(blocks_for(s->plane)), dim3(kBlock), 0, ctx->stream, mask, u,
                       (long long)s->plane, st4[0], st4[1], st4[2], st4[3]);
  if (s->nwalls > 0)
    hipLaunchKernelGGL(k_wall, dim3(blocks_for((long long)s->nwalls * s->wall_len)), dim3(kBlock), 0, ctx->stream,
                       s->d_walls, s->nwalls, s->wall_len, s->d_patches, u, (long long)s->plane, s->wall_g1, s->d,
                       (const float*)s->d_wall_c);
  return launch_check(ctx, "glue");
}

// transpose of glue_impl: Dirichlet, shells, sectors
fcsd_status glue_adj_impl(fcsd_ctx* ctx, const fcsd_set* s, float* ub, const uint8_t* mask, const float* ds4,
                          double* dparam, const float* glued = nullptr) {
  if (s->nwalls > 0) {
    if (!glued) return fail(ctx, FCSD_EINVAL, "glue reverse mode: the wall condition needs the glued state");
    // one launch per side, then the corners: entries in one launch never
    // share a source point
    for (int only = 0; only < 5; ++only)
      hipLaunchKernelGGL(k_wall_adj, dim3(blocks_for((long long)s->nwalls * s->wall_len)), dim3(kBlock), 0,
                         ctx->stream, s->d_walls, s->nwalls, s->wall_len, s->d_patches, glued, ub,
                         (long long)s->plane, s->wall_g1, s->d, (const float*)s->d_wall_c, only);
  }
  if (mask)
    hipLaunchKernelGGL(k_dirichlet_adj, dim3(blocks_for(s->plane)), dim3(kBlock), 0, ctx->stream, mask, ub,
                       (long long)s->plane, ds4[0], ds4[1], ds4[2], ds4[3], dparam);
  if (s->ninterp > 0)
    hipLaunchKernelGGL(k_interp_adj, dim3(blocks_for(4LL * s->ninterp)), dim3(kBlock), 0, ctx->stream, s->d_interp,
                       s->ninterp, s->d_patches, ub, (long long)s->plane);
  if (s->annulus) {
    const AnnulusDev& A = s->an;
    if (A.nshell > 1) {
      const long long n = (long long)A.n1 * 2 * kNf * A.nsec * A.nshell;
      hipLaunchKernelGGL(k_glue_shells_adj, dim3(blocks_for(n)), dim3(kBlock), 0, ctx->stream, s->d_patches, A, ub,
                         (long long)s->plane);
    }
    if (A.nsec > 1) {
      const long long n = (long long)A.n2 * 2 * kNf * A.nsec * A.nshell;
      hipLaunchKernelGGL(k_glue_sectors_adj, dim3(blocks_for(n)), dim3(kBlock), 0, ctx->stream, s->d_patches, A, ub,
                         (long long)s->plane);
    }
  }
  return launch_check(ctx, "glue_adj");
}

}  // namespace

extern "C" fcsd_status fcsd_glue_adj(fcsd_ctx* ctx, const fcsd_set* s, float* u_bar, int64_t plane,
                                     const uint8_t* dirichlet_mask, const float dstate_dparam[4],
                                     double* dparam_dev, const float* glued) {
  fcsd_status st = check_set(ctx, s, plane);
  if (st) return st;
  if (!u_bar || (dirichlet_mask && (!dstate_dparam || !dparam_dev)))
    return fail(ctx, FCSD_EINVAL, "fcsd_glue_adj: null argument");
  if (s->nwalls > 0 && !glued)
    return fail(ctx, FCSD_EINVAL, "fcsd_glue_adj: the wall condition's reverse mode needs the glued state");
  return glue_adj_impl(ctx, s, u_bar, dirichlet_mask, dstate_dparam, dparam_dev, glued);
}

extern "C" fcsd_status fcsd_glue(fcsd_ctx* ctx, const fcsd_set* s, float* u, int64_t plane,
                                 const uint8_t* dirichlet_mask, const float dirichlet_state[4]) {
  fcsd_status st = check_set(ctx, s, plane);
  if (st) return st;
  if (!u || (dirichlet_mask && !dirichlet_state)) return fail(ctx, FCSD_EINVAL, "fcsd_glue: null argument");
  return glue_impl(ctx, s, u, dirichlet_mask, dirichlet_state);
}

// ======================================================================== fused stage / step

extern "C" fcsd_status fcsd_stage(fcsd_ctx* ctx, const fcsd_set* s, int stage, const float* u0, const float* ui,
                                  float* acc, float* uout, const float* metric, const float* mu, const float ref[4],
                                  float gamma, const float* dt_dev, int64_t plane, void* ws, size_t ws_bytes) {
  fcsd_status st = check_set(ctx, s, plane);
  if (st) return st;
  if (stage < 0 || stage > 4 || !u0 || !ui || !uout || !metric || !ref || !dt_dev || !ws || (stage >= 2 && !acc))
    return fail(ctx, FCSD_EINVAL, "fcsd_stage: bad arguments");
  if (uout == ui || (uout == u0 && stage != 4)) return fail(ctx, FCSD_EINVAL, "fcsd_stage: output aliases an input");
  if (ws_bytes < ws_bytes_of(s, FCSD_WS_RHS)) return fail(ctx, FCSD_EINVAL, "fcsd_stage: workspace too small");
  return rhs_passes(ctx, s, ui, metric, mu, ref, gamma, mu ? FLUX_FULL : FLUX_INVISCID, MODE_RK, nullptr, stage, u0,
                    acc, uout, dt_dev, ws, -1);
}

extern "C" fcsd_status fcsd_stage_per_patch(fcsd_ctx* ctx, const fcsd_set* s, int stage, const float* u0,
                                            const float* ui, float* acc, float* uout, const float* metric,
                                            const float* mu, const float ref[4], float gamma, const float* dt_dev,
                                            int64_t plane, void* ws, size_t ws_bytes) {
  fcsd_status st = check_set(ctx, s, plane);
  if (st) return st;
  if (stage < 0 || stage > 4 || !u0 || !ui || !uout || !metric || !ref || !dt_dev || !ws || (stage >= 2 && !acc))
    return fail(ctx, FCSD_EINVAL, "fcsd_stage_per_patch: bad arguments");
  if (uout == ui || (uout == u0 && stage != 4))
    return fail(ctx, FCSD_EINVAL, "fcsd_stage_per_patch: output aliases an input");
  if (ws_bytes < ws_bytes_of(s, FCSD_WS_RHS)) return fail(ctx, FCSD_EINVAL, "fcsd_stage_per_patch: workspace too small");
  for (int p = 0; p < s->npatch; ++p) {
    st = rhs_passes(ctx, s, ui, metric, mu, ref, gamma, mu ? FLUX_FULL : FLUX_INVISCID, MODE_RK, nullptr, stage, u0,
                    acc, uout, dt_dev, ws, p);
    if (st) return st;
  }
  return FCSD_OK;
}

extern "C" fcsd_status fcsd_stage_pass(fcsd_ctx* ctx, const fcsd_set* s, int pass, int stage, const float* u0,
                                       const float* ui, float* acc, float* uout, const float* metric, const float* mu,
                                       const float ref[4], float gamma, const float* dt_dev, int64_t plane, void* ws,
                                       size_t ws_bytes) {
  fcsd_status st = check_set(ctx, s, plane);
  if (st) return st;
  if (pass < 0 || pass > 5 || stage < 0 || stage > 4 || !u0 || !ui || !uout || !metric || !ref || !dt_dev || !ws ||
      (stage >= 2 && !acc))
    return fail(ctx, FCSD_EINVAL, "fcsd_stage_pass: bad arguments");
  if (uout == ui || (uout == u0 && stage != 4)) return fail(ctx, FCSD_EINVAL, "fcsd_stage_pass: output aliases an input");
  if (pass == 5 && !s->wide_ok)
    return fail(ctx, FCSD_EINVAL, "fcsd_stage_pass: q2 tiles of four complex lines per grid line do not fit the LDS");
  if (ws_bytes < ws_bytes_of(s, FCSD_WS_RHS)) return fail(ctx, FCSD_EINVAL, "fcsd_stage_pass: workspace too small");
  return rhs_passes(ctx, s, ui, metric, mu, ref, gamma, mu ? FLUX_FULL : FLUX_INVISCID, MODE_RK, nullptr, stage, u0,
                    acc, uout, dt_dev, ws, -1, pass == 4 ? 6u | 16u : (pass == 5 ? 6u | 32u : 1u << pass));
}

namespace {

// Spectral filter of the state, q1 lines then q2 lines (in may equal out).
fcsd_status filter_impl(fcsd_ctx* ctx, const fcsd_set* s, const float* in, float* out, float gamma) {
  PassArgs a = base_args(s, 1);
  a.gamma = gamma;
  a.in = in;
  a.out = out;
  fcsd_status st = launch_lines(s, 1, k_filter<1>, a, -1, 2);
  if (st) return st;
  PassArgs b = a;
  b.plans = s->dir[1].d_plans;
  b.in = out;
  return launch_lines(s, 2, k_filter<2>, b, -1, 2);
}

// Reverse mode of filter_impl at state e: out_bar (cotangent of the
// filtered state) -> u_bar (of e; may alias out_bar).  w: 8 planes (the
// filtered state, recomputed, and the cotangent between the two passes).
fcsd_status filter_adj_impl(fcsd_ctx* ctx, const fcsd_set* s, const float* e, const float* out_bar, float* u_bar,
                            float gamma, float* w) {
  const long long pl = s->plane;
  fcsd_status st = filter_impl(ctx, s, e, w, gamma);
  if (st) return st;
  PassArgs a = base_args(s, 2);
  a.gamma = gamma;
  a.in = out_bar;
  a.u = w;
  a.out = w + 4 * pl;
  if ((st = launch_lines(s, 2, k_filter_adj<2>, a, -1, 2))) return st;
  PassArgs b = base_args(s, 1);
  b.gamma = gamma;
  b.in = w + 4 * pl;
  b.u = e;
  b.out = u_bar;
  return launch_lines(s, 1, k_filter_adj<1>, b, -1, 2);
}

// planes of a step record after the stage inputs, mu, the maximisers and the
// pre-filter state: the q1 and q2 derivatives of e - e_ref of each stage input
constexpr long long kRecD1 = 26, kRecD2 = 46;
static_assert(kRecD2 + 20 == FCSD_RECORD_PLANES, "record layout");

fcsd_status step_body(fcsd_ctx* ctx, const fcsd_set* s, const fcsd_step_args* a, void* ws) {
  const long long pl = s->plane;
  float* w = (float*)ws;
  void* rhs_ws = w;
  float* Ua = w + 16 * pl;
  float* Ub = w + 20 * pl;
  float* ACC = w + 24 * pl;
  void* av_ws = w + 28 * pl;
  AvWs A = carve_av(s, av_ws);
  fcsd_status st;
  if ((st = glue_impl(ctx, s, a->u, a->dirichlet_mask, a->dirichlet_state))) return st;
  if (a->w && !a->fixed_tau)
    if ((st = sdnn_impl(ctx, s, a->u, a->gamma, a->w, a->tau, nullptr, A.phi))) return st;
  if (a->w || a->fixed_tau)
    if ((st = viscosity_impl(ctx, s, a->u, a->tau, a->gamma, a->mu, a->argmax, A))) return st;
  const long long n4 = 4 * pl;
  float* rec = a->record;
  hipStream_t sm = ctx->stream;
  if (rec) {
    if (a->mu) HIPCHK(ctx, hipMemcpyAsync(rec + 5 * n4, a->mu, pl * sizeof(float), hipMemcpyDeviceToDevice, sm));
    if (a->w || a->fixed_tau)
      HIPCHK(ctx, hipMemcpyAsync(rec + 5 * n4 + pl, a->argmax, pl * sizeof(int32_t), hipMemcpyDeviceToDevice, sm));
    if (a->filter)
      HIPCHK(ctx, hipMemcpyAsync(rec + 5 * n4 + 2 * pl, a->u, n4 * sizeof(float), hipMemcpyDeviceToDevice, sm));
  }
  if (a->filter) {
    if ((st = filter_impl(ctx, s, a->u, a->u, a->gamma))) return st;
    if ((st = glue_impl(ctx, s, a->u, a->dirichlet_mask, a->dirichlet_state))) return st;
  }
  if (!a->fixed_dt)
    if ((st = cfl_dt_impl(ctx, s, a->u, a->mu, a->cfl, a->gamma, a->dt_dev, A.red))) return st;
  const float* ins[5] = {a->u, Ua, Ub, Ua, Ub};
  float* outs[5] = {Ua, Ub, Ua, Ub, a->u};
  if (rec) {  // stage inputs 1..4 are computed straight into the record
    HIPCHK(ctx, hipMemcpyAsync(rec, a->u, n4 * sizeof(float), hipMemcpyDeviceToDevice, sm));
    for (int k = 1; k < 5; ++k) {
      ins[k] = rec + k * n4;
      outs[k - 1] = rec + k * n4;
    }
  }
  for (int k = 0; k < 5; ++k) {
    if (k > 0)
      if ((st = glue_impl(ctx, s, const_cast<float*>(ins[k]), a->dirichlet_mask, a->dirichlet_state))) return st;
    float* d1r = rec && a->mu ? rec + kRecD1 * pl + k * n4 : nullptr;
    float* d2r = rec && a->mu ? rec + kRecD2 * pl + k * n4 : nullptr;
    st = rhs_passes(ctx, s, ins[k], a->metric, a->mu, a->ref, a->gamma, a->mu ? FLUX_FULL : FLUX_INVISCID, MODE_RK,
                    nullptr, k, a->u, ACC, outs[k], a->dt_dev, rhs_ws, -1, 15u, d1r, d2r);
    if (st) return st;
  }
  return FCSD_OK;
}

}  // namespace

extern "C" fcsd_status fcsd_step(fcsd_ctx* ctx, const fcsd_set* s, const fcsd_step_args* a, int64_t plane, void* ws,
                                 size_t ws_bytes, int use_graph) {
  fcsd_status st = check_set(ctx, s, plane);
  if (st) return st;
  if (!a || !a->u || !a->metric || !a->dt_dev || !ws) return fail(ctx, FCSD_EINVAL, "fcsd_step: null argument");
  if ((a->w || a->fixed_tau) && (!a->tau || !a->mu))
    return fail(ctx, FCSD_EINVAL, "fcsd_step: network needs tau and mu buffers");
  if (a->filter && !s->filter_on) return fail(ctx, FCSD_EINVAL, "fcsd_step: filter not configured (fcsd_set_filter)");
  if (a->record && (a->w || a->fixed_tau) && !a->argmax)
    return fail(ctx, FCSD_EINVAL, "fcsd_step: a record with classes needs the argmax buffer");
  if (ws_bytes < ws_bytes_of(s, FCSD_WS_STEP)) return fail(ctx, FCSD_EINVAL, "fcsd_step: workspace too small");
  if (!use_graph) return step_body(ctx, s, a, ws);
  if (!ctx->stream) return fail(ctx, FCSD_EINVAL, "fcsd_step: graph capture needs a non-default stream");
  std::vector<unsigned char> key(sizeof(*a) + sizeof(void*) + (a->w ? sizeof(fcsd_mlp) : 0));
  memcpy(key.data(), a, sizeof(*a));
  memcpy(key.data() + sizeof(*a), &ws, sizeof(void*));
  if (a->w) memcpy(key.data() + sizeof(*a) + sizeof(void*), a->w, sizeof(fcsd_mlp));
  fcsd_set* ms = const_cast<fcsd_set*>(s);
  for (auto& g : ms->graphs)
    if (g.key == key) {
      HIPCHK(ctx, hipGraphLaunch(g.exec, ctx->stream));
      return FCSD_OK;
    }
  hipGraph_t graph = nullptr;
  HIPCHK(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
  st = step_body(ctx, s, a, ws);
  hipError_t e = hipStreamEndCapture(ctx->stream, &graph);
  if (st || e != hipSuccess) {
    // a body that failed part-way leaves a partial graph: never kept
    if (graph) (void)hipGraphDestroy(graph);
    if (st) return st;
    return fail(ctx, FCSD_EHIP, std::string("capture: ") + hipGetErrorString(e));
  }
  GraphEntry g;
  g.key = key;
  e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return fail(ctx, FCSD_EHIP, std::string("instantiate: ") + hipGetErrorString(e));
  // bounded cache: the oldest graph goes once kMaxGraphs argument sets are
  // held (after the stream has drained, so it is not running)
  if (ms->graphs.size() >= kMaxGraphs) {
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    (void)hipGraphExecDestroy(ms->graphs.front().exec);
    ms->graphs.erase(ms->graphs.begin());
  }
  ms->graphs.push_back(g);
  HIPCHK(ctx, hipGraphLaunch(g.exec, ctx->stream));
  return FCSD_OK;
}

namespace {

// Line tiles of the wall patches, per direction (from the single-field tile
// sets, in their launch order), for the FC derivatives of theta.
fcsd_status rebuild_wall_tiles(fcsd_set* s) {
  fcsd_ctx* ctx = s->ctx;
  fcsd_status r;
  for (int dir = 0; dir < 2; ++dir) {
    (void)hipFree(s->d_wtiles[dir]);
    s->d_wtiles[dir] = nullptr;
    s->nwtiles[dir] = 0;
    if (s->wall_patch.empty()) continue;
    const DirPlan& D = s->dir[dir];
    std::vector<TileDev> t;
    for (const TileDev& T : D.ts[0].tiles)
      if (T.nl > 0 && s->wall_patch[D.plans[T.plan].patch]) t.push_back(T);
    if ((r = upload(ctx, &s->d_wtiles[dir], t))) return r;
    s->nwtiles[dir] = (int)t.size();
  }
  return FCSD_OK;
}

}  // namespace

extern "C" fcsd_status fcsd_set_walls(fcsd_set* s, const uint8_t* sides, float gamma) {
  if (!s) return FCSD_EINVAL;
  fcsd_ctx* ctx = s->ctx;
  if (!(gamma > 1.0f)) return fail(ctx, FCSD_EINVAL, "fcsd_set_walls: need gamma > 1");
  std::vector<WallDev> walls;
  std::vector<uint8_t> wp(s->npatch, 0);
  int len = 0;
  if (sides)
    for (int p = 0; p < s->npatch; ++p) {
      const uint8_t* f = sides + 4 * p;
      const fcsd_patch_desc& q = s->desc[p];
      for (int side = 0; side < 4; ++side) {
        if (!f[side]) continue;
        if ((side < 2 ? q.n1 : q.n2) < s->d + 1)
          return fail(ctx, FCSD_EINVAL, "fcsd_set_walls: patch too short across its wall");
        if ((side < 2 ? q.n2 : q.n1) < s->d + 1)
          return fail(ctx, FCSD_EINVAL, "fcsd_set_walls: patch too short along its wall");
        const int length = side < 2 ? q.n2 : q.n1;
        // points shared with a perpendicular wall are corners, owned by the q1 side
        const bool lo_c = side < 2 ? f[2] : f[0], hi_c = side < 2 ? f[3] : f[1];
        walls.push_back(WallDev{p, side, lo_c ? 1 : 0, hi_c ? length - 1 : length, -1});
        if (side < 2) {
          if (lo_c) walls.push_back(WallDev{p, side, 0, 1, 0});
          if (hi_c) walls.push_back(WallDev{p, side, 0, 1, 1});
        }
        len = std::max(len, length);
        wp[p] = 1;
      }
    }
  // Neumann boundary value: p(0) = c[0] g + sum_{k=1}^{d-1} c[k] F_k for the
  // polynomial of degree < d with p(k) = F_k and p'(0) = g (grid units);
  // a_0 of the solution of the d x d system, by Gaussian elimination with
  // partial pivoting in long double
  const int d = s->d;
  std::vector<float> c(d, 0.f);
  for (int col = 0; col < d; ++col) {  // c[col]: a_0 for the data unit vector e_col
    long double A[8][9];
    for (int r = 0; r < d; ++r)
      for (int m = 0; m < d; ++m) A[r][m] = r < d - 1 ? std::pow((long double)(r + 1), m) : (m == 1 ? 1.0L : 0.0L);
    for (int r = 0; r < d; ++r)  // right-hand side: rows 0..d-2 the values F_1..F_{d-1}, row d-1 g
      A[r][d] = (col == 0 ? r == d - 1 : r == col - 1) ? 1.0L : 0.0L;
    for (int k = 0; k < d; ++k) {
      int piv = k;
      for (int r = k + 1; r < d; ++r)
        if (std::fabs(A[r][k]) > std::fabs(A[piv][k])) piv = r;
      for (int m = 0; m <= d; ++m) std::swap(A[k][m], A[piv][m]);
      for (int r = 0; r < d; ++r)
        if (r != k) {
          const long double f = A[r][k] / A[k][k];
          for (int m = k; m <= d; ++m) A[r][m] -= f * A[k][m];
        }
    }
    c[col] = (float)(A[0][d] / A[0][0]);
  }
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  for (auto& g : s->graphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  s->graphs.clear();
  (void)hipFree(s->d_walls);
  (void)hipFree(s->d_wall_c);
  (void)hipFree(s->d_wchunks);
  (void)hipFree(s->d_wplanes);
  s->d_walls = nullptr;
  s->d_wall_c = nullptr;
  s->d_wchunks = nullptr;
  s->d_wplanes = nullptr;
  s->nwalls = 0;
  s->nwchunks = 0;
  s->wall_patch.clear();
  fcsd_status r;
  if ((r = upload(ctx, &s->d_walls, walls)) || (r = upload(ctx, &s->d_wall_c, c))) return r;
  // wall patches: their plans' flag, point chunks, line tiles and the set's
  // scratch planes for theta and its derivatives
  const bool any = !walls.empty();
  for (int dir = 0; dir < 2; ++dir) {
    DirPlan& D = s->dir[dir];
    for (PlanDev& P : D.plans) P.wallp = any ? wp[P.patch] : 0;
    (void)hipFree(D.d_plans);
    D.d_plans = nullptr;
    if ((r = upload(ctx, &D.d_plans, D.plans))) return r;
  }
  if (any) {
    s->wall_patch = wp;
    std::vector<ChunkDev> wc;
    for (int p = 0; p < s->npatch; ++p)
      if (wp[p])
        for (long long k = 0; k < patch_storage(s->desc[p].n1, s->desc[p].n2, s->layout); k += kChunk)
          wc.push_back(ChunkDev{p, (int)k});
    if ((r = upload(ctx, &s->d_wchunks, wc))) return r;
    s->nwchunks = (int)wc.size();
    HIPCHK(ctx, hipMalloc((void**)&s->d_wplanes, 6 * (size_t)s->plane * sizeof(float)));
    HIPCHK(ctx, hipMemset(s->d_wplanes, 0, 6 * (size_t)s->plane * sizeof(float)));
  }
  if ((r = rebuild_wall_tiles(s))) return r;
  s->nwalls = (int)walls.size();
  s->wall_len = len;
  s->wall_g1 = gamma - 1.0f;
  return FCSD_OK;
}

namespace {

// Evaluation of a patch map (fcsd_patch_map) and of its inverse.
struct MapEval {
  const fcsd_patch_map& m;
  int n1, n2;

  // the S-type arc l (order 0), l' (1) or l'' (2) at t
  void arc(double t, int order, double& x, double& y) const {
    x = y = 0.0;
    for (int k = 0; k < m.nmodes; ++k) {
      const double c = std::cos(k * t), sn = std::sin(k * t);
      double fc = c, fs = sn;
      if (order == 1) {
        fc = -k * sn;
        fs = k * c;
      } else if (order == 2) {
        fc = -(double)k * k * c;
        fs = -(double)k * k * sn;
      }
      x += m.cx[k] * fc + m.sx[k] * fs;
      y += m.cy[k] * fc + m.sy[k] * fs;
    }
  }
  // unit normal nu(t) = side * (l'_y, -l'_x) / |l'| and its derivative
  void normal(double t, double nu[2], double dnu[2]) const {
    double ax, ay, bx, by;
    arc(t, 1, ax, ay);
    arc(t, 2, bx, by);
    const double n = std::hypot(ax, ay), dot = ax * bx + ay * by, sd = m.side;
    nu[0] = sd * ay / n;
    nu[1] = -sd * ax / n;
    dnu[0] = sd * (by / n - ay * dot / (n * n * n));
    dnu[1] = -sd * (bx / n - ax * dot / (n * n * n));
  }
  void image(double i, double j, double& x, double& y) const {
    switch (m.kind) {
      case FCSD_MAP_CARTESIAN:
        x = m.a0 + i * m.da;
        y = m.b0 + j * m.db;
        return;
      case FCSD_MAP_POLAR: {
        const double th = m.a0 + i * m.da, r = m.b0 + j * m.db;
        x = r * std::cos(th);
        y = r * std::sin(th);
        return;
      }
      case FCSD_MAP_AFFINE:
        x = m.x0 + i * m.ux + j * m.vx;
        y = m.y0 + i * m.uy + j * m.vy;
        return;
      default: {
        const double t = m.a0 + i * m.da, sv = m.b0 + j * m.db;
        double lx, ly, nu[2], dn[2];
        arc(t, 0, lx, ly);
        normal(t, nu, dn);
        x = lx + sv * nu[0];
        y = ly + sv * nu[1];
      }
    }
  }
  // fractional grid indices of (x, y); false where an S-type inverse does
  // not settle
  bool preimage(double x, double y, double& xi, double& eta) const {
    switch (m.kind) {
      case FCSD_MAP_CARTESIAN:
        xi = (x - m.a0) / m.da;
        eta = (y - m.b0) / m.db;
        return true;
      case FCSD_MAP_POLAR:
        xi = (std::atan2(y, x) - m.a0) / m.da;
        eta = (std::hypot(x, y) - m.b0) / m.db;
        return true;
      case FCSD_MAP_AFFINE: {
        const double det = m.ux * m.vy - m.vx * m.uy, dx = x - m.x0, dy = y - m.y0;
        xi = (dx * m.vy - dy * m.vx) / det;
        eta = (m.ux * dy - m.uy * dx) / det;
        return true;
      }
      default:
        break;
    }
    // S-type: start at the foot point on the arc -- of the arc parameters of
    // the grid columns (and one beyond each end), the one where (x, y) - l(t)
    // is most nearly normal to the arc -- then Newton's method on
    // l(t) + s nu(t) = (x, y)
    double t = m.a0, sv = 0.0, best = 1e300;
    for (int i = -1; i <= n1; ++i) {
      const double tc = m.a0 + i * m.da;
      double lx, ly, tx, ty, nu[2], dn[2];
      arc(tc, 0, lx, ly);
      arc(tc, 1, tx, ty);
      normal(tc, nu, dn);
      const double dx = x - lx, dy = y - ly, tn = std::hypot(tx, ty);
      const double along = std::fabs(dx * tx + dy * ty) / tn, across = dx * nu[0] + dy * nu[1];
      const double score = along + 1e-3 * std::fabs(across);
      if (score < best) {
        best = score;
        t = tc;
        sv = across;
      }
    }
    const double scale = 1.0 + std::fabs(x) + std::fabs(y);
    for (int it = 0; it < 60; ++it) {
      double lx, ly, ax, ay, nu[2], dn[2];
      arc(t, 0, lx, ly);
      arc(t, 1, ax, ay);
      normal(t, nu, dn);
      const double fx = lx + sv * nu[0] - x, fy = ly + sv * nu[1] - y;
      const double j11 = ax + sv * dn[0], j21 = ay + sv * dn[1], j12 = nu[0], j22 = nu[1];
      const double det = j11 * j22 - j12 * j21;
      if (!(std::fabs(det) > 0.0)) return false;
      const double dt = (fx * j22 - fy * j12) / det, ds = (j11 * fy - j21 * fx) / det;
      t -= dt;
      sv -= ds;
      if (std::hypot(fx, fy) <= 1e-14 * scale && std::fabs(dt) <= 1e-13 * (1.0 + std::fabs(t))) break;
    }
    double lx, ly, nu[2], dn[2];
    arc(t, 0, lx, ly);
    normal(t, nu, dn);
    if (!(std::hypot(lx + sv * nu[0] - x, ly + sv * nu[1] - y) <= 1e-12 * scale)) return false;
    xi = (t - m.a0) / m.da;
    eta = (sv - m.b0) / m.db;
    return true;
  }
};

bool map_valid(const fcsd_patch_map& m) {
  switch (m.kind) {
    case FCSD_MAP_CARTESIAN:
    case FCSD_MAP_POLAR:
      return m.da > 0 && m.db > 0;
    case FCSD_MAP_AFFINE:
      return std::isfinite(m.ux * m.vy - m.vx * m.uy) && std::fabs(m.ux * m.vy - m.vx * m.uy) > 0;
    case FCSD_MAP_STYPE:
      return m.da > 0 && m.db > 0 && m.nmodes >= 1 && m.nmodes <= 8 && (m.side == 1.0 || m.side == -1.0);
    default:
      return false;
  }
}

}  // namespace

extern "C" fcsd_status fcsd_set_interp(fcsd_set* s, const fcsd_patch_map* maps, int nf, int64_t* nrecv) {
  if (!s) return FCSD_EINVAL;
  fcsd_ctx* ctx = s->ctx;
  if (!maps) return fail(ctx, FCSD_EINVAL, "fcsd_set_interp: null patch maps");
  if (s->annulus) return fail(ctx, FCSD_EUNSUPPORTED, "fcsd_set_interp: index-aligned sets glue by copy");
  const int np = s->npatch;
  for (int p = 0; p < np; ++p)
    if (!map_valid(maps[p]))
      return fail(ctx, FCSD_EINVAL, "fcsd_set_interp: bad patch map " + std::to_string(p) +
                                        " (unknown kind, non-positive steps, singular affine map, or an S-type "
                                        "arc without 1..8 modes or side +-1)");
  int minside = 1 << 30;
  for (const fcsd_patch_desc& q : s->desc) minside = std::min(minside, std::min(q.n1, q.n2));
  if (nf < 1 || 2 * nf + 3 > minside) return fail(ctx, FCSD_EINVAL, "fcsd_set_interp: fringe width out of range");
  std::vector<MapEval> ev;
  for (int p = 0; p < np; ++p) ev.push_back(MapEval{maps[p], s->desc[p].n1, s->desc[p].n2});
  // physical bounding box of every patch (its boundary sampled at the grid
  // points, a polar side's arc also at the axis crossings it spans), to skip
  // the preimage of patches that cannot hold a point
  std::vector<std::array<double, 4>> box(np);
  for (int p = 0; p < np; ++p) {
    const fcsd_patch_desc& q = s->desc[p];
    const fcsd_patch_map& m = maps[p];
    double x0 = 1e300, x1 = -1e300, y0 = 1e300, y1 = -1e300, hmax = 0.0, px = 0.0, py = 0.0;
    bool first = true;
    auto add = [&](double x, double y) {
      x0 = std::min(x0, x);
      x1 = std::max(x1, x);
      y0 = std::min(y0, y);
      y1 = std::max(y1, y);
    };
    // the boundary walked in order (consecutive samples give the largest
    // boundary spacing)
    auto pt = [&](double i, double j) {
      double x, y;
      ev[p].image(i, j, x, y);
      add(x, y);
      if (!first) hmax = std::max(hmax, std::hypot(x - px, y - py));
      first = false;
      px = x;
      py = y;
    };
    for (int i = 0; i < q.n1; ++i) pt(i, 0);
    for (int j = 0; j < q.n2; ++j) pt(q.n1 - 1, j);
    for (int i = q.n1 - 1; i >= 0; --i) pt(i, q.n2 - 1);
    for (int j = q.n2 - 1; j >= 0; --j) pt(0, j);
    if (m.kind == FCSD_MAP_POLAR) {  // axis crossings inside the angular range
      const double t0 = m.a0, t1 = m.a0 + (q.n1 - 1) * m.da, rmax = m.b0 + (q.n2 - 1) * m.db;
      for (int k = -8; k <= 8; ++k) {
        const double a = k * 0.5 * 3.14159265358979323846;
        if (a > t0 && a < t1) add(rmax * std::cos(a), rmax * std::sin(a));
      }
    }
    // generous margin: two of the largest boundary spacings (covers the
    // bulge of a curved side between its samples); the box only spares work
    const double pad = 2.0 * hmax + 1e-9 * (1.0 + std::max(x1 - x0, y1 - y0));
    box[p] = {x0 - pad, x1 + pad, y0 - pad, y1 + pad};
  }
  auto in_box = [&](int d, double x, double y) {
    return x >= box[d][0] && x <= box[d][1] && y >= box[d][2] && y <= box[d][3];
  };
  // fringe points: the nf grid lines nearest to every internal side
  auto recv = [&](int p, int i, int j) {
    const fcsd_patch_desc& q = s->desc[p];
    return (q.internal[0] && i < nf) || (q.internal[1] && i >= q.n1 - nf) || (q.internal[2] && j < nf) ||
           (q.internal[3] && j >= q.n2 - nf);
  };
  std::vector<InterpDev> tab;
  for (int p = 0; p < np; ++p) {
    const fcsd_patch_desc& q = s->desc[p];
    for (int j = 0; j < q.n2; ++j)
      for (int i = 0; i < q.n1; ++i) {
        if (!recv(p, i, j)) continue;
        double x, y;
        ev[p].image(i, j, x, y);
        // donor: the other patch holding a full stencil around the point's
        // preimage in which the point lies farthest from the boundary (the
        // lower index on ties)
        int best = -1;
        double bd = 0.0, bxi = 0.0, beta = 0.0;
        for (int d = 0; d < np; ++d) {
          if (d == p || !in_box(d, x, y)) continue;
          double xi, eta;
          if (!ev[d].preimage(x, y, xi, eta)) continue;
          const fcsd_patch_desc& dq = s->desc[d];
          const double dist = std::min(std::min(xi, dq.n1 - 1 - xi), std::min(eta, dq.n2 - 1 - eta));
          if (dist >= 1.0 && (best < 0 || dist > bd)) {
            best = d;
            bd = dist;
            bxi = xi;
            beta = eta;
          }
        }
        if (best < 0)
          return fail(ctx, FCSD_EINVAL, "fcsd_set_interp: fringe point (" + std::to_string(p) + ", " +
                                            std::to_string(i) + ", " + std::to_string(j) + ") has no donor");
        const fcsd_patch_desc& dq = s->desc[best];
        const int ic = std::min(std::max((int)std::floor(bxi + 0.5), 1), dq.n1 - 2);
        const int jc = std::min(std::max((int)std::floor(beta + 0.5), 1), dq.n2 - 2);
        for (int b = -1; b <= 1; ++b)
          for (int a = -1; a <= 1; ++a)
            if (recv(best, ic + a, jc + b))
              return fail(ctx, FCSD_EINVAL, "fcsd_set_interp: donor stencil of fringe point (" + std::to_string(p) +
                                                ", " + std::to_string(i) + ", " + std::to_string(j) +
                                                ") holds fringe points of patch " + std::to_string(best));
        tab.push_back(InterpDev{p, i, j, best, ic, jc, (float)(bxi - ic), (float)(beta - jc)});
      }
  }
  // smoothing operator: every point of a patch that lies in another patch's
  // closed parameter rectangle also takes that patch's window sums at the
  // grid point nearest to its preimage (rnd(n + 1/2) = n + 1)
  std::vector<OvlTarget> ovl;
  std::vector<long long> osrc;
  for (int p = 0; p < np; ++p) {
    const fcsd_patch_desc& q = s->desc[p];
    PatchDev P{};
    P.n1 = q.n1;
    P.n2 = q.n2;
    P.off = q.off;
    P.nb1 = s->layout == FCSD_LAYOUT_B8X4 ? (q.n1 + 7) >> 3 : 0;
    for (int j = 0; j < q.n2; ++j)
      for (int i = 0; i < q.n1; ++i) {
        double x, y;
        ev[p].image(i, j, x, y);
        const int begin = (int)osrc.size();
        for (int d = 0; d < np; ++d) {
          if (d == p || !in_box(d, x, y)) continue;
          double xi, eta;
          if (!ev[d].preimage(x, y, xi, eta)) continue;
          const fcsd_patch_desc& dq = s->desc[d];
          if (!(xi >= 0.0 && xi <= dq.n1 - 1 && eta >= 0.0 && eta <= dq.n2 - 1)) continue;
          const long long I = (long long)std::floor(xi + 0.5), J = (long long)std::floor(eta + 0.5);
          osrc.push_back(dq.off + J * dq.n1 + I);
        }
        if ((int)osrc.size() > begin)
          ovl.push_back(OvlTarget{pidx(P, i, j), q.off + (long long)j * q.n1 + i, begin, (int)osrc.size()});
      }
  }
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  for (auto& g : s->graphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  s->graphs.clear();
  (void)hipFree(s->d_interp);
  (void)hipFree(s->d_ovl);
  (void)hipFree(s->d_ovl_src);
  s->d_interp = nullptr;
  s->d_ovl = nullptr;
  s->d_ovl_src = nullptr;
  s->ninterp = s->novl = 0;
  fcsd_status r;
  if ((r = upload(ctx, &s->d_interp, tab)) || (r = upload(ctx, &s->d_ovl, ovl)) || (r = upload(ctx, &s->d_ovl_src, osrc)))
    return r;
  s->ninterp = (int)tab.size();
  s->novl = (int)ovl.size();
  if (nrecv) *nrecv = (int64_t)tab.size();
  return FCSD_OK;
}

extern "C" fcsd_status fcsd_smear(fcsd_ctx* ctx, const fcsd_set* s, const float* u, const uint8_t* region,
                                  float* out, int64_t plane, float gamma, double alpha, int p, double c, double r,
                                  void* ws, size_t ws_bytes) {
  fcsd_status st = check_set(ctx, s, plane);
  if (st) return st;
  if (!u || !region || !out || !ws) return fail(ctx, FCSD_EINVAL, "fcsd_smear: null argument");
  if (!(alpha >= 0.0) || !std::isfinite(alpha) || p < 2 || p > 64 || p % 2)
    return fail(ctx, FCSD_EINVAL, "fcsd_smear: need alpha >= 0 finite and an even p in [2, 64]");
  if (!(c >= 0.0) || !(r > 0.0) || !(c / 2 + r <= 1e6))
    return fail(ctx, FCSD_EINVAL, "fcsd_smear: need c >= 0, r > 0 and c/2 + r <= 1e6 grid spacings");
  if (ws_bytes < ws_bytes_of(s, FCSD_WS_SMEAR)) return fail(ctx, FCSD_EINVAL, "fcsd_smear: workspace too small");
  if (s->npatch > 65535) return fail(ctx, FCSD_EUNSUPPORTED, "fcsd_smear: more than 65535 patches");
  fcsd_set* ms = const_cast<fcsd_set*>(s);
  if (!ms->d_ks || ms->ks_alpha != alpha || ms->ks_p != p) {
    // factors of every distinct extended length, offsets per direction and plan
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    std::vector<float2> ks;
    std::map<std::tuple<int, int, int>, int> at_L;
    std::vector<int> off[2];
    for (int dir = 0; dir < 2; ++dir)
      for (const PlanDev& P : s->dir[dir].plans) {
        const auto fkey = filter_key(P);
        if (!at_L.count(fkey)) {
          at_L[fkey] = (int)ks.size();
          std::vector<float> t;
          filter_table(P, alpha, p, t);
          for (int n = 0; n < P.L; ++n) ks.push_back(make_float2(t[2 * n], t[2 * n + 1]));
        }
        off[dir].push_back(at_L[fkey]);
      }
    (void)hipFree(ms->d_ks);
    (void)hipFree(ms->d_ksoff[0]);
    (void)hipFree(ms->d_ksoff[1]);
    ms->d_ks = nullptr;
    ms->d_ksoff[0] = ms->d_ksoff[1] = nullptr;
    ms->ks_alpha = -1.0;
    fcsd_status r2;
    if ((r2 = upload(ctx, &ms->d_ks, ks)) || (r2 = upload(ctx, &ms->d_ksoff[0], off[0])) ||
        (r2 = upload(ctx, &ms->d_ksoff[1], off[1])))
      return r2;
    ms->ks_alpha = alpha;
    ms->ks_p = p;
  }
  int max1 = 0, max2 = 0;
  for (const fcsd_patch_desc& q : s->desc) {
    max1 = std::max(max1, q.n1);
    max2 = std::max(max2, q.n2);
  }
  float* w1 = (float*)ws;
  float* w2 = w1 + s->plane;
  const float c2 = (float)(c / 2), rf = (float)r;
  hipLaunchKernelGGL(k_smear_window<1>, dim3((unsigned)((max2 + kBlock - 1) / kBlock), (unsigned)s->npatch),
                     dim3(kBlock), 0, ctx->stream, s->d_patches, region, w1, c2, rf);
  hipLaunchKernelGGL(k_smear_window<2>, dim3((unsigned)((max1 + kBlock - 1) / kBlock), (unsigned)s->npatch),
                     dim3(kBlock), 0, ctx->stream, s->d_patches, region, w2, c2, rf);
  if ((st = launch_check(ctx, "smear window"))) return st;
  PassArgs a = base_args(s, 1);
  a.gamma = gamma;
  a.in = u;
  a.out = out;
  a.kf = ms->d_ks;
  a.koff = ms->d_ksoff[0];
  a.win = w1;
  if ((st = launch_lines(s, 1, k_smear<1>, a, -1, 2))) return st;
  PassArgs b = a;
  b.plans = s->dir[1].d_plans;
  b.in = out;
  b.koff = ms->d_ksoff[1];
  b.win = w2;
  return launch_lines(s, 2, k_smear<2>, b, -1, 2);
}

extern "C" fcsd_status fcsd_filter(fcsd_ctx* ctx, const fcsd_set* s, const float* u, float* out, int64_t plane,
                                   float gamma) {
  fcsd_status st = check_set(ctx, s, plane);
  if (st) return st;
  if (!u || !out) return fail(ctx, FCSD_EINVAL, "fcsd_filter: null argument");
  if (!s->filter_on) return fail(ctx, FCSD_EINVAL, "fcsd_filter: filter not configured (fcsd_set_filter)");
  return filter_impl(ctx, s, u, out, gamma);
}

extern "C" fcsd_status fcsd_filter_adj(fcsd_ctx* ctx, const fcsd_set* s, const float* u, const float* out_bar,
                                       float* u_bar, int64_t plane, float gamma, void* ws, size_t ws_bytes) {
  fcsd_status st = check_set(ctx, s, plane);
  if (st) return st;
  if (!u || !out_bar || !u_bar || !ws) return fail(ctx, FCSD_EINVAL, "fcsd_filter_adj: null argument");
  if (u_bar == u) return fail(ctx, FCSD_EINVAL, "fcsd_filter_adj: u_bar may not alias u");
  if (!s->filter_on) return fail(ctx, FCSD_EINVAL, "fcsd_filter_adj: filter not configured (fcsd_set_filter)");
  if (ws_bytes < ws_bytes_of(s, FCSD_WS_FILTER_ADJ))
    return fail(ctx, FCSD_EINVAL, "fcsd_filter_adj: workspace too small");
  return filter_adj_impl(ctx, s, u, out_bar, u_bar, gamma, (float*)ws);
}

// ======================================================================== reverse mode of the RHS

namespace {

// Reverse mode of the right-hand side; given1 / given2 (nullable): the q1
// and q2 derivatives of e - e_ref at u, recorded by the forward step, which
// are then not recomputed.
fcsd_status rhs_adj_impl(fcsd_ctx* ctx, const fcsd_set* s, const float* u, const float* metric, const float* mu,
                         const float ref[4], float gamma, const float* rhs_bar, float* u_bar, float* mu_bar,
                         void* ws, const float* given1, const float* given2, int flux = FLUX_FULL) {
  fcsd_status st;
  const long long pl = s->plane;
  float* w = (float*)ws;
  const float* d1e = given1 ? given1 : w;
  const float* d2e = given2 ? given2 : w + 4 * pl;
  float* Hb = w + 8 * pl;
  float* G1 = w + 16 * pl;
  float* G2 = w + 20 * pl;
  const int visc = mu != nullptr;
  PassArgs a = base_args(s, 1);
  set_ref(a, ref, gamma);
  a.u = u;
  a.metric = metric;
  a.mu = mu;
  a.mode = flux;   // FLUX_VISC: the viscous term alone (no flux cotangent)
  // wall patches: theta's derivatives for the energy's product rule (the
  // recorded derivatives already hold the rule's energy lane)
  const bool walls = visc && s->nwchunks > 0;
  const float* D1TH = walls ? s->d_wplanes + pl : nullptr;
  const float* D2TH = walls ? s->d_wplanes + 2 * pl : nullptr;
  if (walls)
    if ((st = wall_theta_derivs(ctx, s, u, ref, gamma, -1))) return st;
  if (visc) {
    PassArgs b = a;
    if (!given1) {
      b.out = w;
      b.plans = s->dir[0].d_plans;
      if ((st = s->a_wide ? launch_lines(s, 1, k_dev_diff2<1>, b, -1, 2) : launch_lines(s, 1, k_dev_diff<1>, b)))
        return st;
      if (walls)
        hipLaunchKernelGGL(k_energy_rule, dim3(chunk_grid(s->nwchunks)), dim3(kBlock), 0, ctx->stream, s->d_wchunks,
                           s->nwchunks, s->d_patches, u, pl, gamma - 1.0f, D1TH, w);
    }
    if (!given2) {
      b.out = w + 4 * pl;
      b.plans = s->dir[1].d_plans;
      if ((st = launch_lines(s, 2, k_dev_diff2<2>, b, -1, 2))) return st;
      if (walls)
        hipLaunchKernelGGL(k_energy_rule, dim3(chunk_grid(s->nwchunks)), dim3(kBlock), 0, ctx->stream, s->d_wchunks,
                           s->nwchunks, s->d_patches, u, pl, gamma - 1.0f, D2TH, w + 4 * pl);
    }
  }
  {
    const DirPlan& D = s->dir[0];
    PassArgs b = a;
    b.plans = D.d_plans;
    b.tiles = D.ts[0].d_tiles;
    hipLaunchKernelGGL(k_adjHb1, dim3((unsigned)D.ts[0].tiles.size()), dim3(D.ts[0].threads), D.ts[0].lds,
                       ctx->stream, b, rhs_bar, Hb);
    if ((st = launch_check(ctx, "adj C"))) return st;
  }
  // the viscous q2 reverse on tiles of all four components, with the q2
  // transpose of G2 in the same tile (not with the split schedule, and not
  // on wall sets, whose energy rule acts on G1 and G2 first)
  const bool wide = visc && !walls && s->wide_ok && s->schedule != FCSD_SCHED_SPLIT;
  {
    const DirPlan& D = s->dir[1];
    PassArgs b = a;
    b.plans = D.d_plans;
    b.tiles = D.ts[1].d_tiles;
    if (wide) {
      b.tiles = D.ts[2].d_tiles;
      hipLaunchKernelGGL(k_adjHb2w, dim3((unsigned)D.ts[2].tiles.size()), dim3(D.ts[2].threads), D.ts[2].lds,
                         ctx->stream, b, rhs_bar, (const float*)Hb, (const float*)d1e, (const float*)d2e, G1, mu_bar,
                         u_bar);
    } else if (visc)
      hipLaunchKernelGGL(k_adjHb2p<true>, dim3((unsigned)D.ts[1].tiles.size()), dim3(D.ts[1].threads), D.ts[1].lds,
                         ctx->stream, b, rhs_bar, Hb, (const float*)d1e, (const float*)d2e, G1, G2, mu_bar, u_bar);
    else
      hipLaunchKernelGGL(k_adjHb2p<false>, dim3((unsigned)D.ts[1].tiles.size()), dim3(D.ts[1].threads), D.ts[1].lds,
                         ctx->stream, b, rhs_bar, Hb, (const float*)d1e, (const float*)d2e, G1, G2, mu_bar, u_bar);
    if ((st = launch_check(ctx, "adj B2"))) return st;
  }
  if (visc) {
    if (walls) {
      // the energy rule transposed: G1, G2 move the energy lane's cotangent
      // onto rho, m and theta's lanes (TB1, TB2), the rule's coefficients
      // add to u_bar; theta's cotangent D1^T TB1 + D2^T TB2 then goes
      // through d theta / d e
      float* TB1 = s->d_wplanes + 3 * pl;
      float* TB2 = s->d_wplanes + 4 * pl;
      float* THB = s->d_wplanes + 5 * pl;
      hipLaunchKernelGGL(k_energy_rule_adj, dim3(chunk_grid(s->nwchunks)), dim3(kBlock), 0, ctx->stream,
                         s->d_wchunks, s->nwchunks, s->d_patches, u, pl, gamma - 1.0f, d1e, D1TH, G1, TB1, u_bar);
      hipLaunchKernelGGL(k_energy_rule_adj, dim3(chunk_grid(s->nwchunks)), dim3(kBlock), 0, ctx->stream,
                         s->d_wchunks, s->nwchunks, s->d_patches, u, pl, gamma - 1.0f, d2e, D2TH, G2, TB2, u_bar);
      hipLaunchKernelGGL(k_fill, dim3(blocks_for(pl)), dim3(kBlock), 0, ctx->stream, THB, 0.f, pl);
      for (int dir = 1; dir <= 2; ++dir) {
        PassArgs c = base_args(s, dir);
        c.in = dir == 1 ? TB1 : TB2;
        c.out = THB;
        c.nf = 1;
        auto kern = dir == 1 ? k_fcdiff<1, true> : k_fcdiff<2, true>;
        if ((st = launch_tiles(s, dir, kern, c, s->d_wtiles[dir - 1], s->nwtiles[dir - 1]))) return st;
      }
      hipLaunchKernelGGL(k_theta_adj, dim3(chunk_grid(s->nwchunks)), dim3(kBlock), 0, ctx->stream, s->d_wchunks,
                         s->nwchunks, s->d_patches, u, pl, gamma - 1.0f, (const float*)THB, u_bar);
      if ((st = launch_check(ctx, "energy rule reverse"))) return st;
    }
    // u_bar += D2^T G2 + D1^T G1 (deviation form: the constant reference has
    // no adjoint; the wide q2 kernel has already added D2^T G2)
    if (!wide)
      if ((st = fc_diff_adj(ctx, s, 2, 4, G2, u_bar, pl))) return st;
    if ((st = fc_diff_adj(ctx, s, 1, 4, G1, u_bar, pl))) return st;
  }
  return FCSD_OK;
}

}  // namespace

extern "C" fcsd_status fcsd_rhs_adj(fcsd_ctx* ctx, const fcsd_set* s, const float* u, const float* metric,
                                    const float* mu, const float ref[4], float gamma, const float* rhs_bar,
                                    float* u_bar, float* mu_bar, int64_t plane, void* ws, size_t ws_bytes) {
  fcsd_status st = check_set(ctx, s, plane);
  if (st) return st;
  if (!u || !metric || !ref || !rhs_bar || !u_bar || !ws) return fail(ctx, FCSD_EINVAL, "fcsd_rhs_adj: null argument");
  if (ws_bytes < ws_bytes_of(s, FCSD_WS_RHS_ADJ)) return fail(ctx, FCSD_EINVAL, "fcsd_rhs_adj: workspace too small");
  return rhs_adj_impl(ctx, s, u, metric, mu, ref, gamma, rhs_bar, u_bar, mu_bar, ws, nullptr, nullptr);
}

extern "C" fcsd_status euler_rhs_adj(fcsd_ctx* ctx, const fcsd_set* s, const float* u, const float* metric,
                                     const float ref[4], float gamma, const float* rhs_bar, float* u_bar,
                                     int64_t plane, void* ws, size_t ws_bytes) {
  fcsd_status st = check_set(ctx, s, plane);
  if (st) return st;
  if (!u || !metric || !ref || !rhs_bar || !u_bar || !ws) return fail(ctx, FCSD_EINVAL, "euler_rhs_adj: null argument");
  if (ws_bytes < ws_bytes_of(s, FCSD_WS_RHS_ADJ)) return fail(ctx, FCSD_EINVAL, "euler_rhs_adj: workspace too small");
  return rhs_adj_impl(ctx, s, u, metric, nullptr, ref, gamma, rhs_bar, u_bar, nullptr, ws, nullptr, nullptr);
}

extern "C" fcsd_status av_apply_adj(fcsd_ctx* ctx, const fcsd_set* s, const float* u, const float* metric,
                                    const float* mu, const float ref[4], const float* rhs_bar, float* u_bar,
                                    float* mu_bar, int64_t plane, void* ws, size_t ws_bytes) {
  fcsd_status st = check_set(ctx, s, plane);
  if (st) return st;
  if (!u || !metric || !mu || !ref || !rhs_bar || !u_bar || !ws)
    return fail(ctx, FCSD_EINVAL, "av_apply_adj: null argument");
  if (ws_bytes < ws_bytes_of(s, FCSD_WS_RHS_ADJ)) return fail(ctx, FCSD_EINVAL, "av_apply_adj: workspace too small");
  return rhs_adj_impl(ctx, s, u, metric, mu, ref, 1.4f, rhs_bar, u_bar, mu_bar, ws, nullptr, nullptr, FLUX_VISC);
}

extern "C" fcsd_status fcsd_stage_adj(fcsd_ctx* ctx, const fcsd_set* s, int stage, const float* ui,
                                      const float* metric, const float* mu, const float ref[4], float gamma,
                                      const float* dt_dev, const float* uout_bar, float* u0_bar, float* ui_bar,
                                      float* acc_bar, float* mu_bar, int64_t plane, void* ws, size_t ws_bytes) {
  fcsd_status st = check_set(ctx, s, plane);
  if (st) return st;
  if (stage < 0 || stage > 4 || !ui || !metric || !ref || !dt_dev || !uout_bar || !u0_bar || !ui_bar || !ws ||
      (stage >= 2 && !acc_bar))
    return fail(ctx, FCSD_EINVAL, "fcsd_stage_adj: bad arguments");
  if (ws_bytes < ws_bytes_of(s, FCSD_WS_STAGE_ADJ)) return fail(ctx, FCSD_EINVAL, "fcsd_stage_adj: workspace too small");
  const long long n4 = 4 * (long long)s->plane;
  float* rb = (float*)ws + 24 * s->plane;
  // register update transposed (rhs_bar written), then the right-hand side's
  hipLaunchKernelGGL(k_rk_adj, dim3(blocks_for(n4)), dim3(kBlock), 0, ctx->stream, stage, dt_dev, uout_bar, u0_bar,
                     ui_bar, acc_bar, rb, n4);
  if ((st = launch_check(ctx, "fcsd_stage_adj rk"))) return st;
  return rhs_adj_impl(ctx, s, ui, metric, mu, ref, gamma, rb, ui_bar, mu ? mu_bar : nullptr, ws, nullptr, nullptr);
}

extern "C" fcsd_status sdnn_infer_adj(fcsd_ctx* ctx, const fcsd_set* s, const float* u, float gamma,
                                      const fcsd_mlp* w, const float* logits_bar, float* feat_bar, int64_t plane,
                                      void* ws, size_t ws_bytes) {
  fcsd_status st = check_set(ctx, s, plane);
  if (st) return st;
  if (!u || !w || !logits_bar || !feat_bar || !ws || !w->W1 || !w->b1 || !w->W2 || !w->b2 || !w->W3 || !w->b3)
    return fail(ctx, FCSD_EINVAL, "sdnn_infer_adj: null argument");
  if (ws_bytes < ws_bytes_of(s, FCSD_WS_AV)) return fail(ctx, FCSD_EINVAL, "sdnn_infer_adj: workspace too small");
  float* phi = carve_av(s, ws).phi;
  hipLaunchKernelGGL(k_proxy, dim3(chunk_grid(s->nchunks)), dim3(kBlock), 0, ctx->stream, s->d_chunks, s->nchunks,
                     s->d_patches, u, (long long)s->plane, gamma, phi, (float*)nullptr);
  MlpPtr m{w->W1, w->b1, w->W2, w->b2, w->W3, w->b3};
  // the padding between patches is not a point: its feature cotangents are left as they are
  hipLaunchKernelGGL(k_sdnn_adj, dim3(chunk_grid(s->nchunks)), dim3(kBlock), sdnn_adj_lds_bytes(), ctx->stream,
                     s->d_chunks, s->nchunks, s->d_patches, (const float*)phi, m, logits_bar, feat_bar,
                     (long long)s->plane);
  return launch_check(ctx, "sdnn_infer_adj");
}

// ======================================================================== reverse mode of a step

extern "C" fcsd_status fcsd_step_adj(fcsd_ctx* ctx, const fcsd_set* s, const fcsd_step_args* a, const float* u_in,
                                     float* u_bar, const float dstate_dparam[4], double* dparam_dev, int64_t plane,
                                     void* ws, size_t ws_bytes) {
  fcsd_status st = check_set(ctx, s, plane);
  if (st) return st;
  if (!a || !a->metric || !a->dt_dev || (!u_in && !a->record) || !u_bar || !ws)
    return fail(ctx, FCSD_EINVAL, "fcsd_step_adj: null argument");
  if (a->dirichlet_mask && (!dstate_dparam || !dparam_dev))
    return fail(ctx, FCSD_EINVAL, "fcsd_step_adj: Dirichlet data needs dstate_dparam and dparam_dev");
  const bool visc_net = a->w != nullptr || a->fixed_tau;
  if (visc_net && (!a->tau || !a->mu || !a->argmax))
    return fail(ctx, FCSD_EINVAL, "fcsd_step_adj: classes need tau, mu and argmax buffers");
  if (ws_bytes < ws_bytes_of(s, FCSD_WS_STEP_ADJ)) return fail(ctx, FCSD_EINVAL, "fcsd_step_adj: workspace too small");
  if (a->filter && !s->filter_on) return fail(ctx, FCSD_EINVAL, "fcsd_step_adj: filter not configured (fcsd_set_filter)");
  const long long pl = s->plane, n4 = 4 * pl;
  float* w = (float*)ws;
  const bool have = a->record != nullptr;  // the forward step recorded what the reverse needs
  float* STG = have ? a->record : w;        // glued stage inputs 0..4
  float* ACC = w + 20 * pl;
  float* OUT = w + 24 * pl;  // step output; with the filter: the glued state before it (PRE)
  float* YB = w + 28 * pl;  // cotangent of the current stage output
  float* UIB = w + 32 * pl; // cotangent of the current stage input
  float* U0B = w + 36 * pl; // cotangent of the glued step input
  float* ACCB = w + 40 * pl;
  float* RB = w + 44 * pl;
  float* MUB = w + 48 * pl;
  float* RWS = w + 49 * pl;  // 24 planes
  AvWs A = carve_av(s, w + 73 * pl);
  hipStream_t sm = ctx->stream;
  auto stg = [&](int k) { return STG + (long long)k * n4; };
  float* PRE = have ? a->record + 5 * n4 + 2 * pl : OUT;
  const float* mu = a->mu ? (have ? a->record + 5 * n4 : a->mu) : nullptr;
  const int32_t* amax = have ? (const int32_t*)(a->record + 5 * n4 + pl) : a->argmax;
  const int flux = mu ? FLUX_FULL : FLUX_INVISCID;
  // forward recomputation with the recorded classes and step size (unless
  // the forward step recorded its stage inputs)
  if (!have) {
    HIPCHK(ctx, hipMemcpyAsync(stg(0), u_in, n4 * sizeof(float), hipMemcpyDeviceToDevice, sm));
    if ((st = glue_impl(ctx, s, stg(0), a->dirichlet_mask, a->dirichlet_state))) return st;
    if (visc_net)
      if ((st = viscosity_impl(ctx, s, stg(0), a->tau, a->gamma, a->mu, a->argmax, A))) return st;
    if (a->filter) {
      HIPCHK(ctx, hipMemcpyAsync(PRE, stg(0), n4 * sizeof(float), hipMemcpyDeviceToDevice, sm));
      if ((st = filter_impl(ctx, s, stg(0), stg(0), a->gamma))) return st;
      if ((st = glue_impl(ctx, s, stg(0), a->dirichlet_mask, a->dirichlet_state))) return st;
    }
  }
  for (int k = 0; k < 5 && !have; ++k) {
    if (k > 0)
      if ((st = glue_impl(ctx, s, stg(k), a->dirichlet_mask, a->dirichlet_state))) return st;
    // the step output is not needed in reverse: with the filter it goes to
    // planes of the right-hand-side workspace that the forward passes leave free
    float* out = k < 4 ? stg(k + 1) : (a->filter ? RWS + 16 * pl : OUT);
    if ((st = rhs_passes(ctx, s, stg(k), a->metric, mu, a->ref, a->gamma, flux, MODE_RK, nullptr, k, stg(0), ACC, out,
                         a->dt_dev, RWS, -1)))
      return st;
  }
  // reverse sweep over the stages (register form, exact transpose)
  const unsigned b4 = blocks_for(n4);
  hipLaunchKernelGGL(k_fill, dim3(b4), dim3(kBlock), 0, sm, U0B, 0.f, n4);
  hipLaunchKernelGGL(k_fill, dim3(b4), dim3(kBlock), 0, sm, ACCB, 0.f, n4);
  hipLaunchKernelGGL(k_fill, dim3(blocks_for(pl)), dim3(kBlock), 0, sm, MUB, 0.f, pl);
  hipLaunchKernelGGL(k_fill, dim3(b4), dim3(kBlock), 0, sm, YB, 0.f, n4);
  hipLaunchKernelGGL(k_axpy, dim3(b4), dim3(kBlock), 0, sm, 1.f, (const float*)u_bar, YB, n4);
  float* yb = YB;
  float* uib = UIB;
  for (int k = 4; k >= 0; --k) {
    float* tgt = k > 0 ? uib : U0B;
    // the stage's u_i cotangent starts from its register-update share
    // (written, not accumulated)
    hipLaunchKernelGGL(k_rk_adj, dim3(b4), dim3(kBlock), 0, sm, k, a->dt_dev, (const float*)yb, U0B, uib, ACCB, RB,
                       n4, true);
    if ((st = launch_check(ctx, "step_adj rk"))) return st;
    const float* g1 = have && mu ? a->record + kRecD1 * pl + k * n4 : nullptr;
    const float* g2 = have && mu ? a->record + kRecD2 * pl + k * n4 : nullptr;
    if ((st = rhs_adj_impl(ctx, s, stg(k), a->metric, mu, a->ref, a->gamma, RB, tgt, mu ? MUB : nullptr, RWS, g1, g2)))
      return st;
    if (k > 0) {
      if ((st = glue_adj_impl(ctx, s, uib, a->dirichlet_mask, dstate_dparam, dparam_dev, stg(k)))) return st;
      float* t = yb;
      yb = uib;
      uib = t;
    }
  }
  const float* vin = stg(0);
  if (a->filter) {
    if ((st = glue_adj_impl(ctx, s, U0B, a->dirichlet_mask, dstate_dparam, dparam_dev, stg(0)))) return st;
    if ((st = filter_adj_impl(ctx, s, PRE, U0B, U0B, a->gamma, RWS))) return st;
    vin = PRE;
  }
  if (visc_net)
    if ((st = av_viscosity_adj(ctx, s, vin, a->tau, amax, a->gamma, MUB, U0B, plane, w + 73 * pl,
                               ws_bytes_of(s, FCSD_WS_AV))))
      return st;
  if ((st = glue_adj_impl(ctx, s, U0B, a->dirichlet_mask, dstate_dparam, dparam_dev, vin))) return st;
  HIPCHK(ctx, hipMemcpyAsync(u_bar, U0B, n4 * sizeof(float), hipMemcpyDeviceToDevice, sm));
  return launch_check(ctx, "fcsd_step_adj");
}
