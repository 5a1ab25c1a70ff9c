/*
 * fcsdnn.h -- C ABI of the MI355X FC-SDNN hot path (libfcsdnn.so).
 *
 * Method: Bruno & Leibovici, "General-domain FC-based shock-dynamics solver
 * I: Basic elements".  Conserved variables e = (rho, rho u, rho v, E) live
 * on logically rectangular patches (Sec. 3.1); every patch is advanced with
 * FC-Gram spectral derivatives along its two parameter directions (Sec. 2.2),
 * the curvilinear chain rule with the inverse-Jacobian metric terms
 * (Sec. 3.3), the network-driven smooth artificial viscosity (Secs. 2.3, 5)
 * and a five-stage SSP Runge-Kutta scheme (Sec. 4.1).
 *
 * Conventions for every entry point below:
 *   - Return value: FCSD_OK or an error code; nothing aborts or throws.  The
 *     message of the last error of a context is fcsd_last_error(ctx).
 *   - Pointers named in/out/u/... are DEVICE pointers owned by the caller
 *     (FP32 unless stated).  The library owns only its context and patch
 *     sets (and the device tables inside them).
 *   - All work is enqueued asynchronously on the context's HIP stream; no
 *     entry point synchronises the device except the *_create functions.
 *   - Plane layout: a "plane" holds one scalar field of all patches.  Patch p
 *     occupies elements [off_p, off_p + n1_p*n2_p) with element (i, j) at
 *     off_p + j*n1_p + i (i along q1 is contiguous).  Multi-field arrays
 *     store field f at base + f*plane.  State field order (rho, rho u, rho v,
 *     E); metric order (dq1/dx, dq1/dy, dq2/dx, dq2/dy).
 *   - Argument errors (null pointers, bad sizes, unsupported FFT lengths)
 *     return FCSD_EINVAL / FCSD_EUNSUPPORTED before anything is launched.
 *   - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef FCSDNN_H
#define FCSDNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FCSD_OK = 0,
  FCSD_EINVAL = 1,       /* invalid argument */
  FCSD_ENOMEM = 2,       /* host or device allocation failed */
  FCSD_EDEVICE = 3,      /* no usable HIP device */
  FCSD_EHIP = 4,         /* a HIP runtime call failed */
  FCSD_EUNSUPPORTED = 5, /* valid but unsupported (e.g. L = N + C not 13-smooth) */
  FCSD_ENONFINITE = 6    /* the state monitor saw a non-finite or non-positive value */
} fcsd_status;

typedef struct fcsd_ctx fcsd_ctx;
typedef struct fcsd_set fcsd_set;

/* One patch (Sec. 3.2.1): n1 x n2 parameter-space points with spacing
 * h = 1/(n-1) along each direction; C1 / C2 continuation points for lines
 * along q1 / q2 (C = 0: the direction is periodic, plain Fourier
 * differentiation with h = 1/n); hhat / htilde the upper / lower bounds of
 * the physical grid spacing (Sec. 5.1 item 6, eq. CFL); internal[s] != 0
 * marks side s = (q1-, q1+, q2-, q2+) as internal (Sec. 3.4), which removes
 * the n_v = 9 nearest lines from the viscosity-generation subgrid (eq.
 * viscosity_generation). */
typedef struct {
  int32_t n1, n2;
  int32_t C1, C2;
  int64_t off;
  double hhat, htilde;
  uint8_t internal[4];
  int32_t reserved;
} fcsd_patch_desc;

/* Create a context on HIP device `device` that enqueues on `stream` (a
 * hipStream_t; NULL = a new non-blocking stream owned by the context).
 * FCSD_EDEVICE when no device is present.  Synchronises once. */
fcsd_status fcsd_ctx_create(int device, void* stream, fcsd_ctx** out);
fcsd_status fcsd_ctx_destroy(fcsd_ctx* ctx);
/* Replace the stream of a context (e.g. torch's current stream). */
fcsd_status fcsd_ctx_set_stream(fcsd_ctx* ctx, void* stream);
/* Message of the last failure on ctx ("" if none).  Owned by ctx. */
const char* fcsd_last_error(const fcsd_ctx* ctx);
/* The hipStream_t the context enqueues on (its own non-blocking stream when
 * created with stream = NULL). */
void* fcsd_ctx_stream(fcsd_ctx* ctx);
/* Block the host until the context's stream is idle. */
fcsd_status fcsd_ctx_sync(fcsd_ctx* ctx);

/* Plane storage of the patches of a set (every plane an entry point takes:
 * state, metric, viscosity, masks, classes, outputs, workspaces). */
enum {
  /* point (i, j) of patch p at off_p + j n1_p + i */
  FCSD_LAYOUT_ROWS = 0,
  /* 8 x 4 blocks (8 points along q1, 4 along q2; 128 bytes): point (i, j)
   * at off_p + 32 ((j/4) nb1_p + i/8) + 8 (j%4) + i%8, nb1_p = ceil(n1_p/8);
   * a patch occupies ceil8(n1_p) ceil4(n2_p) elements, off_p a multiple of
   * 32.  Line tiles along both directions then read whole cache lines. */
  FCSD_LAYOUT_B8X4 = 1
};
/* Build a patch set: validates the descriptors (n >= 2d+1, n <= 4096,
 * 0 <= C <= 256, 1 <= d <= 8, patches inside [0, plane) and disjoint),
 * factors every extension length L = n + C into radices 2..16 (primes up to
 * 13); a line whose L has a larger prime factor has its circulant operators
 * (derivative, filter; Sec. 2.2 eq. fc_der, Sec. 4.3.1 eq. filtering) applied
 * as a cyclic convolution of the smallest 13-smooth length M >= n + L, the
 * line zero-padded to M and the operator's first column wrapped onto it, the
 * same operator exactly in exact arithmetic at about twice the transform
 * work (FCSD_EUNSUPPORTED when M exceeds 8192 or the smallest tile of such
 * lines does not fit a workgroup's LDS), computes the FC-Gram continuation matrices
 * (Sec. 2.2, eq. continuation) in binary128 arithmetic, the FP32 twiddle
 * and derivative-multiplier tables and the tile schedules, and uploads them.
 * `ring_sectors` / `ring_shells` > 0 declare the index-aligned annulus
 * layout (sector s of shell k is patch k*ring_sectors + s, neighbours overlap
 * by 2 n_v + 1 = 19 lines) used by the fringe exchange and by the
 * multi-patch smoothing-blending operator; 0 means independent patches.
 * `layout` (FCSD_LAYOUT_*) fixes the storage of every plane passed to the
 * set's entry points; the blocked layout needs offsets that are multiples of
 * 32 and room for the padded patch. */
fcsd_status fcsd_set_create(fcsd_ctx* ctx, int npatch, const fcsd_patch_desc* patches,
                            int d, int64_t plane, int ring_sectors, int ring_shells,
                            int layout, fcsd_set** out);
fcsd_status fcsd_set_destroy(fcsd_set* set);
/* Launch order of the batched line tiles. */
enum {
  FCSD_ORDER_LPT = 0, /* longest tile first over all patches */
  FCSD_ORDER_XCD = 1  /* whole patches dealt to the 8 dies (one L2 each),
                         balanced by work; the default */
};
/* Re-split the line tiles of a set.  Three tile sets: [0] q1 lines (passes
 * A, C), [1] q2 lines (pass B2, transposes), [2] q2 lines holding two
 * complex lines per grid line (pass B1, the fused B pass).  For each, the
 * workgroup LDS budget in bytes (8 KB .. 160 KB; default 64 KB or the
 * FCSD_LDS_BUDGET environment variable at creation) and the workgroup size
 * (64, 128, 256, 512 or 1024 threads; default 256); and the launch order of
 * all tiles.  Larger budgets mean more lines per tile, fewer workgroups per
 * compute unit; larger workgroups put more threads on each line.  A tile
 * whose smallest storage-aligned size exceeds its budget takes more (a
 * launch takes its largest tile's LDS); the q2 tiles of four complex lines
 * per grid line (the wide fused pass, the reverse mode's q2 pass) share the
 * third budget and workgroup size, and when their tiles exceed it they are
 * built for the device's whole LDS per workgroup with 1024 threads.
 * Synchronises the context's stream and drops captured step graphs.  Returns
 * FCSD_EINVAL for an out-of-range argument.  Used by the autotuner. */
fcsd_status fcsd_set_tune(fcsd_set* set, const int lds_budget[3], const int threads[3], int order);

/* How the line passes of one right-hand side or stage are launched (the
 * schedule of the four passes A, B1, B2, C of the chain-rule right-hand
 * side, Sec. 3.3, eq. general_curvilinear; every schedule gives the same
 * results bit for bit). */
enum {
  FCSD_SCHED_SPLIT = 0,      /* four launches: A, B1, B2, C */
  FCSD_SCHED_FUSED = 1,      /* three launches: A, B1 + B2 on one q2 tile, C (the default) */
  FCSD_SCHED_PERSISTENT = 2, /* one launch per stage: resident workgroups take A, B and C
                                tiles from a queue; a B tile starts once its patch's A
                                tiles are done, a C tile once its patch's B tiles are */
  FCSD_SCHED_FUSED_WIDE = 3   /* three launches like FCSD_SCHED_FUSED, the q2 pass on tiles
                                that hold all eight H fields in LDS (four complex lines per
                                grid line, half as many lines per tile); FCSD_EINVAL when
                                such tiles do not fit a workgroup's LDS */
};
/* Select the schedule of `set` for fcsd_rhs, fcsd_stage and fcsd_step (the
 * per-patch and per-pass entry points always launch the passes one by one).
 * The reverse modes of the right-hand side (fcsd_rhs_adj, av_apply_adj,
 * fcsd_stage_adj, fcsd_step_adj) run their viscous q2 pass on tiles of all
 * four components, fused with the q2 transpose of its output, except with
 * FCSD_SCHED_SPLIT (and on sets with walls); the results agree to FP32
 * rounding (the transposes' tail folds sum in a tile-dependent order).
 * The persistent schedule uses the q1 tile set's workgroup size for every
 * task and the larger of the two tile sets' LDS plus 16 bytes (the queue
 * slot); it needs that to fit the device's LDS per workgroup (budgets of at
 * most 160 KB - 16), else FCSD_EINVAL.  It is used for every stage of sets
 * without wall sides; stages of sets with walls (whose energy rule runs
 * between passes A and B) fall back to the fused schedule.  A dependency
 * wait that gives up (never expected: it would take about a second) sets
 * bit 0 of the word fcsd_stage_errors reads.  Synchronises the context's
 * stream and drops captured step graphs. */
fcsd_status fcsd_set_schedule(fcsd_set* set, int schedule);
/* Read and clear the set's device error word (blocking read).  Bit 0: a
 * persistent stage's dependency wait gave up.  Bit 1: the network weights
 * of a sdnn_infer call (also inside fcsd_step) let the operands of its
 * fp16 matrix products reach the fp16 range -- a bound from the weights,
 * with the features in [-1, 1], on the weights and every hidden activation
 * is 65000 or more (or not finite) -- so its classes and logits are not to
 * be trusted. */
fcsd_status fcsd_stage_errors(fcsd_set* set, int32_t* flags);

/* Bytes of device workspace an operation needs (op: FCSD_WS_*). */
enum { FCSD_WS_RHS = 0, FCSD_WS_AV = 1, FCSD_WS_STEP = 2, FCSD_WS_RHS_ADJ = 3, FCSD_WS_STEP_ADJ = 4,
       FCSD_WS_FILTER_ADJ = 5, FCSD_WS_SMEAR = 6, FCSD_WS_STAGE_ADJ = 7 };
fcsd_status fcsd_workspace_size(const fcsd_set* set, int op, size_t* bytes);

/* ---- FC-Gram line operators (Sec. 2.2) --------------------------------- */

/* Continuation along direction dir (1: q1 lines = rows, 2: q2 lines =
 * columns), eq. continuation: for every line of every patch writes the N
 * samples followed by the C continuation values
 *     tail = A_l Q^T F_l + A_r Q^T F_r.
 * ext holds, per field, the lines of patch 0, then patch 1, ..., each line
 * L = N + C floats; ext_plane = fcsd_ext_size(set, dir) floats per field. */
fcsd_status fcsd_ext_size(const fcsd_set* set, int dir, int64_t* floats);
fcsd_status fc_continue(fcsd_ctx* ctx, const fcsd_set* set, int dir, int nf,
                        const float* in, int64_t plane, float* ext, int64_t ext_plane);
/* Transpose of fc_continue: in_bar += E^T ext_bar. */
fcsd_status fc_continue_adj(fcsd_ctx* ctx, const fcsd_set* set, int dir, int nf,
                            const float* ext_bar, int64_t ext_plane, float* in_bar, int64_t plane);

/* Spectral filter of FC expansions (paper Sec. 4.3.1, eq. filtering).
 * fcsd_set_filter fixes its parameters for the set: every line of length L =
 * N + C has its extension's coefficient at signed wavenumber k multiplied
 * by sigma(2k/L) = exp(-alpha (2k/L)^p) (the paper uses alpha = 10, p = 14).
 * alpha >= 0 finite, p even in [2, 64], else FCSD_EINVAL.  Synchronises the
 * context's stream, uploads the factor tables and drops captured step
 * graphs; until it is called, fcsd_filter and steps with a->filter return
 * FCSD_EINVAL. */
fcsd_status fcsd_set_filter(fcsd_set* set, double alpha, int p);

/* The per-step state filter: for every patch, the one-dimensional filter
 * along q1 lines and then along q2 lines of rho, rho u, rho v and theta =
 * p / rho (eqs. perfect_gas, p_T); E is not filtered but rebuilt as
 * rho theta / (gamma - 1) + |rho u|^2 / (2 rho) (eq. perfect_gas_T).
 * u, out: [4][plane] states; out may equal u (in place).  Points outside
 * the patches are not touched.  Asynchronous on the context's stream. */
fcsd_status fcsd_filter(fcsd_ctx* ctx, const fcsd_set* set, const float* u, float* out, int64_t plane,
                        float gamma);

/* Reverse mode of fcsd_filter at state u: given the cotangent out_bar of
 * the filtered state, writes the cotangent of u to u_bar (may alias
 * out_bar, not u).  Each line filter R S E (S the real symmetric circulant)
 * is transposed as E^T S R^T; the temperature and the rebuilt energy by
 * their vector-Jacobian products.  ws: fcsd_workspace_size(
 * FCSD_WS_FILTER_ADJ) bytes (the filtered state is recomputed there). */
fcsd_status fcsd_filter_adj(fcsd_ctx* ctx, const fcsd_set* set, const float* u, const float* out_bar,
                            float* u_bar, int64_t plane, float gamma, void* ws, size_t ws_bytes);

/* No-slip adiabatic walls (paper Remarks adiabatic_th, adiabatic; Neumann
 * data in the FC continuation, Sec. 2.2).  sides: [npatch][4] flags
 * (q1-, q1+, q2-, q2+; NULL clears every wall).  At every glue (fcsd_glue,
 * every stage of fcsd_step), after the fringe exchange and the Dirichlet
 * overwrite, each point of a wall line gets rho u = rho v = 0 and
 * E = rho theta_w / (gamma - 1), theta_w the value at the wall of the
 * polynomial of degree < d through theta = p / rho at the d - 1 points next
 * to the wall along the grid line that meets it, with zero derivative at
 * the wall (the Neumann continuation's boundary value); rho is left to
 * evolve.  Where two walls meet at a corner, the corner's theta is the
 * tensor product of the two one-sided values over the (d-1)^2 interior
 * points next to it.  On patches with a wall side the right-hand side's
 * energy derivatives (in the viscous flux) are formed by the sum and
 * product rules from those of rho, rho u, rho v and theta (Remark
 * adiabatic).  The set then holds six planes of device memory of its own
 * (theta, its derivatives and reverse-mode scratch) until the walls are
 * cleared or the set is destroyed.  A side shorter than d + 1 points, across
 * or along, returns FCSD_EINVAL.  Host-side set-up, synchronises the
 * context's stream. */
fcsd_status fcsd_set_walls(fcsd_set* set, const uint8_t* sides, float gamma);

/* Map of a patch's grid (fractional indices i, j) to the plane (Sec. 3.1,
 * eqs. mappings, param_S):
 *   FCSD_MAP_CARTESIAN (x, y) = (a0 + i da, b0 + j db);
 *   FCSD_MAP_POLAR     (theta, r) = (a0 + i da, b0 + j db),
 *                      (x, y) = r (cos theta, sin theta);
 *   FCSD_MAP_AFFINE    (x, y) = (x0, y0) + i (ux, uy) + j (vx, vy): the C- and
 *                      I-type patches;
 *   FCSD_MAP_STYPE     the S-type patch of eq. param_S, l(t) + s nu(t) with
 *                      t = a0 + i da, s = b0 + j db, the arc
 *                      l(t) = sum_{k < nmodes} (cx[k] cos kt + sx[k] sin kt,
 *                                               cy[k] cos kt + sy[k] sin kt)
 *                      and nu(t) the unit normal, the tangent l'(t) turned by
 *                      -90 degrees (side = +1) or +90 degrees (side = -1);
 *                      preimages by Newton's method on (t, s).
 * Unused fields are ignored. */
enum { FCSD_MAP_CARTESIAN = 0, FCSD_MAP_POLAR = 1, FCSD_MAP_AFFINE = 2, FCSD_MAP_STYPE = 3 };
typedef struct {
  int32_t kind;
  double a0, da, b0, db;
  double x0, y0, ux, uy, vx, vy;
  double side;
  int32_t nmodes; /* 1 .. 8 */
  double cx[8], sx[8], cy[8], sy[8];
} fcsd_patch_map;

/* Inter-patch communication by interpolation (paper Sec. 3.4.1, Remark
 * overlap_cond) for patches that overlap without sharing grid lines: every
 * point within nf grid lines of an internal side (fcsd_patch_desc.internal)
 * receives, at every glue (fcsd_glue, every stage of fcsd_step), the value
 * interpolated from a donor patch: of the other patches whose grid holds a
 * 3 x 3 stencil around the point's preimage (fractional indices xi, eta,
 * min(xi, n1-1-xi, eta, n2-1-eta) >= 1), the one where that distance is
 * largest (lower index on ties); the stencil is centred on
 * floor(xi + 1/2), floor(eta + 1/2) moved inwards to stay on the grid; the
 * value is iterated quadratic interpolation with Neville's recurrence in the
 * donor's parameters, along q1 on the three rows, then along q2.  Fails
 * with FCSD_EINVAL (and a message naming the point) when a fringe point has
 * no donor or a donor stencil holds fringe points (the decomposition check
 * of the Remark).  The same maps extend the smoothing-blending operator of
 * the viscosity across the patches (eqs. multipatch_W, zeta,
 * multipatch_W_norm): a point that lies in another patch's closed
 * parameter rectangle adds that patch's window sums at the grid point
 * nearest to its preimage (rnd(n + 1/2) = n + 1) to its numerator and
 * denominator.  maps: npatch entries; *nrecv (nullable) receives the number
 * of fringe points.  Not for index-aligned annulus sets (they glue by copy
 * and smooth on one global lattice).  fcsd_glue_adj, av_viscosity_adj and
 * fcsd_step_adj transpose both (the interpolation with the Lagrange weights
 * of the quadratic Neville's recurrence evaluates; accumulated with atomic
 * adds, so their rounding depends on the order).  Host-side set-up,
 * synchronises the context's stream. */
fcsd_status fcsd_set_interp(fcsd_set* set, const fcsd_patch_map* maps, int nf, int64_t* nrecv);

/* Localized discontinuity-smearing of initial data (paper Sec. 4.3.2, eqs.
 * q and qf), applied once before time stepping.  region: [plane] labels,
 * one per point; the initial data is taken as discontinuous between two
 * line neighbours whose labels differ (at the midpoint between them).
 * Along q1 lines, then along q2 lines of the result, each of rho, rho u,
 * rho v and theta = p / rho becomes w F~ + (1 - w) F, with F~ the line
 * filtered by eq. filtering with (alpha, p) (the paper: 10, 2) and w the
 * window of eq. qf in grid units of the line (the paper: c = 18, r = 9):
 * 1 within c/2 of a discontinuity, cos^2(pi (s - c/2) / (2 r)) up to
 * c/2 + r, 0 beyond; discontinuities closer than c + 2 r share one window
 * that is 1 between them.  E is rebuilt (eq. perfect_gas_T) everywhere, so
 * away from discontinuities it changes by rounding only; the other fields
 * of lines without a discontinuity keep their values.  u, out: [4][plane]
 * (out may equal u);
 * ws: fcsd_workspace_size(FCSD_WS_SMEAR) bytes (the two window planes).
 * At most 65535 patches. */
fcsd_status fcsd_smear(fcsd_ctx* ctx, const fcsd_set* set, const float* u, const uint8_t* region, float* out,
                       int64_t plane, float gamma, double alpha, int p, double c, double r, void* ws,
                       size_t ws_bytes);

/* FC derivative d/dq^dir of nf fields (eq. fc_der): continuation, FFT of
 * length L, multiplication by 2 pi i k / beta (beta = L h, h = 1/(N-1);
 * Nyquist of even L set to zero), inverse FFT, restriction to N points.
 * out may not alias in. */
fcsd_status fc_diff(fcsd_ctx* ctx, const fcsd_set* set, int dir, int nf,
                    const float* in, float* out, int64_t plane);
/* Transpose: in_bar += D^T out_bar, D^T = E^T (-S) R^T. */
fcsd_status fc_diff_adj(fcsd_ctx* ctx, const fcsd_set* set, int dir, int nf,
                        const float* out_bar, float* in_bar, int64_t plane);

/* ---- right-hand side (Secs. 2.1, 2.3, 3.3) ------------------------------ */

/* rhs = - div_x f(u) (eq. general_curvilinear, chain-rule form
 * sum_{m,a} dq^m/dx_a d/dq^m f_a).  ref = reference primitive state
 * (rho, u, v, p): fluxes are differentiated in deviation form
 * f(u) - f(u_ref), which leaves the result unchanged up to the FC
 * derivative of a constant.  ws: fcsd_workspace_size(FCSD_WS_RHS) bytes. */
fcsd_status euler_rhs(fcsd_ctx* ctx, const fcsd_set* set, const float* u, const float* metric,
                      const float ref[4], float gamma, float* rhs, int64_t plane,
                      void* ws, size_t ws_bytes);
/* rhs += div_x (mu grad_x u) for all four components (eqs. f_visc,
 * convection diffusion eqn). */
fcsd_status av_apply(fcsd_ctx* ctx, const fcsd_set* set, const float* u, const float* metric,
                     const float* mu, const float ref[4], float* rhs, int64_t plane,
                     void* ws, size_t ws_bytes);
/* rhs = - div_x f(u) + div_x (mu grad_x u) in one pass sequence (mu may be
 * NULL: inviscid). */
fcsd_status fcsd_rhs(fcsd_ctx* ctx, const fcsd_set* set, const float* u, const float* metric,
                     const float* mu, const float ref[4], float gamma, float* rhs, int64_t plane,
                     void* ws, size_t ws_bytes);
/* Reverse mode of fcsd_rhs at the point (u, mu): u_bar += (dL/du)^T rhs_bar,
 * mu_bar += (dL/dmu)^T rhs_bar (mu_bar may be NULL; mu NULL = inviscid). */
fcsd_status fcsd_rhs_adj(fcsd_ctx* ctx, const fcsd_set* set, const float* u, const float* metric,
                         const float* mu, const float ref[4], float gamma, const float* rhs_bar,
                         float* u_bar, float* mu_bar, int64_t plane, void* ws, size_t ws_bytes);

/* Transpose of euler_rhs at u (Secs. 2.1, 3.3, eq. general_curvilinear):
 * u_bar += (d rhs / du)^T rhs_bar, with the flux Jacobians' transposes at
 * every point and the transposed FC derivatives (the deviation reference is
 * a constant and has no cotangent).  rhs_bar [4][plane] is read, u_bar
 * [4][plane] accumulated; ws: fcsd_workspace_size(FCSD_WS_RHS_ADJ) bytes.
 * FCSD_EINVAL for a null pointer or a small workspace. */
fcsd_status euler_rhs_adj(fcsd_ctx* ctx, const fcsd_set* set, const float* u, const float* metric,
                          const float ref[4], float gamma, const float* rhs_bar, float* u_bar,
                          int64_t plane, void* ws, size_t ws_bytes);
/* Transpose of av_apply at (u, mu) (Sec. 2.3, eqs. f_visc, convection
 * diffusion eqn, in the chain-rule form of Sec. 3.3): the term
 * div_x (mu grad_x u) is linear in u for fixed mu and in mu for fixed u;
 * u_bar += its u-transpose applied to rhs_bar, mu_bar (nullable, one plane)
 * += grad_x u . (grad_x-divergence transpose of rhs_bar).  Accumulates;
 * ws: FCSD_WS_RHS_ADJ bytes; mu is required. */
fcsd_status av_apply_adj(fcsd_ctx* ctx, const fcsd_set* set, const float* u, const float* metric,
                         const float* mu, const float ref[4], const float* rhs_bar, float* u_bar,
                         float* mu_bar, int64_t plane, void* ws, size_t ws_bytes);

/* ---- time stepping (Sec. 4.1) ------------------------------------------ */

/* One stage s = 0..4 of the five-stage fourth-order SSP Runge-Kutta scheme
 * in three-register form on 4 fields:
 *   s=0: uout = u0 + b0 dt r
 *   s=1: uout = a10 u0 + a11 ui + b1 dt r
 *   s=2: uout = a20 u0 + a22 ui + b2 dt r ;  acc  = a42 ui
 *   s=3: uout = a30 u0 + a33 ui + b3 dt r ;  acc += a43 ui + b43 dt r
 *   s=4: uout = acc + a44 ui + b4 dt r
 * (ui = output of the previous stage, r = L(ui), dt read from dt_dev).
 * uout may alias u0 at s = 4 only. */
fcsd_status rk_stage(fcsd_ctx* ctx, const fcsd_set* set, int stage, const float* dt_dev,
                     const float* rhs, const float* u0, const float* ui, float* acc, float* uout,
                     int64_t plane);
/* Reverse of rk_stage: given uout_bar (and acc_bar for s <= 3 after s = 4),
 * accumulates u0_bar, ui_bar, rhs_bar (= dt-scaled) and acc_bar in place. */
fcsd_status rk_stage_adj(fcsd_ctx* ctx, const fcsd_set* set, int stage, const float* dt_dev,
                         const float* uout_bar, float* u0_bar, float* ui_bar, float* acc_bar,
                         float* rhs_bar, int64_t plane);

/* dt = (1/pi) min_p cfl / (max S/h~_p + max mu/h~_p^2), S = |u|+|v|+a
 * (eq. CFL); written to dt_dev[0].  mu may be NULL. */
fcsd_status fcsd_cfl_dt(fcsd_ctx* ctx, const fcsd_set* set, const float* u, const float* mu,
                        float cfl, float gamma, float* dt_dev, int64_t plane,
                        void* ws, size_t ws_bytes);

/* fcsd_cfl_dt for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same result, with the per-patch maxima kept in a static device array
 * of the library (two words per patch) instead of a workspace.  Allocates
 * nothing and calls no allocating routine.  At most 16384 patches
 * (FCSD_EINVAL beyond, before any launch).  The array is one per device and
 * shared by every call on it; each call clears it (fill kernel, no memset)
 * before use, and calls that overlap on one device (different streams,
 * threads or contexts of the same device) race on it. */
fcsd_status fcsd_cfl_dt_noalloc(fcsd_ctx* ctx, const fcsd_set* set, const float* u, const float* mu,
                                float cfl, float gamma, float* dt_dev, int64_t plane);

/* State monitor (the admissibility the paper reports its runs keep without
 * limiters, Remark adiabatic_th: positive density and pressure): over the
 * grid points of every patch of a state u [4][plane] (padding is not looked
 * at), *flags_dev (one int32 in device memory, overwritten, stream-ordered)
 * becomes the OR of 1 (a non-finite component), 2 (rho <= 0) and 4
 * (p = (gamma - 1)(E - |m|^2 / (2 rho)) <= 0, or not a number); 0 when the
 * state is admissible.  No host synchronisation.  FCSD_EINVAL for a null
 * pointer or gamma <= 1. */
fcsd_status fcsd_check(fcsd_ctx* ctx, const fcsd_set* set, const float* u, float gamma,
                       int32_t* flags_dev, int64_t plane);

/* ---- network-driven viscosity (Sec. 5) ---------------------------------- */

/* Network weights (device FP32, row-vector convention y = x W + b):
 * W1 [16][64], b1 [64], W2 [64][64], b2 [64], W3 [64][4], b3 [4]. */
typedef struct {
  const float *W1, *b1, *W2, *b2, *W3, *b3;
} fcsd_mlp;

/* Smoothness classes tau (int8 plane; 0 outside the viscosity-generation
 * subgrid) from the proxy Phi = |u| sqrt(rho/(gamma p)) (Sec. 5.1): per
 * point and direction, the 16-sample window of Phi at offsets -8..7 (indices
 * clamped to the line) rescaled to [-1, 1] feeds the 16-64-64-4 ReLU
 * network; tau = 1 + argmax (lowest index on ties), 2D class = min of the two
 * directions.  logits (nullable): FP32 [2][plane][4] network outputs.
 * The products run on the fp16 matrix cores with every operand split into
 * an fp16 high part and a scaled fp16 low part (FP32 accuracy); weights that
 * could take an operand out of the fp16 range set bit 1 of the set's error
 * word (fcsd_stage_errors).
 * ws: fcsd_workspace_size(FCSD_WS_AV) bytes. */
fcsd_status sdnn_infer(fcsd_ctx* ctx, const fcsd_set* set, const float* u, float gamma,
                       const fcsd_mlp* w, int8_t* tau, float* logits, int64_t plane,
                       void* ws, size_t ws_bytes);

/* mu = Lambda[mu^], mu^ = R(tau) max_{7x7} S h^ on the viscosity-generation
 * subgrid (eqs. V2D_unscaled, W, multipatch_W_norm, Lambda), R = (1.5, 1,
 * 0.5, 0), window cos^2(pi k/18), |k| <= 8.  argmax (nullable): int32 plane
 * of the patch-local flat index of each 7x7 maximiser (first in row-major
 * order on ties).  ws: fcsd_workspace_size(FCSD_WS_AV). */
fcsd_status av_viscosity(fcsd_ctx* ctx, const fcsd_set* set, const float* u, const int8_t* tau,
                         float gamma, float* mu, int32_t* argmax, int64_t plane,
                         void* ws, size_t ws_bytes);
/* u_bar += (dmu/du)^T mu_bar with tau and argmax frozen. */
fcsd_status av_viscosity_adj(fcsd_ctx* ctx, const fcsd_set* set, const float* u, const int8_t* tau,
                             const int32_t* argmax, float gamma, const float* mu_bar, float* u_bar,
                             int64_t plane, void* ws, size_t ws_bytes);

/* ---- multi-patch glue (Secs. 3.4, 4.2) ---------------------------------- */

/* In-place fringe copy (n_f = 5 lines from the index-aligned neighbour;
 * sectors first, then shells) followed by the Dirichlet overwrite with
 * `dirichlet_state` (4 floats, host) on the points flagged in the uint8
 * plane `dirichlet_mask` (nullable).  No-op for independent patches. */
fcsd_status fcsd_glue(fcsd_ctx* ctx, const fcsd_set* set, float* u, int64_t plane,
                      const uint8_t* dirichlet_mask, const float dirichlet_state[4]);
/* Transpose of fcsd_glue on a cotangent u_bar (in place): the wall
 * condition's transpose at the glued state `glued` ([4][plane], the output
 * of the fcsd_glue being reversed; required on sets with walls, else
 * FCSD_EINVAL, and may be NULL without walls), then the Dirichlet points'
 * cotangent is dotted with dstate_dparam (4 floats, host) into
 * dparam_dev[0] (device FP64, incremented) and zeroed; then every fringe
 * receiver's cotangent moves onto its donor (shells, then sectors).
 * dstate_dparam / dparam_dev may be NULL without a mask. */
fcsd_status fcsd_glue_adj(fcsd_ctx* ctx, const fcsd_set* set, float* u_bar, int64_t plane,
                          const uint8_t* dirichlet_mask, const float dstate_dparam[4],
                          double* dparam_dev, const float* glued);

/* Transpose of the classifier network (Sec. 5.1) at the features of the
 * state u: for every point of the viscosity-generation subgrid and each
 * direction d = 0, 1 (q1, q2 lines), feat_bar[d][p][0..15] = the cotangent
 * of the 16 window features given logits_bar[d][p][0..3], through the ReLU
 * masks of the forward pass at those features (the solver's reverse mode
 * freezes the classes and does not use this).  Layouts [2][plane][4] and
 * [2][plane][16] at each point's storage index; feat_bar is overwritten at
 * grid points (zero outside the subgrid), padding untouched.  ws:
 * FCSD_WS_AV bytes.  FCSD_EINVAL for a null pointer or weight. */
fcsd_status sdnn_infer_adj(fcsd_ctx* ctx, const fcsd_set* set, const float* u, float gamma,
                           const fcsd_mlp* w, const float* logits_bar, float* feat_bar, int64_t plane,
                           void* ws, size_t ws_bytes);

/* ---- fused stage and step ------------------------------------------------ */

/* One fused SSPRK stage: right-hand side of ui (with viscosity mu, NULL =
 * inviscid) and the register update of rk_stage, batched over all patches
 * (4 passes, one launch each). */
fcsd_status fcsd_stage(fcsd_ctx* ctx, const fcsd_set* set, int stage, const float* u0,
                       const float* ui, float* acc, float* uout, const float* metric,
                       const float* mu, const float ref[4], float gamma, const float* dt_dev,
                       int64_t plane, void* ws, size_t ws_bytes);
/* Reverse mode of fcsd_stage (Sec. 4.1) at its input ui, mu fixed: the
 * register update transposed (as rk_stage_adj: u0_bar and ui_bar
 * accumulated, acc_bar read and updated for stages >= 2, the dt-scaled
 * right-hand-side cotangent formed in the workspace), then the right-hand
 * side's transpose at ui added to ui_bar and, when mu and mu_bar are given,
 * to mu_bar.  At stage 0 the right-hand side is evaluated at u0: pass the
 * same buffer as u0_bar and ui_bar to collect both parts.  ws:
 * fcsd_workspace_size(FCSD_WS_STAGE_ADJ) bytes. */
fcsd_status fcsd_stage_adj(fcsd_ctx* ctx, const fcsd_set* set, int stage, const float* ui,
                           const float* metric, const float* mu, const float ref[4], float gamma,
                           const float* dt_dev, const float* uout_bar, float* u0_bar, float* ui_bar,
                           float* acc_bar, float* mu_bar, int64_t plane, void* ws, size_t ws_bytes);

/* One of the four passes of fcsd_stage (0: q1 derivatives of the state,
 * 1: q2 derivatives and the combined fluxes H, 2: q2 derivatives of H,
 * 3: q1 derivatives of H and the register update), or 4: passes 1 and 2 in
 * one launch (the fused schedule's q2 pass), 5: the same on tiles holding
 * all eight H fields (the wide fused schedule's), for timing and profiling.
 * Running passes 0..3 (or 0, 4, 3) in order equals one fcsd_stage call;
 * with mu == NULL passes 0 and 1 together are the pointwise inviscid H. */
fcsd_status fcsd_stage_pass(fcsd_ctx* ctx, const fcsd_set* set, int pass, int stage, const float* u0,
                            const float* ui, float* acc, float* uout, const float* metric,
                            const float* mu, const float ref[4], float gamma, const float* dt_dev,
                            int64_t plane, void* ws, size_t ws_bytes);

/* Per-patch plain variant of fcsd_stage: the same kernels launched once per
 * patch (npatch launches per pass). */
fcsd_status fcsd_stage_per_patch(fcsd_ctx* ctx, const fcsd_set* set, int stage, const float* u0,
                                 const float* ui, float* acc, float* uout, const float* metric,
                                 const float* mu, const float ref[4], float gamma,
                                 const float* dt_dev, int64_t plane, void* ws, size_t ws_bytes);

/* Step state kept by the library for fcsd_step. */
typedef struct {
  float* u;             /* [4][plane] state, advanced in place */
  const float* metric;  /* [4][plane] */
  float* mu;            /* [plane] viscosity (output when w != NULL, else input) */
  int8_t* tau;          /* [plane] classes (used when w != NULL) */
  int32_t* argmax;      /* [plane] 7x7 maximisers (nullable) */
  float* dt_dev;        /* [1] step size (output unless fixed_dt) */
  const uint8_t* dirichlet_mask;  /* nullable */
  float dirichlet_state[4];
  float ref[4];
  float gamma, cfl;
  int fixed_dt;         /* 1: use *dt_dev as given */
  const fcsd_mlp* w;    /* NULL: mu given (unless fixed_tau) */
  int fixed_tau;        /* 1: classes given in tau (network not run), mu
                           computed from them: replays a recorded step */
  int filter;           /* 1: apply the spectral filter configured by
                           fcsd_set_filter after the viscosity (then glue
                           again), before the step size */
  float* record;        /* nullable [FCSD_RECORD_PLANES][plane]: fcsd_step
                           stores what its reverse mode needs (below) and
                           fcsd_step_adj reads it instead of recomputing
                           the forward step */
} fcsd_step_args;

/* Planes of a step record: 0..19 the five glued stage inputs [5][4][plane]
 * (stage 0 = the state after glue, viscosity and filter), 20 mu, 21 the 7x7
 * maximisers as int32 (with classes), 22..25 the glued state before the
 * filter (with a->filter), 26..45 and 46..65 the q1 and q2 FC derivatives
 * of e - e_ref of every stage input [5][4][plane] (with a viscosity). */
#define FCSD_RECORD_PLANES 66

/* One full time step (Algorithm 1): glue, network classes and viscosity
 * (when w != NULL), spectral filter and glue (when a->filter), step size,
 * five fused stages with glue on every stage input.  use_graph = 1 captures
 * the step once into a hipGraph and replays it on later calls with identical
 * arguments; the set keeps the graphs of its 8 most recent argument sets
 * (capturing a ninth synchronises the stream and drops the oldest), and a
 * capture whose body fails is discarded.  With a->record the stage
 * inputs, mu, the maximisers (argmax required then, with classes) and the
 * pre-filter state are written to the record as well; the step's result is
 * the same. */
fcsd_status fcsd_step(fcsd_ctx* ctx, const fcsd_set* set, const fcsd_step_args* a,
                      int64_t plane, void* ws, size_t ws_bytes, int use_graph);

/* Reverse mode of fcsd_step with the step's decisions frozen (classes tau,
 * step size *dt_dev; the 7x7 maximisers are recomputed and equal the
 * recorded ones): given the cotangent of the step output in u_bar, replaces
 * it by the cotangent of the step input u_in (the state before the first
 * glue; not modified).  The forward step is recomputed from u_in into the
 * workspace, unless a->record holds the record that fcsd_step wrote for this
 * step with the same arguments (then u_in may be NULL, nothing is
 * recomputed and mu and argmax are read from the record).  With a Dirichlet mask, dparam_dev[0] (device FP64) is
 * incremented by u_bar_glued . dstate_dparam summed over the flagged points
 * of every glue, i.e. the derivative through the boundary state with
 * respect to a scalar parameter whose state derivative (4 floats, host) is
 * dstate_dparam.  Classes and viscosity follow a->w / a->fixed_tau as in
 * fcsd_step (tau, mu, argmax buffers required then; mu is rewritten);
 * constant mu (a->w == NULL, fixed_tau == 0) is not differentiated.
 * ws: fcsd_workspace_size(FCSD_WS_STEP_ADJ) bytes (paper Sec. 4, Algorithm 1,
 * transposed stage by stage; with a->filter the spectral filter and the
 * glue after it are transposed too). */
fcsd_status fcsd_step_adj(fcsd_ctx* ctx, const fcsd_set* set, const fcsd_step_args* a,
                          const float* u_in, float* u_bar, const float dstate_dparam[4],
                          double* dparam_dev, int64_t plane, void* ws, size_t ws_bytes);

/* ---- host-only helpers (no device needed) ------------------------------- */

/* FC-Gram continuation matrix A_r Q^T (C x d, row-major FP64) exactly as the
 * library builds it; A_l Q^T[m][j] = A_r Q^T[C-1-m][d-1-j]. */
fcsd_status fcsd_fc_matrix(int d, int C, double* out);
/* Checks a patch table exactly as fcsd_set_create does, without a device;
 * writes a message into msg (msglen bytes) on failure. */
fcsd_status fcsd_validate_patches(int npatch, const fcsd_patch_desc* patches, int d, int64_t plane,
                                  int ring_sectors, int ring_shells, int layout, char* msg,
                                  int msglen);
/* Radix factorisation of L (returns FCSD_EUNSUPPORTED if none). */
fcsd_status fcsd_fft_plan(int L, int* nstages, int radices[8]);
const char* fcsd_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FCSDNN_H */
