/*
 * dpvba.h -- C ABI of the patch-graph Gauss-Newton bundle adjustment library
 * (gfx950 / MI355X).
 *
 * The problem is the one stated in the DPV-SLAM paper (Lipson, Teed, Deng,
 * arXiv 2408.01654), Sec. 3.1: frames i with camera-to-world poses G_i, p x p
 * patches P_ik owned by frame i with an inverse depth, a directed edge set of
 * (i, k, j) linking patch k of frame i to frame j, per-edge ideal
 * reprojections I_ikj ("targets") and confidences w_ikj ("weights").  The
 * reprojection is eq. (2), P'_ikj = Pi[G_j^-1 G_i Pi^-1(P_ik)], and bundle
 * adjustment minimises eq. (3), the confidence-weighted sum of squared
 * differences between reprojections and targets.  The solver eliminates the
 * per-patch depths by a Schur complement and factors the reduced pose block
 * by Cholesky (Appendix A), serving both the sliding-window BA of the
 * odometry (Sec. 3.1) and the global BA after a proximity loop closure
 * (Sec. 3.2).
 *
 * Readings fixed by this library where the paper is silent:
 *   - one inverse depth per patch; only the patch centre enters the residual
 *     (the whole patch is available through dpvba_reproject);
 *   - cost = 1/2 sum_e (w_x r_x^2 + w_y r_y^2): confidences multiply;
 *   - poses are camera-to-world (tx,ty,tz,qx,qy,qz,qw), unit quaternion,
 *     updated on the right, G <- G Exp(xi), xi = (rho, phi), full SE(3) Exp;
 *   - damping H~ = H + lambda (Diag(H) + I) on the full system;
 *   - an edge is valid iff d_k > 0 and q_z > z_min d_k (q the point in the
 *     target camera scaled by d_k); invalid edges contribute nothing;
 *   - poses [0, n_fixed) are held, all depths are free;
 *   - a fixed number of iterations, no step rejection.
 *
 * Memory and ownership.  Unless marked "host", every pointer is a device
 * pointer owned by the caller, who keeps it alive until the work enqueued on
 * the given stream has completed.  The library never frees or retains caller
 * buffers.  A context owns all of its workspace.  The analyses
 * (dpvba_analyze, dpvba_analyze_batch) are the only calls that allocate
 * device memory; the numeric calls (dpvba_solve, dpvba_solve_backward,
 * dpvba_reduced_system, dpvba_reproject, dpvba_solve_batch) allocate
 * nothing and only enqueue work on the caller's stream (a non-NULL report
 * is one device-to-host copy into it, read by the caller after
 * synchronising the stream).  The exception to "no synchronisation" is the
 * float64 fallback decision of DPVBA_MIXED on reduced systems whose solve is
 * not one workgroup's (see dpvba_solve).  A context is used by one host
 * thread at a time.
 *
 * Errors.  Every call returns a dpvba_status.  Argument errors found on the
 * host return immediately with nothing enqueued.  Conditions found on the
 * device are reported through dpvba_report.status once the stream has
 * completed; failures that invalidate results (an expired bounded wait,
 * invalid inputs) are also recorded in the context and returned as
 * DPVBA_EDEVICE by every later call (dpvba_device_status).  No C++
 * exception crosses this interface and nothing aborts.
 */
#ifndef DPVBA_H
#define DPVBA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DPVBA_OK = 0,
  DPVBA_EINVAL = 1,   /* bad argument, index out of range, inconsistent patch owner */
  DPVBA_ENOTPD = 2,   /* reduced camera system not positive definite            */
  DPVBA_ENOMEM = 3,   /* device allocation failed (dpvba_analyze / create)       */
  DPVBA_EHIP = 4,     /* a HIP runtime call failed                               */
  DPVBA_ESTATE = 5,   /* numeric call without a matching dpvba_analyze           */
  DPVBA_EDEVICE = 6,  /* an earlier call's device work failed: a bounded device-
                         wide wait expired, or it met a target / weight outside
                         the documented range; see dpvba_device_status          */
  DPVBA_ELIMIT = 7    /* the problem exceeds a fixed capacity of the call
                         (dpvba_solve_noalloc) or an output's capacity
                         (dpvba_proximity_edges); dpvba_last_error says which   */
} dpvba_status;

typedef enum {
  DPVBA_FP32 = 0,       /* float32 assembly, factorisation and solve             */
  DPVBA_MIXED = 1,      /* float32 assembly and state; shares gathered in float64;
                           float32 Cholesky refined against the float64 residual,
                           float64 Cholesky when that does not converge          */
  DPVBA_FP64 = 2        /* float64 throughout (parity mode)                      */
} dpvba_precision;

typedef struct dpvba_ctx dpvba_ctx;

/* One BA problem (paper Sec. 3.1, eq. 1-3).  Host struct holding device
 * pointers.
 *   n_frames   N, number of poses.
 *   n_patches  P, number of patches (patch k has one inverse depth).
 *   n_edges    E, number of edges (i, k, j).
 *   patch_size p, odd, >= 1.
 *   n_fixed    poses [0, n_fixed) are held constant (gauge); 0 <= n_fixed <= N.
 *   patches    [P, p, p, 2] float32: pixel (x, y) of each patch pixel in its
 *              source frame; row a, column b; the centre ((p-1)/2, (p-1)/2)
 *              enters the residual.
 *   ii, jj, kk [E] int32: source frame, target frame, patch of every edge.
 *              0 <= ii, jj < N, ii != jj, 0 <= kk < P, and every edge of one
 *              patch has the same ii (the patch's owner frame).  Any order;
 *              duplicated edges add up.
 *   target     [E, 2] float32: ideal reprojection I_ikj in pixels.
 *   weight     [E, 2] float32: confidence w_ikj (x, y), finite and >= 0.
 *   fx..cy     pinhole intrinsics shared by every frame.                  */
typedef struct {
  int32_t n_frames, n_patches, n_edges, patch_size, n_fixed;
  const float* patches;
  const int32_t* ii;
  const int32_t* jj;
  const int32_t* kk;
  const float* target;
  const float* weight;
  float fx, fy, cx, cy;
} dpvba_graph;

/* Solver options (host).
 *   n_iters    Gauss-Newton iterations, 0 <= n_iters <= DPVBA_MAX_ITERS.
 *   lambda     damping, finite, >= 0 (rounded to float in DPVBA_FP32).
 *   z_min      validity threshold, finite, >= 0.
 *   precision  dpvba_precision.
 *   flags      0 or an OR of the DPVBA_FLAG_* bits below; any other bit is
 *              EINVAL.                                                   */
#define DPVBA_MAX_ITERS 32
/* Damping H~ = H + lambda I (Levenberg) instead of the default
 * H + lambda (Diag(H) + I) (Levenberg-Marquardt).  Every numeric call.     */
#define DPVBA_FLAG_LEVENBERG 2u
/* DPVBA_MIXED only: solve every iteration with the float64 Cholesky, as if
 * the refined float32 solve had not converged (the float32 factor,
 * refinement and report fields are still computed).  EINVAL otherwise.    */
#define DPVBA_FLAG_FORCE_FP64_CHOL 4u
/* DPVBA_MIXED only: no refinement steps; the float64 residual of the plain
 * float32 solve decides the fallback.  EINVAL otherwise.                  */
#define DPVBA_FLAG_NO_REFINE 8u
typedef struct {
  int32_t n_iters;
  int32_t precision;
  double lambda;
  double z_min;
  uint32_t flags;
} dpvba_opts;

/* Per-solve report, written asynchronously into host memory (pinned
 * memory recommended) and valid after the stream has completed.
 *   cost[t]         1/2 sum w r^2 over valid edges at iterate t (t <= n_iters),
 *                   accumulated in float64.
 *   n_invalid[t]    invalid edges at iterate t (t < n_iters).
 *   min_pivot[t]    smallest L_ii^2 / S_ii of the Cholesky at iteration t.
 *   status          DPVBA_OK, DPVBA_ENOTPD if a pivot was not positive
 *                   (that iteration's step is then zero), DPVBA_EINVAL if a
 *                   target or weight was non-finite or a weight negative
 *                   (the edge is used as given; the results follow that
 *                   arithmetic), or DPVBA_EHIP if a bounded device-wide wait
 *                   expired (the results are then invalid).
 *   refine_resid[t] DPVBA_MIXED: max |s - S dxi| / max |s| in float64 after
 *                   the refinement steps of iteration t (before any float64
 *                   fallback); 0 in the other modes.
 *   fp64_fallback[t] DPVBA_MIXED: 1 if iteration t was re-solved with the
 *                   float64 Cholesky.                                      */
typedef struct {
  int32_t status;
  int32_t n_iters;
  double cost[DPVBA_MAX_ITERS + 1];
  int32_t n_invalid[DPVBA_MAX_ITERS];
  double min_pivot[DPVBA_MAX_ITERS];
  double refine_resid[DPVBA_MAX_ITERS];
  int32_t fp64_fallback[DPVBA_MAX_ITERS];
} dpvba_report;

/* Create a context on HIP device `device`.  Allocates the context's fixed
 * state.  Returns EINVAL for a bad device, ENOMEM/EHIP on failure.        */
dpvba_status dpvba_create(dpvba_ctx** out, int32_t device);

/* Release the context and all of its device memory.  NULL is ignored.   */
void dpvba_destroy(dpvba_ctx* ctx);

/* Symbolic analysis of the edge set (ii, jj, kk) and sizes of `g` (the
 * structure of the block-sparse normal equations of eq. 3, Appendix A):
 * groups every patch's edges, splits each source frame's patches into
 * tiles, and builds the index lists that assemble the reduced camera
 * system.  Copies ii/jj/kk, targets and weights to the host (synchronising
 * `stream`), validates them (weights finite and >= 0, targets finite), and
 * (re)allocates the workspace for this graph, including that of
 * dpvba_solve_backward for up to DPVBA_MAX_ITERS iterations.  Must be repeated
 * whenever ii, jj, kk or any size changes; targets, weights, patches,
 * poses and depths may change freely between numeric calls.
 * Returns EINVAL on any index or ownership violation, ENOMEM on allocation
 * failure.                                                                */
dpvba_status dpvba_analyze(dpvba_ctx* ctx, const dpvba_graph* g, void* stream);

/* Tile-shape choice of the analysis (host).  A tile is a run of at most
 * tile_patches_* patches of one source frame; 0 selects the default (96 for
 * the float32 plan, 32 for the float64 plan).  Larger tiles write smaller
 * partial systems; smaller tiles expose more workgroups.  Both plans are
 * built by every analysis.
 * keep_order: 0 lets the analysis factor a reduced system of more than 252
 * unknowns in a reverse Cuthill-McKee order of the free poses (a symmetric
 * permutation: the same solution, a smaller envelope of fill when loop
 * closures couple distant keyframes; kept only if it shrinks the envelope),
 * 1 keeps the poses' own order.  Results are reported in the poses' order
 * either way.                                                             */
typedef struct {
  int32_t tile_patches_fp32;
  int32_t tile_patches_fp64;
  int32_t keep_order;
} dpvba_tuning;

/* dpvba_analyze with explicit tile shapes (tune may be NULL).  EINVAL for
 * negative entries or keep_order outside {0, 1}.                          */
dpvba_status dpvba_analyze_ex(dpvba_ctx* ctx, const dpvba_graph* g, const dpvba_tuning* tune,
                              void* stream);

/* Sizes of the plan that the last successful analysis built for one
 * precision (host struct).
 *   n_tiles        tiles (runs of one source frame's patches).
 *   n_free         free poses N - n_fixed; the reduced system is 6 n_free.
 *   part_S_elems   elements of the tiles' partial reduced systems.
 *   part_vec_elems elements of the tiles' partial right-hand sides and
 *                  damping diagonals.
 *   grid_cells     (patch, target slot) cells of all tiles (>= n_edges).
 *   u_elems        elements of the stored Schur rows.
 *   lds_bytes      shared memory of the largest tile.
 * Returns EINVAL for a bad precision, ESTATE before a successful analysis. */
typedef struct {
  int32_t n_tiles, n_free;
  int64_t part_S_elems, part_vec_elems, grid_cells, u_elems;
  int32_t lds_bytes, pad;
} dpvba_analysis_info;

dpvba_status dpvba_get_analysis_info(const dpvba_ctx* ctx, int32_t precision,
                                     dpvba_analysis_info* info);

/* Order of the free poses in the factored reduced system (host): block row
 * p of the Cholesky factor is free pose order[p] (0-based among the free
 * poses; pose n_fixed + order[p] of the graph).  The identity when the
 * analysis kept the poses' own order.  Envelope fill (DPV-SLAM Appendix A:
 * the Cholesky of the pose block is the solve's cost) follows this order.
 *   order  [n] int32 (written), n = n_free of the analysis.
 * EINVAL for a NULL order or a different n, ESTATE before an analysis.    */
dpvba_status dpvba_get_system_order(const dpvba_ctx* ctx, int32_t* order, int32_t n);

/* Reprojection of every edge's whole patch (eq. 2) with the patch's one
 * inverse depth.
 *   poses      [N, 7] float32, inv_depth [P] float32 (read).
 *   coords     [E, p, p, 2] float32 (written): reprojected pixel (x, y).
 *   valid      [E] uint8 or NULL (written): the centre validity rule with
 *              threshold z_min (>= 0).
 * Needs no analysis.  EINVAL on bad sizes or NULL pointers.               */
dpvba_status dpvba_reproject(dpvba_ctx* ctx, const dpvba_graph* g, const float* poses,
                             const float* inv_depth, float z_min, float* coords,
                             uint8_t* valid, void* stream);

/* Sim(3) pose-graph optimisation of the classical loop closure (Sec. 3.3,
 * "Optimization", eq. 5-7).  Every keyframe gets an absolute similarity
 * S_i = (R_i, t_i, s_i), x -> s_i R_i x + t_i, initialised from its pose
 * with scale 1; smoothness residuals r_i = log(DeltaS_(i,i+1)^-1 S_i^-1
 * S_(i+1)) with DeltaS_(i,i+1) = S_i^-1 S_(i+1) of the initial similarities,
 * loop residuals r_jk = log(DeltaS^loop_jk S_j^-1 S_k); sum |r|^2 minimised
 * by n_iters damped Gauss-Newton (Levenberg-Marquardt) steps with
 * H~ = H + lambda (Diag(H) + I) (H + lambda I with DPVBA_FLAG_LEVENBERG), a
 * fixed lambda and no step rejection, right perturbations S <- S Exp(xi),
 * xi = (rho, phi, sigma), Exp(xi) = expm([[sigma I + [phi]x, rho], [0, 0]]).
 * The first n_fixed similarities are held (the objective is invariant to a
 * global similarity).  Float64 throughout; the dense 7 (N - n_fixed) system is
 * factored by the library's Cholesky.
 *   poses     [N, 7] float64 camera-to-world (t, q) (read).
 *   loop_j, loop_k  host [L] int32: loop frame pairs, j != k.
 *   loop_rel  [L, 8] float64 (t, q, s): DeltaS^loop_jk (read).
 *   sims      [N, 8] float64 (written): the optimised (t, q, s).
 *   cost      host [n_iters + 1] or NULL: sum |r|^2 before each iteration
 *             and at the end.
 * The call builds its block lists on the host, allocates its workspace in
 * the context (a dense (7 (N - n_fixed))^2 float64 system, N - n_fixed <=
 * 2857), and synchronises `stream` at the end.  Returns DPVBA_ENOTPD if an
 * iteration's system was not positive definite (its step was skipped).
 * EINVAL for bad sizes, indices or flags.                                  */
#define DPVBA_MAX_PGO_ITERS 64
dpvba_status dpvba_pgo_sim3(dpvba_ctx* ctx, int32_t n_frames, int32_t n_fixed, const double* poses, int32_t n_loops,
                            const int32_t* loop_j, const int32_t* loop_k, const double* loop_rel, int32_t n_iters,
                            double lambda, uint32_t flags, double* sims, double* cost, void* stream);

/* The last step of Sec. 3.3: G_i <- (t_i, R_i) and d <- d / s_i for the
 * patches of frame i, [patch_off[i], patch_off[i+1]) (patch_off [N + 1]
 * int32, device).  sims [N, 8] float64 from dpvba_pgo_sim3; poses [N, 7] and
 * inv_depth [P] float32, overwritten.                                      */
dpvba_status dpvba_pgo_apply(dpvba_ctx* ctx, int32_t n_frames, const double* sims, const int32_t* patch_off,
                             float* poses, float* inv_depth, void* stream);

/* Patch correlation of eq. 4 (Sec. 3.1, "Patch correlation"): for every
 * edge, at every patch pixel (u, v), the dot product of the patch feature
 * vector g(u, v) with the target frame's feature map sampled bilinearly at
 * the reprojected pixel shifted by each offset of a 7 x 7 grid centred at 0:
 *   corr[e, u, v, a, b] = < g_kk[e](u, v), f_jj[e](x + a - 3, y + b - 3) >,
 * (x, y) = coords[e, u, v] in feature-map pixels (pixel (x, y) holds
 * map[y, x]); bilinear weights from the point's distances to its four
 * pixels, pixels outside the map count as zero.  The reprojected patches
 * come from dpvba_reproject with patches and intrinsics given at the feature
 * map's resolution.
 *   gmap   [n_patches, p, p, dim] float32: patch features, row u, column v.
 *   fmaps  [n_maps, height, width, dim] float32: feature maps (channels last).
 *   kk, jj [n_edges] int32: patch and feature map of each edge (jj indexes
 *          fmaps, e.g. the slot of the target frame's stored map); an index
 *          out of range gives zeros for that edge and is recorded as an
 *          invalid input (later calls return DPVBA_EDEVICE).
 *   coords [n_edges, p, p, 2] float32 (x, y).
 *   corr   [n_edges, p, p, 7, 7] float32 (written).
 * dim a multiple of 64 up to 256; p odd, at most 15; EINVAL otherwise.
 * Accumulates in float32.  Needs no analysis.                             */
dpvba_status dpvba_patch_correlation(dpvba_ctx* ctx, int32_t n_edges, int32_t patch_size, int32_t dim,
                                     const float* gmap, int32_t n_patches, const float* fmaps, int32_t n_maps,
                                     int32_t height, int32_t width, const int32_t* kk, const int32_t* jj,
                                     const float* coords, float* corr, void* stream);

/* Proximity loop closure (Sec. 3.2, "Proximity Loop Closure" and
 * "Constructing the Patch Graph"): loops are detected from the cameras'
 * proximity to previously visited locations, and every stored patch of an
 * old frame gets a uni-directional edge to each recent frame found near it
 * (the destination frame is the one whose dense features the correlation of
 * eq. 4 needs).  The edges, appended to the temporal ones, form the graph of
 * the global BA that follows.
 * Rule: frame j is a loop target of frame i when j >= first_recent,
 * j - i > min_gap and the camera centres (translations of the poses) satisfy
 * |c_i - c_j|^2 < radius^2; frame i keeps its max_targets nearest targets,
 * ties to the lower frame index.  The comparisons are made in float32 with
 * d2 = (dx*dx + dy*dy) + dz*dz, every operation rounded on its own (no fused
 * multiply-add), against radius*radius rounded to float32.
 *   poses      [N, 7] float32 camera-to-world (read).
 *   patch_off  [N + 1] int32, non-decreasing, patch_off[0] = 0: the patches
 *              of frame i are [patch_off[i], patch_off[i+1]) (read).
 *   counts     [N] int32 (written): loop targets of each frame.
 *   targets    [N, max_targets] int32 (written): frame i's targets in
 *              increasing order, -1 after the last; may be NULL when
 *              max_targets = 0.
 *   edge_off   [N + 1] int64 (written): frame i's edges are
 *              [edge_off[i], edge_off[i+1]).
 *   ii, jj, kk [max_edges] int32 (written): source frame, target frame and
 *              patch of each edge, by frame, then patch, then target.
 *   n_edges    host: total loop edges.  The call synchronises `stream` to
 *              read it; if it exceeds max_edges, the first max_edges edges
 *              are written and DPVBA_ELIMIT is returned.
 * 0 <= first_recent <= N, min_gap >= 0, radius finite and >= 0,
 * 0 <= max_targets <= DPVBA_MAX_LOOP_TARGETS, max_edges >= 0; EINVAL
 * otherwise.  Needs no analysis.                                          */
#define DPVBA_MAX_LOOP_TARGETS 32
dpvba_status dpvba_proximity_edges(dpvba_ctx* ctx, const float* poses, int32_t n_frames, const int32_t* patch_off,
                                   int32_t first_recent, int32_t min_gap, float radius, int32_t max_targets,
                                   int32_t* counts, int32_t* targets, int64_t* edge_off, int32_t* ii, int32_t* jj,
                                   int32_t* kk, int64_t max_edges, int64_t* n_edges, void* stream);

/* Damped reduced camera system at the given iterate (eq. 3 linearised,
 * Appendix A): S = B~ - E C~^-1 E^T and s = -v + E C~^-1 w over the free
 * poses, n = 6 (N - n_fixed).
 *   S          [n, n] (float or double per opts->precision), written in
 *              full (both triangles), row-major.
 *   s          [n] same type, written.
 *   cost       one double (device) or NULL: 1/2 sum w r^2 at this iterate.
 * Needs dpvba_analyze on this graph.                                      */
dpvba_status dpvba_reduced_system(dpvba_ctx* ctx, const dpvba_graph* g, const float* poses,
                                  const float* inv_depth, const dpvba_opts* opts, void* S,
                                  void* s, double* cost, void* stream);

/* opts->n_iters Gauss-Newton iterations of eq. (3): per iteration assemble
 * the block-sparse normal equations, eliminate depths, factor and solve
 * the reduced system, back-substitute the depths, retract the free poses.
 *   poses      [N, 7] read and overwritten with the result (quaternions
 *              renormalised): float32, or float64 when opts->precision is
 *              DPVBA_FP64 (the pointer is then reinterpreted).
 *   inv_depth  [P] read and overwritten, same element type as poses.
 *   report     host memory or NULL; with NULL the final-iterate cost is
 *              not computed.
 * Needs dpvba_analyze on this graph.                                      */
dpvba_status dpvba_solve(dpvba_ctx* ctx, const dpvba_graph* g, float* poses, float* inv_depth,
                         const dpvba_opts* opts, dpvba_report* report, void* stream);

/* dpvba_solve for callers that cannot allocate device memory during the
 * call -- code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation: the same iteration and kernels as dpvba_solve on the
 * single-launch path, with the per-call buffers (tile partial systems,
 * stored Schur rows, tile-ordered depths and rays, ping-pong poses, the
 * packed reduced system, step, status words and report staging) taken from
 * a fixed static device array of 16 MiB instead of the context's workspace.
 * The array exists once per device for the life of the process and is
 * shared by every call on that device: each call overwrites what it uses
 * before reading it, so results never depend on an earlier call's contents,
 * but calls whose work overlaps on one device (other streams, other
 * contexts) race on it and must be serialised by the caller.  The context
 * still provides the analysis tables and its barrier and failure words.
 * Arguments, results and report as dpvba_solve; precision DPVBA_FP32 or
 * DPVBA_FP64 only (EINVAL for DPVBA_MIXED), n_iters >= 1 (EINVAL for 0).
 * DPVBA_ELIMIT when 6 (N - n_fixed) + 1 > 96 (the reduced system is not
 * the single-launch solver's) or when the buffers exceed the 16 MiB array
 * (dpvba_last_error gives the size).  Calls no allocator, host or device.
 * Needs dpvba_analyze on this graph.                                      */
dpvba_status dpvba_solve_noalloc(dpvba_ctx* ctx, const dpvba_graph* g, float* poses, float* inv_depth,
                                 const dpvba_opts* opts, dpvba_report* report, void* stream);

/* Launch mode of the kernels whose workgroups wait for each other: the
 * single-launch solver that dpvba_solve uses for small reduced systems
 * (6 x free poses + 1 <= 96; the sliding window of Sec. 3.1), whose
 * workgroups meet at grid-wide barriers, and the chained triangular solves
 * of larger systems, whose workgroups wait for the blocks before theirs.
 * Neither grid exceeds the workgroups the device holds at once.
 * cooperative = 0 (the default): ordinary launches, which rely on the device
 * placing every workgroup while the first ones wait -- true when the
 * device's other work finishes; every wait is bounded, so a violation is
 * reported (report status DPVBA_EHIP, later calls DPVBA_EDEVICE) rather
 * than hanging.  cooperative = 1: cooperative launches, whose co-residency
 * the runtime guarantees, at a higher cost per launch.  Results are
 * identical bit for bit.  EINVAL for other values.                        */
dpvba_status dpvba_set_cooperative(dpvba_ctx* ctx, int32_t cooperative);

/* Adjoint of dpvba_solve, for training through the BA layer (Sec. 2: the
 * network is supervised on the camera poses that bundle adjustment
 * produces; objective eq. 3).  Given the gradient of a loss with respect to
 * the poses and inverse depths that opts->n_iters iterations produce from
 * (poses0, inv_depth0), writes the gradient of that loss with respect to
 * every edge's target and weight.  The iterations are replayed from the
 * start, keeping the iterates; each iteration's Schur system is recomputed
 * at its iterate when walking back.  The derivative is that of the
 * iteration as computed: fixed iteration count, validity decided at each
 * iterate (an invalid edge contributes nothing), the damping's dependence
 * on Diag(H) included, and the Jacobians' dependence on the iterate
 * included (second derivatives of the projection).  An iteration whose
 * factorisation failed (its pose step was skipped) passes the gradient
 * through unchanged.
 *   poses0, inv_depth0  [N, 7], [P]: the starting point given to dpvba_solve
 *              (read only).
 *   grad_poses [N, 7] or NULL (zero): dL/d(final poses) in the stored
 *              (t, q) coordinates; components along q are projected out by
 *              the quaternion normalisation.
 *   grad_inv_depth [P] or NULL (zero): dL/d(final inverse depths).
 *   grad_target, grad_weight [E, 2] (written): dL/d target, dL/d weight.
 * All six arrays are float32, or float64 when opts->precision is DPVBA_FP64
 * (the pointers are then reinterpreted).  The workspace (about
 * (n_iters + 1) 7 N + n_iters (P + 6 N) + 15 E float64 elements for
 * n_iters = DPVBA_MAX_ITERS) is allocated by dpvba_analyze.
 * Needs dpvba_analyze on this graph.  EINVAL on bad arguments.             */
dpvba_status dpvba_solve_backward(dpvba_ctx* ctx, const dpvba_graph* g, const float* poses0,
                                  const float* inv_depth0, const dpvba_opts* opts,
                                  const float* grad_poses, const float* grad_inv_depth,
                                  float* grad_target, float* grad_weight, void* stream);

/* dpvba_solve and dpvba_solve_backward over n independent problems at once
 * (the batch of sliding windows whose adjoints the update operator's
 * training needs, Sec. 2): problem i runs on context ctxs[i], analysed for
 * graphs[i], with the i-th entry of every array (host arrays of n device
 * pointers; grad_poses / grad_inv_depth may be NULL, or hold NULL entries,
 * for zero; reports NULL or n host reports, complete once `stream` has
 * completed).  The problems run concurrently,
 * each on a stream of its own context, ordered after the work already on
 * `stream`; `stream` waits for all of them.  Launches whose workgroups
 * wait for each other are cooperative here (dpvba_set_cooperative(1) for
 * the duration of the call), so concurrent grids cannot starve them; the
 * single-launch solver of small problems is then slower than alone, so
 * dpvba_solve_many pays off for large problems, and the adjoint (whose
 * small problems need no such launch) for any.  The contexts must be
 * distinct and on one device.  Returns the first failure
 * (every problem is still enqueued and joined); EINVAL for a bad n or
 * context list.                                                           */
dpvba_status dpvba_solve_many(int32_t n, dpvba_ctx* const* ctxs, const dpvba_graph* graphs,
                              float* const* poses, float* const* inv_depth, const dpvba_opts* opts,
                              dpvba_report* reports, void* stream);
dpvba_status dpvba_solve_backward_many(int32_t n, dpvba_ctx* const* ctxs, const dpvba_graph* graphs,
                                       const float* const* poses0, const float* const* inv_depth0,
                                       const dpvba_opts* opts, const float* const* grad_poses,
                                       const float* const* grad_inv_depth, float* const* grad_target,
                                       float* const* grad_weight, void* stream);

/* A batch of independent problems packed back to back (many uneven
 * sliding windows, Sec. 3.1, solved together).  Host struct; the offset and
 * n_fixed arrays are host memory, the data arrays device memory.
 *   n_problems B >= 1.
 *   frame_off, patch_off, edge_off  [B + 1] prefix offsets: problem b owns
 *              poses [frame_off[b], frame_off[b+1]) of the packed [sum N, 7]
 *              pose array, inverse depths and patches
 *              [patch_off[b], patch_off[b+1]) and edges
 *              [edge_off[b], edge_off[b+1]).
 *   n_fixed    [B] held poses of each problem (its first n_fixed[b]).
 *   ii, jj, kk [sum E] indices LOCAL to the edge's problem.
 *   patches, target, weight, patch_size, fx..cy as in dpvba_graph (one
 *              camera for the whole batch).                               */
typedef struct {
  int32_t n_problems, patch_size;
  const int32_t* frame_off;
  const int32_t* patch_off;
  const int32_t* edge_off;
  const int32_t* n_fixed;
  const float* patches;
  const int32_t* ii;
  const int32_t* jj;
  const int32_t* kk;
  const float* target;
  const float* weight;
  float fx, fy, cx, cy;
} dpvba_batch;

/* Symbolic analysis of a batch (replaces any previous batch analysis; the
 * single-problem analysis is kept).  tile_patches: host [B] patches per
 * tile for each problem in float32 and mixed modes (<= 0: default), e.g.
 * from an autotuner, or NULL; float64 uses the default.  The same checks as
 * dpvba_analyze, per problem, plus: offsets non-decreasing with at least one
 * frame per problem, and at most 42 free poses per problem (EINVAL).      */
dpvba_status dpvba_analyze_batch(dpvba_ctx* ctx, const dpvba_batch* b, const int32_t* tile_patches,
                                 void* stream);

/* Flag of dpvba_opts for dpvba_solve_batch: record the call's launches in a
 * HIP graph on first use and replay that graph on later calls with the same
 * arguments (pointers, options and stream); any change re-records.  The
 * report, if requested, is produced outside the graph.  Needs a stream other
 * than the null stream (EINVAL otherwise); ignored while tracing.        */
#define DPVBA_FLAG_GRAPH 1u

/* opts->n_iters iterations of every problem of the analysed batch: the
 * tiles of all problems are assembled by one launch per iteration, then one
 * workgroup per problem gathers, factors and solves its reduced system and
 * retracts its poses (see dpvba_solve for the iteration).
 *   poses      [sum N, 7], inv_depth [sum P]: read and overwritten; float32
 *              (DPVBA_FP32, DPVBA_MIXED) or float64 (DPVBA_FP64).
 *   reports    host [B] or NULL: one report per problem.
 *   opts->flags  0 or DPVBA_FLAG_GRAPH.
 * Needs dpvba_analyze_batch on this batch (same index arrays).            */
dpvba_status dpvba_solve_batch(dpvba_ctx* ctx, const dpvba_batch* b, float* poses, float* inv_depth,
                               const dpvba_opts* opts, dpvba_report* reports, void* stream);

/* Phase timing with HIP events (tracing).  While tracing is on, the
 * numeric calls record an event pair on their stream around every
 * `sample_every`-th launch of each phase (sample_every >= 1); the pairs are
 * resolved by dpvba_trace_end.  Phases: tile assembly of the reduced system;
 * its gather into the dense damped matrix; the Cholesky factorisation and
 * triangular solves; depth back-substitution; pose retraction; final cost.
 * dpvba_trace_begin creates the events (it may allocate host and driver
 * resources); it returns EINVAL for sample_every < 1 or max_pairs < 1.   */
typedef enum {
  DPVBA_PHASE_ASSEMBLE = 0,
  DPVBA_PHASE_GATHER = 1,
  DPVBA_PHASE_FACTOR = 2,
  DPVBA_PHASE_BACKSUB = 3,
  DPVBA_PHASE_RETRACT = 4,
  DPVBA_PHASE_COST = 5,
  DPVBA_N_PHASES = 6
} dpvba_phase;

dpvba_status dpvba_trace_begin(dpvba_ctx* ctx, int32_t sample_every, int32_t max_pairs);

/* Stop tracing: waits for the recorded events and writes, per phase, the
 * summed duration of the sampled launches in milliseconds, the number of
 * sampled launches and the number of launches seen (host arrays of
 * DPVBA_N_PHASES entries; any may be NULL).                               */
dpvba_status dpvba_trace_end(dpvba_ctx* ctx, double* ms, int32_t* n_sampled, int64_t* n_launched);

/* Device-side failures of the calls enqueued so far on this context.
 * Kernels that detect a failure -- a bounded device-wide wait that expired
 * (the co-residency that a grid barrier or a chained solve needs was not
 * met), or a non-finite target / weight or a negative weight -- record it
 * in a host-visible word of the context.  Every later call on the context
 * checks that word first and, once such a failure has been recorded,
 * returns DPVBA_EDEVICE without enqueuing anything (results of the failed
 * call and of calls enqueued after it are invalid).  This call
 * synchronises `stream`, returns DPVBA_EDEVICE if a failure was recorded
 * (DPVBA_OK otherwise), and clears the record, re-arming the context's
 * device-wide barriers; *cause (host, may be NULL) receives the failure
 * bits: 1 expired grid barrier, 2 expired chained triangular solve,
 * 4 invalid target or weight.                                             */
dpvba_status dpvba_device_status(dpvba_ctx* ctx, void* stream, int32_t* cause);

/* Text of the last HIP failure seen by a call on this context (the failing
 * call and HIP's message), "" if none.  Owned by the context.             */
const char* dpvba_last_error(const dpvba_ctx* ctx);

/* Static text for a status code. */
const char* dpvba_status_string(dpvba_status s);

#ifdef __cplusplus
}
#endif

#endif /* DPVBA_H */
