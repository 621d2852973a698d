/*
 * traj.h -- C-ABI of the MI355X (gfx950) batched non-holonomic trajectory optimizer.
 *
 * Method: Adajania et al., "Multi-Modal Model Predictive Control through Batch
 * Non-Holonomic Trajectory Optimization" (arXiv 2109.10392). Many goal-directed
 * instances of the problem of eq. (1a-e) are solved at once by the alternating
 * minimisation of Algorithm 1 (Sec. III-D) on the multi-convex reformulation of
 * eqs. (8a-c), then ranked by the meta-costs of Sec. III-F.
 *
 * Conventions for every entry point
 *   - Return value: TRAJ_OK (0) or a negative TRAJ_E_* code; traj_last_error()
 *     then returns a message for the calling thread. No C++ exception crosses
 *     this boundary.
 *   - "device" pointers are HIP device memory owned by the caller (for example
 *     PyTorch tensors); "host" pointers are ordinary host memory read during
 *     the call only. The handle owns only its operator tables.
 *   - stream is a hipStream_t (NULL = the null stream). Solve and score enqueue
 *     kernels on it and return without synchronising; they do not allocate and
 *     do not read device memory on the host.
 *   - A handle must not be used from two host threads at once.
 *   - Layouts: goal index fastest. c and lam are [3][11][n_goals] float
 *     (axis 0 = x, 1 = y, 2 = heading psi; then the 11 Bernstein coefficients).
 */
#ifndef TRAJ_H
#define TRAJ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TRAJ_OK 0
#define TRAJ_E_INVAL (-1) /* bad argument: null pointer, size, non-finite parameter, ... */
#define TRAJ_E_SHAPE (-2) /* shape index out of range / not set up                    */
#define TRAJ_E_HIP (-3)   /* HIP runtime error (message in traj_last_error)             */
#define TRAJ_E_NOMEM (-4) /* device allocation failed (setup only)                      */

/* traj_solve_batch flags */
#define TRAJ_INIT_COLD 0x0u       /* cold start (boundary-only minimum-acceleration QP)      */
#define TRAJ_INIT_FROM_STATE 0x1u /* start from (c, lam) in the state (resume, warm start)   */
#define TRAJ_WARM_FALLBACK 0x2u   /* with FROM_STATE, group kernel: the first iteration also
                                     runs from the cold start; each goal keeps whichever has
                                     the lower max(r_obs, r_acc, r_nh) after it (a NaN
                                     component makes the given state's residual lose)    */
#define TRAJ_KEEP_DONE 0x4u       /* traj_converge only: scene_done and scene_iters are kept, not
                                     reset; scenes already done are left untouched and the
                                     others start as the other flags say                      */
#define TRAJ_PREC_FP32 0x0u       /* FP32 arithmetic, x/y step operators in FP64 (default)   */
#define TRAJ_PREC_BF16X3 0x10u    /* matrix-core kernel: every contraction in split BF16 (hi
                                     + lo, three products), every inverse x right-hand side
                                     in a three-part split (six products), FP32 accumulation */
#define TRAJ_KERNEL_AUTO 0x0u     /* kernel from the handle's tile setting (traj_set_tile)   */
#define TRAJ_KERNEL_WAVE 0x100u   /* one wavefront per goal, lanes over time                 */
#define TRAJ_KERNEL_MFMA 0x200u   /* matrix-core kernel: goal groups x 16-sample time tiles  */
#define TRAJ_KERNEL_GROUP 0x400u  /* matrix-core kernel, one wavefront per goal group sweeping
                                     its time tiles; cost-sorted work list (needs state.work) */

#define TRAJ_N_COEF 11 /* Bernstein degree 10: coefficients per axis */

/* Solver constants shared by every instance of the batch (the Note after eq. 1
 * and Remark 1: bounds and obstacles are common to all goals). */
typedef struct {
  int32_t n_coef; /* must be TRAJ_N_COEF */
  float rho;      /* penalty weight rho_xy of eq. 10, also used for the heading block (eq. 13) */
  float a, b;     /* obstacle ellipse semi-axes incl. ego inflation (eq. 1e); > 0 */
  float v_min, v_max; /* velocity bounds (eq. 1d); 0 < v_min <= v_max (eq. 21 needs v_min > 0) */
  float a_max;        /* acceleration bound (eq. 1d, eq. 5); >= 2^-63 (about 1.1e-19), so
                         that a_max^2 is a normal FP32 number */
  float psi_max;      /* heading post-filter bound in radians (Sec. III, assumption 2) */
} traj_params;

/* One horizon/obstacle-count combination. The operator tables depend on both:
 * F_o stacks P once per obstacle (eq. 7 and the text after it), so F^T F and
 * the KKT inverses of eqs. 17/19 change with m. */
typedef struct {
  int32_t n_time; /* samples of the horizon, 11 <= n_time <= 192, t_i = i t_f/(n_time-1) */
  float t_f;      /* horizon length in seconds, > 0 */
  int32_t n_obs;  /* obstacles m of every scene using this shape, 0 <= m <= 64 */
} traj_shape;

/* A batch of scenes. Scene s owns goals [goal_off[s], goal_off[s+1]) and
 * obstacles [obs_off[s], obs_off[s+1]); obs_off[s+1]-obs_off[s] must equal the
 * n_obs of shape shape_id[s]. All arrays are device memory. */
typedef struct {
  int32_t n_scenes;
  int32_t n_goals;         /* == goal_off[n_scenes] */
  const int32_t *goal_off; /* device [n_scenes+1], non-decreasing, goal_off[0] = 0 */
  const int32_t *obs_off;  /* device [n_scenes+1] */
  const int32_t *shape_id; /* device [n_scenes], index into the shapes given to traj_setup */
  const float *ego;  /* device [n_scenes][8]: x0, y0, vx0, vy0, ax0, ay0, psi0, psidot0 */
  const float *obs;  /* device [n_obs_total][4]: x, y, vx, vy at t = 0 (constant velocity, Sec. III assumption 3) */
  const float *goal; /* device [n_goals][2]: x_f, y_f; final lateral velocity/acceleration and heading are 0 */
} traj_batch;

/* Iterate of every goal. With TRAJ_INIT_FROM_STATE, c and lam are read as the
 * starting point; on return they hold the last iterate. */
typedef struct {
  float *c;       /* device [3][11][n_goals] */
  float *lam;     /* device [3][11][n_goals] */
  float *resid;   /* device [4][n_goals]: r_obs, r_acc, r_nh, r_psi after the last iteration (may be NULL) */
  int32_t *iters; /* device [n_goals]: iterations performed (may be NULL) */
  int32_t *work;  /* device scratch of work_ints int32 for TRAJ_KERNEL_GROUP (the work list and
                     its claim counter; contents are overwritten by every solve), else may be NULL */
  int64_t work_ints;
  int32_t *scene_done; /* device [n_scenes] or NULL. Solve leaves every scene with a non-zero
                          entry untouched (its goals are not iterated and nothing of theirs is
                          written); traj_converge sets it to 1 for the converged scenes. */
} traj_state;

/* Meta-cost of Sec. III-F. */
typedef struct {
  int32_t kind;       /* 0: cruise, eq. 25; 1: high speed near the right lane, eq. 26 */
  const float *v_ref; /* device [n_scenes]: v_cruise (kind 0) or v_max (kind 1) */
  float w1, w2;       /* weights of eq. 26 (ignored for kind 0) */
  const float *y_rl;  /* device [n_scenes]: lateral position of the right lane (kind 1; may be NULL for kind 0) */
  float clear_min;    /* collision post-check, 0 = off: a goal whose trajectory comes closer than
                         clear_min to an obstacle, in the scaled distance sqrt((dx/a)^2 + (dy/b)^2)
                         of eq. 1e against the constant-velocity predictions, is discarded (cost
                         +inf); 1 discards every trajectory that enters an obstacle ellipse */
} traj_metacost;

/*
 * traj_setup -- build the constant operators of every shape (Remark 1; eqs. 17-20:
 * the left-hand sides do not depend on the batch index, so one inverse serves
 * every goal). Bernstein basis, Gram matrices and the KKT matrices of the x, y,
 * heading and cold-start systems are formed and inverted in FP64 on the GPU;
 * FP32 tables are derived from them. Allocates the handle's device memory (the
 * only allocation of the library) and synchronises the stream before returning.
 *   params: host, copied. shapes: host [n_shapes], copied; 1 <= n_shapes <= 4096.
 *   handle_out: host, receives the handle.
 * Errors: TRAJ_E_INVAL for bad parameters or shapes, TRAJ_E_NOMEM, TRAJ_E_HIP.
 */
int traj_setup(const traj_params *params, const traj_shape *shapes, int n_shapes, void *stream,
               void **handle_out);

/*
 * traj_solve_batch -- run `iters` iterations of Algorithm 1 on every goal of the
 * batch: x/y QP with the shared inverse (eq. 12 via eq. 18), heading QP with the
 * convex surrogate (eq. 13 via eq. 20), velocity (eq. 21), obstacle polar
 * variables (eq. 22 and the clipped 1-D minimiser of eq. 15), acceleration polar
 * variables (eq. 16), multipliers (eqs. 23-24).
 *   flags: TRAJ_INIT_COLD or TRAJ_INIT_FROM_STATE, | TRAJ_PREC_FP32 or
 *          TRAJ_PREC_BF16X3, | TRAJ_KERNEL_AUTO, TRAJ_KERNEL_WAVE,
 *          TRAJ_KERNEL_MFMA or TRAJ_KERNEL_GROUP (BF16X3 runs on a matrix-core
 *          kernel: the group kernel if asked for, else the MFMA kernel). The
 *          MFMA kernel holds the obstacle predictions of a whole horizon in LDS:
 *          n_tiles (144 n_obs + 4096) bytes (n_tiles = ceil(n_time / 16), from
 *          the handle's longest horizon and largest obstacle count) must stay
 *          within 150 KiB, e.g. n_time <= 176 with 64 obstacles; larger handles
 *          get TRAJ_E_INVAL for it (the wave and group kernels take every shape
 *          traj_setup accepts).
 *   tol: <= 0 runs exactly `iters` iterations; > 0 stops at the first multiple
 *        of 5 iterations where max(r_obs, r_acc, r_nh) <= tol: per goal in the
 *        wave kernel, per goal group (all of its goals) in the matrix-core kernels.
 *   The group kernel needs state->work with at least traj_work_ints(...) entries
 *   (TRAJ_E_INVAL otherwise). Two solves that share a work buffer must not run
 *   concurrently.
 *   iters: 0 <= iters <= 100000. n_goals == 0 is a no-op.
 * Shape mismatches found on the device (unknown shape id, wrong obstacle count,
 * an obstacle range starting before the array) set that scene's residuals to
 * NaN and its obstacles are not read; nothing aborts. Input values that are not
 * finite are found on the device too: a scene whose ego state or any obstacle
 * state is not finite has every goal marked, a goal whose target is not finite
 * is marked alone. A marked goal's c, lam and residuals become NaN and its
 * iteration count 0 (traj_score gives it a NaN cost and never picks it); the
 * other goals are solved as if the marked ones were absent.
 * Errors: TRAJ_E_INVAL (null pointers, negative sizes), TRAJ_E_HIP.
 */
int traj_solve_batch(void *handle, const traj_batch *batch, traj_state *state, int iters, float tol,
                     uint32_t flags, void *stream);

/*
 * traj_solve_batch_noalloc -- traj_solve_batch for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses that
 * forbid allocation): a group-kernel solve takes its work list from a scratch
 * array that the library holds in device memory (one per GPU, reserved when the
 * library is loaded, kept until the process ends) instead of state->work, which
 * is ignored. Everything else (arguments, flags, results, errors) is as
 * traj_solve_batch; the wave and MFMA kernels use no scratch. The call makes no
 * allocation of any kind.
 *   Limit: the work list (traj_work_ints for the batch and the handle's group
 *   size) must fit in TRAJ_NOALLOC_WORK_INTS int32 (2 MiB), e.g. 118,830 goals
 *   in 512 scenes at every group size; larger batches get TRAJ_E_INVAL.
 *   The current device must be the one the handle was set up on (TRAJ_E_INVAL).
 *   Every call on a GPU shares that GPU's scratch: two calls whose work overlaps
 *   on one GPU (other streams, other threads, other handles) race and give wrong
 *   results. Each call rebuilds the list before reading it, so nothing carries
 *   over from the previous call.
 */
#define TRAJ_NOALLOC_WORK_INTS 524288
int traj_solve_batch_noalloc(void *handle, const traj_batch *batch, traj_state *state, int iters, float tol,
                             uint32_t flags, void *stream);

/*
 * traj_score -- meta-cost per goal (eq. 25 or 26, v(t) = |(x'(t), y'(t))| of the
 * final coefficients) with the heading post-filter (cost = +inf when
 * max_t |psi(t)| > psi_max, Sec. III assumption 2) and, if mc->clear_min > 0,
 * the collision post-check (cost = +inf when the trajectory comes closer than
 * clear_min to an obstacle), then per scene the lowest index attaining the
 * minimum finite cost.
 *   cost: device [n_goals]. best: device [n_scenes], index within the scene, -1
 *   if every goal of the scene is filtered.
 * Errors: TRAJ_E_INVAL, TRAJ_E_HIP.
 */
int traj_score(void *handle, const traj_batch *batch, const traj_state *state, const traj_metacost *mc,
               float *cost, int32_t *best, void *stream);

/*
 * traj_converge -- iterate until the stopping rule of Sec. IV (residuals of the
 * order 1e-3 for the trajectory that is executed): chunks of `chunk` iterations,
 * each followed by the scoring of traj_score; a scene is done once its current
 * best goal has max(r_obs, r_acc, r_nh) <= tol, and later chunks neither iterate
 * nor re-score it (its state, costs and best goal stay as they were). At most max_iters
 * iterations per scene. Everything is enqueued on the stream without host
 * synchronisation (graph-capturable); the loop length is fixed by max_iters and
 * chunk, so finished scenes cost only the skipped launches.
 *   flags: as traj_solve_batch for the first chunk (cold, warm, warm with
 *          TRAJ_WARM_FALLBACK; precision; kernel); later chunks resume the state.
 *          With TRAJ_KEEP_DONE the call continues an earlier one: scene_done and
 *          scene_iters are not reset, the scenes marked done are neither solved
 *          nor re-scored, the others start as the flags say (for example a cold
 *          restart of the scenes a warm start left unconverged) and scene_iters
 *          adds this call's iterations to what it held.
 *   state: c, lam, resid and scene_done are required (scene_done is reset first,
 *          unless TRAJ_KEEP_DONE, and holds 1 for converged scenes on return).
 *   cost, best: as traj_score (the ranking after the last chunk).
 *   scene_iters: device [n_scenes]: iterations the scene ran (a multiple of chunk,
 *          or max_iters).
 * Errors: TRAJ_E_INVAL (NULL arrays, tol <= 0, bad sizes), TRAJ_E_HIP.
 */
int traj_converge(void *handle, const traj_batch *batch, traj_state *state, const traj_metacost *mc,
                  int max_iters, int chunk, float tol, uint32_t flags, float *cost, int32_t *best,
                  int32_t *scene_iters, void *stream);

/*
 * traj_controls -- controls along the chosen trajectory of every scene (the
 * goal index best[s] from traj_score) and its clearance from the obstacles:
 * acceleration v' = (x' x'' + y' y'') / v and steering atan(psi' h / max(v, v_min))
 * (the relation the paper gives for extracting the steering input, Sec. III),
 * h = wheelbase; clearance = smallest sqrt((dx/a)^2 + (dy/b)^2) over samples and
 * obstacles with the constant-velocity predictions (< 1: the trajectory enters
 * an obstacle ellipse of eq. 1e).
 *   accel, steer: device [n_scenes][stride], samples 0 .. n_time - 1 of the scene;
 *   stride >= the longest n_time of the handle. clearance: device [n_scenes]
 *   (+inf without obstacles; NaN where best < 0 or the shape is unknown).
 * Errors: TRAJ_E_INVAL, TRAJ_E_HIP.
 */
int traj_controls(void *handle, const traj_batch *batch, const traj_state *state, const int32_t *best,
                  float wheelbase, int stride, float *accel, float *steer, float *clearance, void *stream);

/* Kernel tile of a handle. kernel: TRAJ_KERNEL_WAVE, TRAJ_KERNEL_MFMA or
 * TRAJ_KERNEL_GROUP; group: goals per matrix-core goal group, 1..16 (the MFMA
 * has 16 goal columns; fewer goals per group spread a small batch over more
 * compute units); persistent (group kernel): 1 = a device-filling grid whose
 * wavefronts claim goal groups from the work list until it is exhausted, 0 = one
 * wavefront per listed group; waves (wave kernel): wavefronts per goal, 1 or 2 (two
 * halve each wave's time samples and add their partial sums through LDS, for
 * batches too small to fill the device with one wave per goal). */
typedef struct {
  int32_t kernel;
  int32_t group;
  int32_t persistent;
  int32_t waves;
} traj_tile;

/*
 * traj_set_tile / traj_get_tile -- the tile used when traj_solve_batch is called
 * with TRAJ_KERNEL_AUTO (the default). Chosen by the autotuner for a workload;
 * the initial setting is {TRAJ_KERNEL_WAVE, 16}. Host-only, no device work.
 * Errors: TRAJ_E_INVAL (unknown kernel, group outside 1..16, persistent not 0/1,
 * waves not 1/2).
 */
int traj_set_tile(void *handle, const traj_tile *tile);
int traj_get_tile(void *handle, traj_tile *tile);

/*
 * traj_work_ints -- entries of the int32 device scratch (traj_state.work) that a
 * group-kernel solve of a batch with n_scenes scenes and n_goals goals needs with
 * the handle's current group sizes: 4 + 2 (ceil(n_goals / group) + n_scenes) +
 * n_goals + n_scenes with group the smallest goals-per-group of any shape (the
 * tile's where a shape sets none; claim counter, the cost-sorted list of goal
 * groups, the goal order of every scene, the goals of each scene that are
 * solved). The wave and MFMA kernels do not use the scratch. Host-only.
 * Errors: TRAJ_E_INVAL (NULL handle or out, negative sizes).
 */
int traj_work_ints(void *handle, int n_scenes, int n_goals, int64_t *out);

/*
 * traj_set_shape_groups / traj_get_shape_groups -- goals per group of the group
 * kernel (TRAJ_KERNEL_GROUP) for the scenes of each shape, as a per-(T, m)
 * autotuner chooses them; the other kernels ignore it. The operation is that of
 * traj_solve_batch (Algorithm 1 per goal, Sec. III-D): the sizes change only how
 * goals are packed onto wavefronts, never a result.
 *   groups: host, one int32 per shape of the handle (setup order): 0 = the tile's
 *           group size (the initial setting), 1..16 = that many goals per group;
 *           NULL sets every shape to 0. get writes the same layout.
 * set copies the shape table to the device with a synchronous copy: no solve on
 * this handle may be running (synchronise its streams first). Raising the
 * smallest group size never invalidates a work buffer sized before; lowering it
 * can (traj_work_ints).
 * The current device must be the one the handle was set up on.
 * Errors: TRAJ_E_INVAL (NULL handle or out, a size outside 0..16, another
 * current device; nothing is changed), TRAJ_E_HIP.
 */
int traj_set_shape_groups(void *handle, const int32_t *groups);
int traj_get_shape_groups(void *handle, int32_t *groups);

/* traj_destroy -- free the handle's device memory. NULL is a no-op. */
int traj_destroy(void *handle);

/* traj_last_error -- message of the last failing call on this thread ("" if none). */
const char *traj_last_error(void);

/*
 * traj_debug_operators -- copy one shape's operator tables to host memory for
 * verification against an independent reference. Synchronises the stream.
 *   out_f64: host, 5 * 17 * 17 doubles: the inverses of the x, y, heading,
 *            cold-start x and cold-start y KKT matrices (eqs. 17 and 19 split
 *            per axis), each stored row-major in a 17x17 block (top-left used).
 *   out_f32: host, traj_debug_table_size(handle, shape) floats (see the layout
 *            note in the implementation). Either pointer may be NULL.
 */
int traj_debug_operators(void *handle, int shape, double *out_f64, float *out_f32, void *stream);
int traj_debug_table_size(void *handle, int shape);

/*
 * traj_debug_reduce -- lane-layout check of the cross-lane reductions the solver
 * uses for its contractions over time. in: device [r][64] floats (value i of
 * lane l at in[i*64 + l]); out: device [64]. r = 32: out[l] = sum over lanes of
 * value l/2; r = 16: out[l] = sum over lanes of value l/4. Asynchronous.
 */
int traj_debug_reduce(const float *in, float *out, int r, void *stream);

/*
 * traj_debug_atan2 -- the solver's atan2 (heading angle theta = atan2(y', x') of
 * eq. 13) applied element-wise, for checking it against a reference:
 * out[i] = atan2(y[i], x[i]). Device arrays of n floats. Asynchronous.
 */
int traj_debug_atan2(const float *y, const float *x, float *out, int n, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* TRAJ_H */
