/*
 * flash.h - C ABI of the MI355X FLASH step library.
 *
 * One call of flash_step advances every environment of a batch by one implicit
 * Euler step of projective-dynamics elasticity with Signorini-Coulomb contact,
 * solved as a non-smooth complementarity problem (FLASH, Sec. III: implicit
 * step Eq. 1, contact-constrained dynamics Eq. 2, projective internal forces
 * Eq. 3, assembled system A q - b - h^2 H^T lambda = 0 of Eq. 4, non-smooth
 * Newton quantities Eq. 5-9; the multi-environment pipeline is Alg. 1 with the
 * block-diagonal batch of Eq. 11-12).  Environments never couple: each keeps
 * its own A = M + h^2 sum_i w_i G_i^T G_i, contact set and multipliers.
 *
 * Conventions
 *  - Every function returns flash_status; no C++ exception crosses the ABI.
 *    flash_last_error() returns a thread-local description of the last error.
 *  - SI units.  Host arrays are xyz-interleaved doubles; device state is
 *    structure-of-arrays in the batch's working precision.
 *  - Ownership: the caller owns every array it passes; inputs are copied
 *    during the call; outputs are caller-allocated with an explicit capacity.
 *    The batch owns all device memory (allocated in flash_create_batch, freed
 *    in flash_destroy_batch).
 *  - An invalid argument returns FLASH_ERR_INVALID_ARG and leaves the batch
 *    unchanged.
 *  - flash_step only enqueues work on the batch's stream; the query calls
 *    (get_state, contacts, residual, stats) synchronise that stream first.
 *  - Determinism: identical inputs and parameters give bitwise identical
 *    results run to run (no floating-point atomics; fixed reduction orders;
 *    ordered contact compaction).
 *  - Threading: one batch per host thread or stream; no global state besides
 *    the thread-local error text.
 */
#ifndef FLASH_MI355X_H
#define FLASH_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct flash_batch flash_batch;   /* opaque; library-owned until destroy */

typedef enum {
  FLASH_OK = 0,
  FLASH_ERR_INVALID_ARG = 1,
  FLASH_ERR_OUT_OF_MEMORY = 2,
  FLASH_ERR_DEVICE = 3,
  FLASH_ERR_CAPACITY = 4,
  FLASH_ERR_NOT_CONVERGED = 5,
  FLASH_ERR_NONFINITE = 6,
  FLASH_ERR_UNSUPPORTED = 7
} flash_status;

enum { FLASH_TET = 0, FLASH_TRI = 1 };
enum { FLASH_PLANE = 0, FLASH_BOX = 1, FLASH_CAPSULE = 2 };
enum { FLASH_FP32 = 0, FLASH_FP64 = 1 };
enum { FLASH_WS_ZERO = 0, FLASH_WS_PREV = 1, FLASH_WS_LEARNED = 2 };
enum { FLASH_MAX_OBSTACLES = 4, FLASH_MAX_GRIPPERS = 2 };

/* One environment: one deformable body.
 * Element maps and weights follow the as-rigid-as-possible reading of Eq. 3:
 * tets project F = D_s D_m^-1 onto SO(3) with w = 2 mu_L V; triangles project
 * the 3x2 F onto matrices with orthonormal columns with w = 2 mu_L A t;
 * mu_L = young / (2 (1 + poisson)).  Masses are lumped by row sums.
 * rest_x [n_vertices*3] and elements [n_elements*4 (tets) | *3 (tris)] are
 * copied.  Tets with negative rest orientation are reordered internally. */
typedef struct {
  int32_t elem;              /* FLASH_TET or FLASH_TRI */
  int32_t n_vertices;
  int32_t n_elements;
  int32_t reserved;
  const double *rest_x;
  const int32_t *elements;
  double density;            /* kg/m^3 */
  double thickness;          /* m, FLASH_TRI only */
  double young;              /* Pa */
  double poisson;
  double bending;            /* FLASH_TRI only: hinge stiffness (0 = none) */
  double mu;                 /* Coulomb coefficient against every obstacle of this env */
} flash_env_desc;

/* Kinematic obstacle (rigid, translating).  Pose at the start of the next step.
 * PLANE: normal = rot * (0,1,0), through center.  BOX: half extents size[0..2].
 * CAPSULE: size = {radius, half_length, 0}, axis = rot * (1,0,0).
 * rot is a row-major 3x3 world-from-local rotation.  The obstacle translates by
 * h * lin_vel during each of the next move_steps steps (negative: forever) and
 * then holds its pose. */
typedef struct {
  int32_t kind;
  int32_t move_steps;
  double center[3];
  double rot[9];
  double size[3];
  double lin_vel[3];
} flash_obstacle;

/* Kinematic gripper for bilateral attachment (supplementary, bilateral constraint
 * for cloth control: x_i - p_grip(t) = 0 for the grasped vertices, which join the
 * set when the gripper is activated within a proximity threshold and leave it on
 * release).  center: pose at the start of the next step; it translates by
 * h * lin_vel during each of the next move_steps steps (negative: forever), then
 * holds.  While grasp != 0 and the gripper holds no vertex, a step's detection
 * attaches every vertex within `radius` of the center (FP64 squared distance,
 * <= r^2) that no other gripper holds, lower gripper index first, and keeps its
 * offset o = x - center; each held vertex then carries three equality rows
 * q_i = center(t+h) + o (always active, no friction cone, unbounded multipliers)
 * in the same contact solve, and no obstacle rows (its position is prescribed).
 * grasp = 0 releases the set. */
typedef struct {
  double center[3];
  double lin_vel[3];
  double radius;                  /* capture threshold, m */
  int32_t move_steps;
  int32_t grasp;                  /* 1: grasp (capture when holding nothing), 0: release */
} flash_gripper;

typedef struct {
  double h;                       /* time step, s */
  double gravity[3];              /* m/s^2 */
  int32_t lg_iterations;          /* K: local-global iterations per step (Alg. 1 k_max) */
  int32_t max_inner_iterations;   /* cap on non-smooth Newton iterations per contact solve */
  double ncp_tol;                 /* NCP residual tolerance, metres (default 1e-6) */
  double contact_margin;          /* delta_c, metres */
  double max_force;               /* |lambda| clamp, newtons */
  int32_t precision;              /* FLASH_FP32 or FLASH_FP64 */
  int32_t warm_start;             /* FLASH_WS_* */
  int32_t use_graph;              /* capture the step in a HIP graph */
  int32_t max_contacts_per_env;   /* contact capacity per env (0: default 320).  One
                                     workgroup holds an env's contact data in the 160 KB of
                                     LDS of a CU: at most 330 when the contact solve runs in
                                     FP64 (FP64 batches; FP32 batches unless contact_fp32),
                                     814 with contact_fp32 = 1; larger values return
                                     FLASH_ERR_INVALID_ARG from flash_create_batch, except with
                                     the lightweight metric, which then solves from global memory
                                     (global_contact_solve) up to 65536 */
  double inner_tol;               /* stopping tolerance of every contact solve, metres
                                     (0: 0.25 * ncp_tol in FP32, 1e-12 in FP64) */
  int32_t contact_fp32;           /* FP32 batches: 0 (default) runs the per-env contact-space
                                     solve in FP64, 1 in FP32 (stalls on stiff, high-friction
                                     contact sets); FP64 batches ignore it */
  int32_t fixed_schedule;         /* 0 (default): the first flash_step times the work schedules of the
                                     explicit-inverse products on this batch and keeps the fastest
                                     (see flash_schedule_info), and every step runs the per-env
                                     contact solves longest-first by the previous step's solve
                                     times (batches of up to 4096 envs); 1: default schedule, envs
                                     in index order.  Every schedule gives bitwise identical
                                     results. */
  int32_t stream_groups;          /* 0 or 1: one stream.  G >= 2: the envs are split into G
                                     contiguous groups, each stepped on a stream of its own so that
                                     one group's contact-solve tail overlaps the others' work
                                     (hip_stream must then be NULL).  Results are bitwise those of
                                     one group: envs never couple.  With the HIP runtime's default
                                     of 4 hardware queues per process, G = 2 or 3 pays off; at 4
                                     the groups share queues and throughput drops. */
  int32_t fused_lg;               /* 0 (default): every phase of the local-global loop is one batched
                                     launch (K x project, assemble, apply, contact solve, position
                                     update).  1: the whole loop is one launch with one workgroup per
                                     env, so that no env waits for the slowest env of the batch
                                     between phases; bitwise the same results.  Steps that record
                                     warm-start training pairs use the per-phase launches. */
  int32_t contact_metric;         /* FLASH_METRIC_EXACT (0, default): every contact subproblem is solved
                                     to inner_tol by semismooth Newton with the exact contact-space
                                     operator (the fully implicit metric Z of Eq. 7).
                                     FLASH_METRIC_LIGHTWEIGHT (1): the paper's fixed-budget mode (Alg. 1
                                     with the inertia-only metric Z~ = J M^-1 J^T + E of Eq. 10): each
                                     local-global iteration makes at most max_inner_iterations
                                     multiplier updates (K W~ + E) delta = -Phi with W~ = h^2 H M^-1 H^T,
                                     Phi at the exact positions, proximal scale h^2 / m_v, no line
                                     search, stopping early at inner_tol; the step then ends wherever
                                     that budget leaves it (flash_residual reports it, and
                                     FLASH_ERR_NOT_CONVERGED when above ncp_tol).  The learned
                                     prediction is not used in this mode. */
  int32_t global_contact_solve;   /* lightweight metric only.  0 (default): the contact update runs
                                     in LDS, one workgroup per env, while max_contacts_per_env fits
                                     one CU's LDS, and from global memory beyond that.  1: always from
                                     global memory: the contact displacement follows lambda through
                                     the position update of Alg. 1 (u = Gbar (b + h^2 H^T lambda)) at
                                     every update instead of through a contact-space operator, so
                                     no per-env storage grows with the square of the contact count
                                     and max_contacts_per_env may reach 65536.  Same iteration; the
                                     two routes round differently.  With the exact metric it must
                                     be 0. */
  int32_t twin_chunk;             /* global-memory lightweight route only: envs that share one
                                     explicit inverse (same mesh and material) run the inverse
                                     products in chunks of this many envs per workgroup, so that
                                     each inverse row read serves the whole chunk.  0 (default):
                                     automatic (8, else 4, while each product keeps at least 512
                                     workgroups, else 1); 1: one env per workgroup; 2..8: that many.
                                     Every choice gives the same bits. */
} flash_params;

enum { FLASH_METRIC_EXACT = 0, FLASH_METRIC_LIGHTWEIGHT = 1 };

/* One constraint row of the last step.  impulse = h F lambda in the world frame
 * (N s); lambda holds the contact-frame multipliers (n, t1, t2) in newtons.
 * mode: 0 separate (lambda = 0), 1 stick, 2 slip, 3 attachment (obstacle =
 * FLASH_MAX_OBSTACLES + gripper index; frame = world axes, gap = the x
 * component of x - target, lambda = world-frame force). */
typedef struct {
  int32_t env, vertex, obstacle, mode;
  double normal[3];
  double tangent1[3];
  double gap;                     /* d0, signed distance at the step start, m */
  double impulse[3];
  double lambda[3];
} flash_contact;

typedef struct {
  int32_t inner_iterations;       /* Newton iterations summed over the step's K contact solves */
  int32_t refactorizations;       /* inverse rebuilds of the contact-space operator */
  int32_t contacts;
  int32_t fp64_polar;             /* tets routed to the FP64 polar decomposition */
  int32_t flags;                  /* bit 0: non-finite state, bit 1: not converged, bit 2: contact
                                     capacity, bit 3: Newton system above its row capacity
                                     (contact capacity above 512) */
  int32_t ws_state;               /* learned warm start: bit 0 the step's first contact solve started
                                     from the network's prediction; bit 2 this step's solve from the
                                     prediction missed the tolerance and was restarted from the plain
                                     start; bits 8-15 count such restarts; bit 1 the prediction is
                                     disabled for this env after 3 of them (cleared by flash_set_state
                                     and flash_ws_load) */
  double residual;                /* NCP residual at the end of the step, m (FP64) */
} flash_env_stats;

/* Creates a batch of n_envs independent environments and runs the create-time
 * precompute (Alg. 1: assemble A per env and its exact inverse, in FP64 on the
 * host, one env at a time; masses, D_m^-1, weights).  Envs whose mesh, material
 * and h are equal share one inverse (host and device).  hip_stream: a
 * hipStream_t or NULL for a stream owned by the batch.  State starts at the rest
 * shapes with zero velocity and no obstacles.  With the environment variable
 * FLASH_PROGRESS set, envs of 20,000 vertices or more report the progress of
 * their factor and inverse on stderr (minutes on the host). */
flash_status flash_create_batch(const flash_env_desc *envs, int32_t n_envs, const flash_params *p,
                                void *hip_stream, flash_batch **out);
flash_status flash_destroy_batch(flash_batch *b);

/* Sets / reads the state of the implicit step: positions q_h and velocities v_h
 * at the start of the next step (Sec. III, Eq. 1, where q~ = q_h + h v_h +
 * h^2 M^-1 f_ext).  env = -1: all envs, concatenated in env order; else the one
 * env.  x, v: host arrays [n_vertices*3] of doubles, xyz-interleaved (v may be
 * NULL on set to keep velocities, NULL on get to skip); both calls synchronise
 * the batch's stream.  Setting the state of an env invalidates its warm-start
 * cache (previous-step multipliers and the learned-start fallback state).
 * Errors: FLASH_ERR_INVALID_ARG for a null batch or x (set), or env outside
 * [-1, n_envs). */
flash_status flash_set_state(flash_batch *b, int32_t env, const double *x, const double *v);
flash_status flash_get_state(flash_batch *b, int32_t env, double *x, double *v);

/* Zero-copy variants of flash_set_state / flash_get_state for device-resident
 * buffers such as PyTorch tensors (the same q_h, v_h of Eq. 1).  x_dev, v_dev
 * are device arrays in structure-of-arrays layout [3][n] (component-major: all
 * x coordinates, then all y, then all z), n = vertices of the env, or of the
 * whole batch in env order for env = -1; elem_size 4 = float, 8 = double
 * (converted to and from the batch's precision on the device: an FP64 batch
 * read into float rounds to nearest).  The calls only enqueue work on the
 * batch's stream (each group's stream for a batch with stream_groups >= 2) and
 * return: the caller must have finished writing x_dev / v_dev before that
 * work runs (for example by creating the batch on the stream that produces
 * them) and must keep the buffers alive and unmodified until it has finished
 * (flash_synchronize).  set: x_dev required, v_dev may be NULL to keep
 * velocities; invalidates the warm-start cache like flash_set_state.  get:
 * either output may be NULL, not both.  Errors: FLASH_ERR_INVALID_ARG for a
 * null batch, missing buffers, env outside [-1, n_envs) or another elem_size;
 * FLASH_ERR_DEVICE if a launch fails. */
flash_status flash_set_state_device(flash_batch *b, int32_t env, const void *x_dev, const void *v_dev,
                                    int32_t elem_size);
flash_status flash_get_state_device(flash_batch *b, int32_t env, void *x_dev, void *v_dev, int32_t elem_size);

/* Replaces the kinematic obstacles that define the contact constraints of one
 * env (env >= 0, n <= FLASH_MAX_OBSTACLES) or of every env (env = -1: o holds
 * n_envs * n entries, env-major): the bodies against which the Signorini-
 * Coulomb conditions of Eq. 2 are imposed (contact Jacobian H and multipliers
 * lambda).  Copied; takes effect at the next flash_step.  Errors:
 * FLASH_ERR_INVALID_ARG for a null batch, env outside [-1, n_envs), n outside
 * [0, FLASH_MAX_OBSTACLES], a null o with n > 0 or an unknown kind. */
flash_status flash_set_obstacles(flash_batch *b, int32_t env, const flash_obstacle *o, int32_t n);
flash_status flash_get_obstacles(flash_batch *b, int32_t env, flash_obstacle *o, int32_t capacity,
                                 int32_t *n_out);

/* Replaces the grippers of one env (env >= 0, n <= FLASH_MAX_GRIPPERS) or of
 * every env (env = -1: g holds n_envs * n entries, env-major), as move and
 * grasp commands for the next step (see flash_gripper).  Vertices already held
 * stay held while their gripper keeps grasping; grippers beyond n release.
 * Attachment rows count against max_contacts_per_env.  Copied; synchronises
 * the batch's stream.  Errors: FLASH_ERR_INVALID_ARG for a null batch, env
 * outside [-1, n_envs), n outside [0, FLASH_MAX_GRIPPERS], a null g with n > 0,
 * a negative radius or a non-finite center. */
flash_status flash_set_grippers(flash_batch *b, int32_t env, const flash_gripper *g, int32_t n);

/* Enqueues n_steps steps of every env (Alg. 1 loop body): contact detection at
 * the obstacles' end-of-step poses, prediction, K local-global iterations each
 * solving the contact subproblem to ncp_tol, finalisation.  Asynchronous. */
flash_status flash_step(flash_batch *b, int32_t n_steps);
flash_status flash_synchronize(flash_batch *b);

/* Contact set of the last step with its multipliers: one record per row block
 * of the contact Jacobian H (Eq. 2) with the multipliers lambda that solve the
 * complementarity problem of Eq. 2b at the end of the step, and the impulse
 * h F lambda.  Sorted by (vertex, obstacle) within an env; env = -1 lists every
 * env in env order.  out: caller array of `capacity` records (may be NULL with
 * capacity 0 to query the count).  Synchronises the batch's stream.  Errors:
 * FLASH_ERR_CAPACITY with *n_out = the required count if capacity is too
 * small; FLASH_ERR_INVALID_ARG for a null batch or n_out, or env outside
 * [-1, n_envs). */
flash_status flash_contacts(flash_batch *b, int32_t env, flash_contact *out, int32_t capacity,
                            int32_t *n_out);

/* Per-env NCP residual of the last step (metres, FP64), its maximum, and
 * Newton iteration counts.  The residual is that of the complementarity
 * function Phi of the contact subproblem (Eq. 2b with the non-smooth Newton
 * quantities of Eq. 5: min-map Signorini, Alart-Curnier Coulomb, scale
 * s = h^2 / m_v) evaluated from the end positions and multipliers, max over
 * contacts of max(|Phi_n|, |Phi_t|); the acceptance tolerance is ncp_tol (the
 * solver tolerance of the scene configuration).  per_env [n_envs], max_out and
 * inner_iters [n_envs] are host outputs, any may be NULL.  Synchronises.
 * Returns, in this order of precedence: FLASH_ERR_NONFINITE if an env holds a
 * non-finite state (its residual reads NaN); FLASH_ERR_CAPACITY if an env
 * detected more contacts than max_contacts_per_env (the step ignored the
 * excess, flag bit 2); FLASH_ERR_NOT_CONVERGED if an env ended above ncp_tol.
 * The outputs are filled in every case. */
flash_status flash_residual(flash_batch *b, double *per_env, double *max_out, int32_t *inner_iters);
flash_status flash_stats(flash_batch *b, flash_env_stats *per_env);

/* Statistics over all envs and steps since the previous reset: worst
 * end-of-step NCP residual (*max_out, metres), failed env-steps (*over_out:
 * ended above ncp_tol, or dropped contacts beyond the capacity), Newton
 * iterations summed over every contact solve
 * (*newton_out) and env-steps taken (*env_steps_out).  Any output may be
 * NULL; reset != 0 clears the statistics after reading. */
flash_status flash_residual_history(flash_batch *b, double *max_out, int64_t *over_out,
                                    int64_t *newton_out, int64_t *env_steps_out, int32_t reset);

/* Per-kernel timing with HIP events recorded on the batch's stream around each
 * launch of the kernel classes selected by `enable` (bit k = class k in the
 * order of flash_kernel_name; 0 = off, the default).  A graph-captured step
 * is replayed without events while timing is on.  flash_kernel_times fills up
 * to cap entries of total milliseconds and launch counts since the last
 * flash_set_kernel_timing call. */
flash_status flash_set_kernel_timing(flash_batch *b, int32_t enable);
flash_status flash_kernel_times(flash_batch *b, double *total_ms, int64_t *launches, int32_t cap,
                                int32_t *n_out);
const char *flash_kernel_name(int32_t i);

/* Work schedule of the explicit-inverse products (global apply and position
 * update; batching over uneven envs, Eq. 11-12).  One workgroup per (env,
 * column tile) work item, items of the largest envs first.  info[0] = columns
 * per tile, info[1] = rows in flight per wave, info[2] = work items, info[3] =
 * 1 if the autotuner chose it, info[4] = stream groups (info holds 5 values).
 * For a grouped batch the choice of group 0 is reported and the work items
 * are summed over the groups.  cand_ms (6 doubles, may be NULL): the
 * autotuner's milliseconds per apply launch for tiles of 8, 16 and 32 bytes
 * per lane, each with 4 and 8 rows in flight (0 when not tuned). */
flash_status flash_schedule_info(flash_batch *b, int32_t *info, double *cand_ms);

/* Diagnostic: ms_out[0..7] = wall-clock milliseconds per env spent in the 8
 * phases of the contact solve (setup, residual/classification, base inverse,
 * right-hand sides, capacitance build, capacitance LU, direction, line
 * search); ms_out[8..11] = per-env counts of capacitance factorisations,
 * factorisation reuses, line-search failures and solves ended above the
 * inner tolerance; ms_out[12] = mean rows of a factored capacitance system,
 * ms_out[13] = the largest, ms_out[14] = Newton iterations per env,
 * ms_out[15] = contact solves per env.  Accumulated since the previous call
 * (then reset).  ms_out holds 16 doubles. */
flash_status flash_phase_times(flash_batch *b, double *ms_out);

/* ---------------------------------------------------------------------------
 * Learned warm start (not part of the paper's method, whose contact solve
 * starts from the previous iterate).  A 16 -> 128 -> 128 -> 128 -> 3 ReLU MLP
 * maps features of each contact at the step start to a prediction of the
 * multipliers of the step's first contact solve.  Every GEMM of inference and
 * training rounds its operands to bfloat16 (nearest even) and accumulates in
 * FP32 on the matrix cores.  The prediction is used for the contacts that have
 * no previous-step multiplier (new contacts; every contact after a reset),
 * where the plain start is a Jacobi estimate of the normal multiplier.  The
 * plain start stays the fallback and the judge: the first contact solve of a
 * step starts from the prediction only if that lowers the merit 0.5 |Phi|^2 of
 * its start, a solve from a prediction that misses the tolerance within the
 * iteration cap is restarted from the plain start, and an env stops using the
 * prediction after three such restarts.  Every solve runs to the same
 * tolerance, so results agree with the plain method within that tolerance and
 * only iteration counts change.
 *
 * Parameters: W1[128x16] b1[128] W2[128x128] b2[128] W3[128x128] b3[128]
 * W4[3x128] b4[3], each W row-major (out x in): FLASH_MLP_PARAMS values.
 * Normalisation norm[FLASH_MLP_NORM]: 16 feature means, 16 feature inverse
 * scales, 3 label scales.  The network sees (f - mean) * inv_scale and
 * predicts label * label_scale.
 * Features per contact (delta_c = contact margin, s = h^2 / m_v):
 *   d0/delta_c; n.(h v + h^2 g)/delta_c; (h v - obstacle displacement) along
 *   n, t1, t2 over delta_c; s lambda_prev / delta_c (3, previous-step warm
 *   start in the new frame); had-previous flag; mu; log10(m_v Gbar_vv);
 *   log10(m_v / 1 g); contacts on the vertex (1 or 2 of the neighbours in the
 *   sorted list); (g.n) h^2/delta_c; (obstacle displacement . n)/delta_c; 1.
 * Label: s (lambda_1 - lambda_prev) / delta_c in the contact frame, where
 * lambda_1 solves the step's first contact subproblem (first local-global
 * iteration) and lambda_prev is the previous-step warm start in the features;
 * the candidate start is lambda_prev + output * delta_c / s on the cone.
 * ------------------------------------------------------------------------- */
enum { FLASH_MLP_FEATURES = 16, FLASH_MLP_HIDDEN = 128, FLASH_MLP_OUTPUTS = 3,
       FLASH_MLP_PARAMS = 35587, FLASH_MLP_NORM = 35 };

/* Loads bf16 weights (host, FLASH_MLP_PARAMS values) and norm (host,
 * FLASH_MLP_NORM floats) into the batch; they are used when the batch was
 * created with warm_start = FLASH_WS_LEARNED.  Clears every env's fallback
 * bit.  A captured step graph is re-captured at the next flash_step. */
flash_status flash_ws_load(flash_batch *b, const uint16_t *weights_bf16, size_t n_params,
                           const float *norm);

/* Use of the learned start over all envs and steps since the previous reset:
 * *started_out = env-steps whose first contact solve started from the
 * network's prediction, *restarted_out = env-steps whose solve from the
 * prediction missed the tolerance and was restarted from the plain start.
 * Either output may be NULL; reset != 0 clears the counts after reading.
 * Synchronises. */
flash_status flash_ws_history(flash_batch *b, int64_t *started_out, int64_t *restarted_out, int32_t reset);

/* ---- Batched depth rendering (supplementary: depth simulation: depth maps, instance
 * segmentation masks and point clouds ray-cast from the simulation state). */

/* Pinhole camera.  rot is the camera-to-world rotation, row-major, whose columns are the image's
 * right, down and optical-axis directions in world coordinates; fx, fy, cx, cy in pixels.  Pixel
 * (u, v) (column, row) casts the ray position + t rot ((u + 0.5 - cx) / fx, (v + 0.5 - cy) / fy, 1),
 * so the parameter t of a hit is its depth along the optical axis. */
typedef struct {
  double position[3];
  double rot[9];
  double fx, fy, cx, cy;
} flash_camera;

typedef struct flash_renderer flash_renderer;

/* A renderer for the surfaces of n_envs bodies described as for flash_create_batch (only elem,
 * n_vertices, n_elements, rest_x and elements are read, host, copied): a cloth env shows its
 * triangles, a tet env the faces that belong to one tet only (its boundary); triangles are
 * two-sided.  Each env's bounding-volume hierarchy is built once on rest_x; every render refits it
 * to the current positions.  Envs with equal surfaces share one hierarchy topology.  hip_stream:
 * the stream the renders run on (NULL: the renderer's own).  FLASH_ERR_INVALID_ARG for an invalid
 * description or a hierarchy deeper than 47 levels. */
flash_status flash_renderer_create(const flash_env_desc *envs, int32_t n_envs, void *hip_stream,
                                   flash_renderer **out);
flash_status flash_renderer_destroy(flash_renderer *r);

/* Renders every env's image.  x_dev: device float positions, structure of arrays [3][ld] over the
 * concatenation of the envs' vertices (env e's vertex i at column n_vertices[0] + ... +
 * n_vertices[e-1] + i; the layout flash_get_state_device writes).  obstacles: host
 * [n_envs * FLASH_MAX_OBSTACLES] records with n_obstacles[e] valid ones per env (planes, boxes and
 * capsules as in flash_set_obstacles, at the given pose), or NULL for none.  cams: host [n_envs].
 * Device outputs, caller-allocated, each optional (NULL skips it), [n_envs][height][width]
 * row-major: depth_dev float (metres along the optical axis, 0 where the ray hits nothing in front
 * of the camera), instance_dev int32 (-1 nothing, 0 the env's surface, 1 + o obstacle o),
 * points_dev float x 3 (world position of the hit, 0 where none).  FP32.  Runs on the renderer's
 * stream and returns when the images are written. */
flash_status flash_render(flash_renderer *r, const float *x_dev, int64_t ld, const flash_obstacle *obstacles,
                          const int32_t *n_obstacles, const flash_camera *cams, int32_t width, int32_t height,
                          float *depth_dev, int32_t *instance_dev, float *points_dev);

/* Checkpoint and resume.  A checkpoint holds, per env, everything the next
 * step reads besides the constant model and the network weights: positions
 * and velocities (Eq. 1's q_h, v_h, in the batch's precision, bit for bit),
 * obstacle tracks (pose, velocity, steps left to move), grippers and the
 * vertices they hold with their capture offsets (supplementary bilateral
 * constraint, Eq. 13), the warm-start cache of previous-step multipliers and
 * the learned-start state.  A batch created from the same envs, parameters
 * and capacity, with any stream grouping, that loads it and steps gives the
 * same bits as the batch that saved it.
 *   flash_checkpoint_size: bytes needed (host).
 *   flash_save_checkpoint: writes into buf (host, caller-owned, capacity
 *     bytes); FLASH_ERR_CAPACITY with *n_bytes = the size needed when buf is
 *     NULL or too small.  Synchronises.
 *   flash_load_checkpoint: n_bytes must equal flash_checkpoint_size; a blob of
 *     another shape, precision or vertex split is rejected with
 *     FLASH_ERR_INVALID_ARG before anything is written.  Synchronises. */
flash_status flash_checkpoint_size(flash_batch *b, size_t *n_bytes);
flash_status flash_save_checkpoint(flash_batch *b, void *buf, size_t capacity, size_t *n_bytes);
flash_status flash_load_checkpoint(flash_batch *b, const void *buf, size_t n_bytes);

/* Training-pair recording.  on != 0: each step also evaluates the features
 * of its contacts at the step start (a captured graph is re-captured).
 * flash_ws_collect, called after a flash_step of one step, appends one row per
 * contact of that step, env by env in contact order, to the device arrays
 * feat_dev [capacity x 16] and lab_dev [capacity x 3] starting at row
 * *n_inout, and advances *n_inout.  FLASH_ERR_CAPACITY (nothing written) if
 * the rows do not fit; FLASH_ERR_INVALID_ARG if recording is off. */
flash_status flash_ws_record(flash_batch *b, int32_t on);
flash_status flash_ws_collect(flash_batch *b, float *feat_dev, float *lab_dev, int64_t capacity,
                              int64_t *n_inout);

/* Network trainer, independent of batches.  Device-resident FP32 master
 * weights, Adam moments (beta 0.9 / 0.999, eps 1e-8) and scratch for
 * max_rows rows.  flash_mlp_create draws He-uniform weights (bound
 * sqrt(6/fan_in)) and zero biases from splitmix64(seed); hip_stream: a
 * hipStream_t or NULL for an owned one.  Arrays named *_dev are device
 * pointers; everything else is host memory.  Deterministic: a fixed seed and
 * data give bitwise identical weights. */
typedef struct flash_mlp flash_mlp;
flash_status flash_mlp_create(int64_t max_rows, uint64_t seed, void *hip_stream, flash_mlp **out);
flash_status flash_mlp_destroy(flash_mlp *m);
/* FP32 master parameters (set also resets the Adam state). */
flash_status flash_mlp_set_params(flash_mlp *m, const float *w, int64_t n);
flash_status flash_mlp_get_params(flash_mlp *m, float *w, int64_t n);
/* Parameters rounded to bf16 (nearest even), ready for flash_ws_load. */
flash_status flash_mlp_get_params_bf16(flash_mlp *m, uint16_t *w, int64_t n);
flash_status flash_mlp_set_norm(flash_mlp *m, const float *norm);
flash_status flash_mlp_get_norm(flash_mlp *m, float *norm);
/* Sets norm from raw data: feature means and 1/std (1 for constant columns,
 * the bias column passes through as 1), label scales 1/rms. */
flash_status flash_mlp_fit_norm(flash_mlp *m, const float *feat_dev, const float *lab_dev, int64_t n);
/* y_dev[n x 3] = network(x_dev[n x 16]) on already-normalised inputs. */
flash_status flash_mlp_forward(flash_mlp *m, const float *x_dev, int64_t n, float *y_dev);
/* Mean-squared loss L = sum (network(x) - target)^2 / (3 n) of normalised
 * inputs and targets (device, n <= max_rows) and its gradient with respect
 * to every parameter (host grad[FLASH_MLP_PARAMS], *loss may be NULL). */
flash_status flash_mlp_grad(flash_mlp *m, const float *x_dev, const float *target_dev, int64_t n,
                            float *grad, float *loss);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the loss and
 * gradient of flash_mlp_grad without a trainer object and without any
 * allocation.  params_dev: FP32 parameters (device, FLASH_MLP_PARAMS values in
 * the layout above); x_dev [n x 16] normalised inputs and target_dev [n x 3]
 * scaled labels (device); grad_dev [FLASH_MLP_PARAMS] and loss_dev [1]
 * (device outputs; loss_dev may be NULL).  1 <= n <= 2048.  Enqueued on
 * hip_stream (NULL: the null stream) and not synchronised.  Every
 * intermediate (activations, backward buffers, split-K partial sums, loss
 * partials: about 9.1 MB) lives in one static device array per GPU, held
 * until the process ends; calls that overlap on one GPU race on it and must
 * be serialised by the caller (one stream, or events).  The result is
 * bitwise that of flash_mlp_grad for the same parameters and rows.  Errors:
 * FLASH_ERR_INVALID_ARG for a null pointer or n <= 0, FLASH_ERR_CAPACITY for
 * n > 2048, FLASH_ERR_DEVICE if a launch fails. */
flash_status flash_mlp_grad_noalloc(const float *params_dev, const float *x_dev, const float *target_dev,
                                    int64_t n, float *grad_dev, float *loss_dev, void *hip_stream);
/* Adam on raw (feature, label) rows: per epoch a splitmix64(seed) shuffle,
 * floor(n / batch) minibatches, normalisation by the trainer's norm.
 * epoch_loss (host, epochs entries, may be NULL) receives the mean
 * minibatch loss of each epoch. */
flash_status flash_mlp_train(flash_mlp *m, const float *feat_dev, const float *lab_dev, int64_t n,
                             int32_t epochs, int32_t batch, float lr, uint64_t seed, float *epoch_loss);
/* Mean-squared loss of raw rows under the current weights and norm. */
flash_status flash_mlp_eval(flash_mlp *m, const float *feat_dev, const float *lab_dev, int64_t n,
                            float *loss);

const char *flash_last_error(void);
const char *flash_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FLASH_MI355X_H */
