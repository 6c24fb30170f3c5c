/*
 * robostep.h -- C ABI of the MI355X (gfx950) batched Robotarium environment
 * step: single-integrator commands mapped to unicycle commands through a
 * projection point, filtered by a barrier-certificate QP, integrated with a
 * fixed dt, with observations, rewards and resets, across many environments
 * at once.
 *
 * The method is JaxRobotarium's simulator (arXiv 2505.06771): Sec. 4.1
 * "Design" (unicycle GRITSBot model, single-integrator/unicycle controllers,
 * control barrier certificates solving a QP, vectorised over environments) and
 * the Navigation (MAPF) scenario of the appendix (observation of own position
 * and goal vector, reward -1 x distance to goal). The paper gives no formulas;
 * the definitions each call implements are stated on the call.
 *
 * Conventions shared by every call:
 *  - All array arguments are DEVICE pointers unless marked "host". They are
 *    owned by the caller, must stay valid until the stream work completes and
 *    must be aligned to their element size. Float arrays hold float (RS_F32)
 *    or double (RS_F64) according to rs_params.dtype, unless typed here.
 *  - Robot-indexed arrays are structure-of-arrays with robot r of environment
 *    e at index e*N + r (uniform batches) or robot_offset[e] + r (mixed).
 *  - `stream` is a hipStream_t (NULL = the null stream). Every call only
 *    enqueues work; results are valid once the stream has reached it.
 *  - Argument errors are detected before anything is enqueued and return
 *    RS_ERR_INVALID_ARG / RS_ERR_UNSUPPORTED with a message in rs_last_error().
 *    Launch failures return RS_ERR_DEVICE. Nothing aborts or throws across the
 *    ABI. An rs_ctx is not thread-safe: use one per host thread.
 *  - Per-environment infeasibility of the QP is data, not an error: the
 *    `infeasible` flag is set and the command falls back to the per-coordinate
 *    clip of the nominal command to its bounds (midpoint where they cross).
 *  - A certificate QP that stops at its iteration cap (qp_max_iters) or on a
 *    numerical failure is never silent: the per-env status outputs carry 2,
 *    the optional qp_stats counters count it, and every call adds it to the
 *    context's failure counters (rs_qp_failures).
 */
#ifndef ROBOSTEP_H
#define ROBOSTEP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RS_OK = 0,
  RS_ERR_INVALID_ARG = 1,
  RS_ERR_UNSUPPORTED = 2,
  RS_ERR_OUT_OF_MEMORY = 3,
  RS_ERR_DEVICE = 4,
  RS_ERR_BUDGET = 5,
  RS_ERR_NOT_FOUND = 6
} rs_status;

enum { RS_F32 = 0, RS_F64 = 1 };
enum { RS_CTRL_DISCRETE = 0, RS_CTRL_GOTO = 1, RS_CTRL_WAYPOINT = 2, RS_CTRL_POSE = 3 };
enum { RS_SCN_NAVIGATION = 0, RS_SCN_PREDATOR_PREY = 1 };
enum { RS_MAX_ROBOTS = 16 };

/* Simulation constants (host struct, copied at each call). Units: m, s, rad.
 * Defaults (rs_params_default): arena [-1.6,1.6]x[-1,1], dt 0.033, projection
 * distance 0.05, barrier gain 100 with a cubic class-K term, safety radius
 * 0.17, wall gain factor 0.4, |u_k| <= 0.2 and |u_nom| <= 0.2, discrete move
 * speed 0.2, go-to-goal gain 1, wheel radius 0.016 and axle 0.105 (wheel
 * speed limit v_max / R), goal radius 0.05, 500-step episodes, reset lattice
 * 1e-4 m inside a 0.2 m margin with 0.3 m separation; waypoints 0.2 ahead,
 * position controller gains k_v 0.8 and k_w pi/2; pose controller gains
 * k_rho 0.8, k_alpha 2, k_beta 0.5; no action noise;
 * Navigation scenario (Predator-Prey: prey 0.3 m/s, tag radius 0.25, tag
 * reward 10). */
typedef struct {
  double x_min, x_max, y_min, y_max;
  double dt;
  double proj_dist;
  double barrier_gain;
  double safety_radius;
  double boundary_gain_factor;
  double v_max;
  double action_speed;
  double kp;
  double wheel_radius; /* 0 disables wheel saturation */
  double base_length;
  double goal_radius;  /* <= 0 disables the all-at-goal termination */
  double reset_margin;
  double min_sep;
  double grid;
  int32_t max_steps;   /* <= 0 disables the time limit */
  int32_t controller;  /* RS_CTRL_DISCRETE, RS_CTRL_GOTO, RS_CTRL_WAYPOINT or RS_CTRL_POSE */
  int32_t dtype;       /* RS_F32 or RS_F64 */
  int32_t qp_max_iters; /* cap on active-set iterations per env; 0 = 8N+32 */
  uint64_t seed;       /* key of the counter-based stream */
  double waypoint_step; /* RS_CTRL_WAYPOINT: waypoint distance of a move action */
  double pos_gain;     /* RS_CTRL_WAYPOINT: k_v (linear speed per metre to go) */
  double ang_gain;     /* RS_CTRL_WAYPOINT: k_w (turn rate at a 90-degree bearing) */
  double action_noise; /* sigma of the uniform action noise; 0 disables it */
  double prey_speed;   /* RS_SCN_PREDATOR_PREY: prey speed */
  double tag_radius;   /* RS_SCN_PREDATOR_PREY: tag when a centre is closer than this */
  double tag_reward;   /* RS_SCN_PREDATOR_PREY: team reward of a step with a tag */
  int32_t scenario;    /* RS_SCN_NAVIGATION or RS_SCN_PREDATOR_PREY */
  double pose_gain_rho;   /* RS_CTRL_POSE: k_rho (linear speed per metre to go) */
  double pose_gain_alpha; /* RS_CTRL_POSE: k_alpha (turn rate per radian of bearing) */
  double pose_gain_beta;  /* RS_CTRL_POSE: k_beta (weight of the goal-heading error) */
} rs_params;

/* Environment batch: device structure-of-arrays views, caller-owned. */
typedef struct {
  int32_t num_envs;
  int32_t robots;              /* N (2..16) for uniform batches */
  void *x, *y, *theta;         /* [E*N] pose */
  void *goal_x, *goal_y;       /* [E*N] goal */
  int32_t *step;               /* [E] steps since the last reset */
  int32_t *episode;            /* [E] episode index (keys the reset sampler) */
  uint64_t env_id_base;        /* global id of env 0 (keys the stream) */
} rs_batch;

/* Policy of the fused rollout: in_dim = 2N+4 -> 64 -> 64 -> 5, ReLU.
 * w1 [in_dim][64], w2 [64][64], w3 [64][5] bfloat16 (uint16 bit patterns,
 * row-major [in][out]); b1 [64], b2 [64], b3 [5] float. Device pointers. */
typedef struct {
  const uint16_t *w1, *w2, *w3;
  const float *b1, *b2, *b3;
  int32_t in_dim;
} rs_policy;

typedef struct rs_ctx rs_ctx;
typedef struct rs_plan rs_plan;

/* Per-env certificate statistics (the optional `qp_stats` outputs): int32
 * [E][RS_QPS_COUNT], accumulated (+=) over every solve of the call, so a
 * caller zeroes them first. Each solve adds 1 to exactly one of slots 0..7:
 * the stage that produced the command (BOX: no row violated at the box clip
 * of the nominal command; ONE_ROW: one active row, projected in closed
 * form; TWO_ROWS: two violated rows on four distinct robots; SHARED_ROBOT:
 * two or three active rows through shared robots with no bound binding,
 * from their Gram system (FP32 also takes this stage when a one-row guess
 * is rejected: the guessed row plus the row it violates; and for exactly
 * three violated rows); ACTIVE_SET: the
 * register-resident dual active-set loop; GENERAL: the general active-set
 * solver with its rows in LDS), or INFEASIBLE (no feasible command) or
 * CAPPED (stopped by the iteration cap or a numerical failure). ITERATIONS
 * sums the active-set iterations of the solves that ran the loop. */
enum {
  RS_QPS_BOX = 0,
  RS_QPS_ONE_ROW = 1,
  RS_QPS_TWO_ROWS = 2,
  RS_QPS_SHARED_ROBOT = 3,
  RS_QPS_ACTIVE_SET = 4,
  RS_QPS_GENERAL = 5,
  RS_QPS_INFEASIBLE = 6,
  RS_QPS_CAPPED = 7,
  RS_QPS_ITERATIONS = 8,
  RS_QPS_COUNT = 9
};

void rs_params_default(rs_params *p);
/* Validates p as every call does (host only, no device work): RS_OK or
 * RS_ERR_INVALID_ARG with the reason in rs_last_error(). */
rs_status rs_params_check(const rs_params *p);
const char *rs_status_string(rs_status s);
/* Message of the last failed call on this host thread ("" if none). */
const char *rs_last_error(void);

/* Create a context on HIP device `device` (workspace, schedule table, graph
 * cache). */
rs_status rs_create(int device, rs_ctx **out);
rs_status rs_destroy(rs_ctx *ctx);

/* Certificate failures counted on the device by every call on ctx
 * (env_step, barrier_certificate, rollout, env_run, server ticks) since the
 * context was created or last reset: solves with no feasible command
 * (*infeasible) and solves stopped by the iteration cap or a numerical
 * failure (*capped). Waits for all work queued on the context's device.
 * reset != 0 zeroes both counters after reading. Either pointer may be NULL. */
rs_status rs_qp_failures(rs_ctx *ctx, int64_t *infeasible, int64_t *capped, int32_t reset);

/* ---------------------------------------------------------------------------
 * env_reset -- reset sampler (start poses uniform with a minimum separation,
 * goals uniform, headings uniform; the single-env navigation configuration of
 * the paper's Sec. 4.2 evaluation scenario and the Navigation appendix).
 * For every env e with mask[e] != 0 (mask NULL = all): positions and goals are
 * drawn on the integer lattice of pitch `grid` inside the arena shrunk by
 * `reset_margin`; robot i keeps the first of up to 64 draws (Philox4x32-10,
 * key = seed, counter = (env_id, episode[e], purpose<<24 | i, attempt),
 * purpose 2 for poses and 3 for goals) whose squared lattice distance to every
 * robot < i is >= round(min_sep/grid)^2, else the first point of a row-major
 * scan of every 500th lattice point that is; headings are -pi + 2 pi u with u
 * the 24-bit uniform of word i&3 of block (env_id, episode, 4<<24 | i>>2, 0).
 * step[e] is set to 0; episode[e] is left as given. obs (may be NULL) gets the
 * observation [E*N][2N+4] of the reset envs (others untouched).
 * RS_SCN_PREDATOR_PREY: every goal slot of env e gets the prey, the goal
 * sampler's first point (robot 0's goal).
 * ------------------------------------------------------------------------- */
rs_status env_reset(rs_ctx *ctx, const rs_params *p, const rs_batch *b, const uint8_t *mask,
                    void *obs, void *stream);

/* ---------------------------------------------------------------------------
 * env_step -- one step of every env of the batch (Sec. 4.1 "Design"):
 *  1. nominal single-integrator command at the projection point
 *     p_i = (x_i + l cos th_i, y_i + l sin th_i): discrete move
 *     action_speed * {0, +x, -x, +y, -y}[a_i] (actions NULL: a_i =
 *     floor(5 r / 2^32), r = word i&3 of block (env_id, t_global, i>>2, 0)),
 *     or kp (g_i - p_i) for RS_CTRL_GOTO, or for RS_CTRL_WAYPOINT (waypoint
 *     actions followed by a unicycle position controller: Sec. 6.1 and the
 *     scenario appendix) the waypoint w_i = (x_i, y_i) + waypoint_step *
 *     {0, +x, -x, +y, -y}[a_i] steered to by v = k_v rho cos(alpha),
 *     w = k_w sin(alpha) (rho = |w_i - (x_i, y_i)|, alpha = bearing of w_i
 *     from the heading; v = w = 0 at the waypoint), taken to the projection
 *     point as (v cos th - l w sin th, v sin th + l w cos th); or for
 *     RS_CTRL_POSE (waypoint poses followed by a unicycle pose controller:
 *     Sec. 4.1, unicycle controllers to positions/poses; Table 1) the pose
 *     waypoint_step ahead along dir(a) with heading along dir(a) (a = 0: the
 *     robot's own pose) steered to by v = k_rho rho cos(alpha), w = k_alpha
 *     alpha + k_rho (sin(alpha) cos(alpha)/alpha)(alpha + k_beta beta)
 *     (alpha = bearing of the goal position from the heading in (-pi, pi],
 *     beta = bearing of it from the goal heading, 0 for these waypoints),
 *     taken to the projection point the same way; then, when
 *     action_noise = sigma > 0 (action-noise domain randomisation, Sec. 7),
 *     plus sigma (2 u - 1) per coordinate with u the 24-bit uniforms of
 *     words 0 (x) and 1 (y) of block (env_id, t_global, 6<<24 | i, 0);
 *     magnitude clipped to v_max;
 *  2. barrier certificate: u = argmin |u - u_nom|^2 subject to, for i<j,
 *     -2 D.u_i + 2 D.u_j <= gamma (|D|^2 - r_s^2)^3 with D = p_i - p_j, and
 *     per coordinate lo <= u <= hi where hi_x = min(v_max, c_b gamma
 *     (x_max - r_s/2 - p_x)^3), lo_x = max(-v_max, -c_b gamma
 *     (p_x - x_min - r_s/2)^3) (same in y), solved exactly;
 *  3. v = cos th u_x + sin th u_y, w = (-sin th u_x + cos th u_y)/l, wheel
 *     speeds (v +- w L/2)/R clipped to +-v_max/R and mapped back;
 *  4. Euler: x += dt v cos th, y += dt v sin th, th += dt w, wrapped to
 *     [-pi, pi];
 *  5. step += 1; reward = -sum_i |(x_i, y_i) - g_i|; done = (all distances <
 *     goal_radius) or step >= max_steps; done envs are reset (episode += 1);
 *     RS_SCN_PREDATOR_PREY (the Predator Prey scenario of the appendix):
 *     every robot's goal slot holds the env's prey q. Before the robots
 *     move, the prey takes the candidate, among staying at q and
 *     clamp(q + prey_speed dt (cos 2 pi k/16, sin 2 pi k/16)) for k = 0..15
 *     (clamped to the arena pulled in by r_s/2; candidates in that order),
 *     that maximises the squared distance to the closest robot centre of
 *     the pre-step state, the first on ties. After both moved, reward =
 *     tag_reward if some centre is closer than tag_radius to the prey, else
 *     0; done = step >= max_steps only;
 *  6. obs [E*N][2N+4] of the post-step (post-reset) state, per robot: x, y,
 *     cos th, sin th, (x_j - x_i, y_j - y_i) for j != i ascending, g_i - (x,y).
 * actions: [E*N] uint8 in 0..4 or NULL. reward [E] (float/double), done [E],
 * max_violation [E] float (NULL ok: largest normalised row/bound violation of
 * the command), infeasible [E] uint8 (NULL ok): the certificate's status,
 * 0 solved, 1 no feasible command (per-coordinate fallback), 2 stopped by the
 * iteration cap or a numerical failure (the intermediate command is used).
 * qp_stats [E][RS_QPS_COUNT] int32 (NULL ok): accumulated statistics.
 * obs/reward/done may be NULL.
 * ------------------------------------------------------------------------- */
rs_status env_step(rs_ctx *ctx, const rs_params *p, const rs_batch *b, const uint8_t *actions,
                   int64_t t_global, void *obs, void *reward, uint8_t *done, float *max_violation,
                   uint8_t *infeasible, int32_t *qp_stats, void *stream);

/* ---------------------------------------------------------------------------
 * env_steps -- `steps` consecutive env_step calls (Sec. 4.1, the step as
 * above) of a uniform batch in one launch, the state held on chip between
 * them: the persistent form of env_step in either precision (p->dtype), e.g.
 * the 1000 steps of a single FP64 env. Step k (0-based) runs at stream time
 * t_global0 + k with the actions env_step draws when given none (the
 * discrete and waypoint controllers; go-to-goal takes none). Results are
 * those of `steps` env_step calls with actions NULL at the same stream
 * times, bit for bit. b is updated in place.
 *  reward_out [steps][E] (float/double by dtype), done_out [steps][E] uint8:
 *    per step, as env_step's reward and done; obs_final [E*N][2N+4]
 *    (float/double): the observation of the final state; qp_stats
 *    [E][RS_QPS_COUNT] int32, accumulated. Each may be NULL.
 *  steps >= 0 (0: nothing is launched); steps * E must fit in int32.
 *  Errors: RS_ERR_INVALID_ARG for a NULL ctx, invalid params or batch, or
 *  steps out of range; RS_ERR_DEVICE if the launch fails.
 * ------------------------------------------------------------------------- */
rs_status env_steps(rs_ctx *ctx, const rs_params *p, const rs_batch *b, int32_t steps,
                    int64_t t_global0, void *reward_out, uint8_t *done_out, void *obs_final,
                    int32_t *qp_stats, void *stream);

/* ---------------------------------------------------------------------------
 * barrier_certificate -- steps 1 (pre-clip) and 2 of env_step alone, for
 * E environments of N robots: given projection points (px, py) and nominal
 * commands (ux_nom, uy_nom) [E*N], writes the exact minimiser (ux, uy) [E*N].
 * lambda (may be NULL): [E][N(N-1)/2] multipliers of the pairwise rows (pairs
 * i<j in lexicographic order) for the objective |u - u_nom|^2; not unique
 * under degeneracy. max_violation [E] float, infeasible [E] (status 0/1/2 as
 * in env_step) and qp_stats [E][RS_QPS_COUNT] (accumulated) may be NULL.
 * ------------------------------------------------------------------------- */
rs_status barrier_certificate(rs_ctx *ctx, const rs_params *p, int32_t num_envs, int32_t robots,
                              const void *px, const void *py, const void *ux_nom,
                              const void *uy_nom, void *ux, void *uy, void *lambda,
                              float *max_violation, uint8_t *infeasible, int32_t *qp_stats,
                              void *stream);

/* ---------------------------------------------------------------------------
 * rollout -- `horizon` fused policy steps in one persistent launch (FP32 state,
 * RS_CTRL_DISCRETE, RS_CTRL_WAYPOINT or RS_CTRL_POSE, action noise and scenario as set).
 * For t = 0..H-1:
 * obs_t of the current state; logits = MLP(bf16(obs_t)) with bf16 weights
 * and activations and FP32 accumulation;
 * a_t drawn by inverse CDF of softmax(logits) with the 24-bit uniform of word
 * i&3 of block (env_id, t_global0 + t, 1<<24 | i>>2, 0); then env_step with a_t
 * (stream time t_global0 + t). Outputs: obs [H][E*N][2N+4] float (may be NULL),
 * actions [H][E*N] uint8, reward [H][E] float, done [H][E] uint8. The batch
 * state is left at the post-rollout state. Requires 2N+4 <= 32.
 * qp_stats [E][RS_QPS_COUNT] int32 (NULL ok) accumulates the certificate
 * statistics of all H steps; it selects a separately compiled kernel that
 * counts them (the kernel without it carries none of that code).
 * The launch is captured once per (shape, pointers) in a hipGraph and replayed.
 * ------------------------------------------------------------------------- */
rs_status rollout(rs_ctx *ctx, const rs_params *p, const rs_batch *b, const rs_policy *policy,
                  int32_t horizon, int64_t t_global0, float *obs, uint8_t *actions,
                  float *reward, uint8_t *done, int32_t *qp_stats, void *stream);

/* Diagnostic builds only (library compiled with RS_PHASE_TIMERS, see
 * paper_2505_06771_amd/build.py --phase-timers): copies the phase cycles of
 * the last rollout launch's first `waves` wavefronts (wavefront w owns envs
 * w*64/G .. w*64/G + 64/G - 1, G = lanes per env) to host out [waves][8]:
 * shader-clock cycles spent in the observation, MLP, sampling, pre-QP, QP
 * and post-QP phases of all steps, the number of steps in which some env of
 * the wavefront ran the active-set loop, and the cycles of the whole step
 * loop. Waits for the device. RS_ERR_UNSUPPORTED in the plain library. */
rs_status rs_phase_cycles(rs_ctx *ctx, int64_t *out, int32_t waves);

/* ---------------------------------------------------------------------------
 * Snapshot / restore (checkpoint and resume) of a batch's state: pose, goal,
 * step and episode arrays. The stream is counter based (env id, stream time),
 * so these are all a bit-identical resume needs. A snapshot is a host buffer
 * of rs_snapshot_bytes bytes: a 32-byte header (magic "RSSNAP1", dtype,
 * num_envs, robots_total), then x, y, theta, goal_x, goal_y ([robots_total]
 * values of dtype each) and step, episode ([num_envs] int32 each).
 * robots_total = num_envs * robots for a uniform batch, or
 * rs_plan_total_robots for a mixed one. Both calls are stream-ordered and
 * synchronise `stream` before returning. Errors: NULL pointers, a buffer
 * smaller than rs_snapshot_bytes, or (restore) a header that does not match
 * dtype / num_envs / robots_total: RS_ERR_INVALID_ARG before any copy;
 * copy failures: RS_ERR_DEVICE.
 * ------------------------------------------------------------------------- */
int64_t rs_snapshot_bytes(int32_t dtype, int32_t num_envs, int64_t robots_total);
rs_status rs_snapshot(rs_ctx *ctx, int32_t dtype, const rs_batch *b, int64_t robots_total,
                      void *host, int64_t bytes, void *stream);
rs_status rs_restore(rs_ctx *ctx, int32_t dtype, const rs_batch *b, int64_t robots_total,
                     const void *host, int64_t bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Mixed-size batches (environments with different robot counts in one launch).
 * A plan holds the schedule: envs grouped by robot count into wavefront tiles
 * (lanes per env and envs per wavefront chosen per robot count by the
 * autotuner or `schedule`).
 * robots_per_env is a HOST array [E] of counts in 2..16; the robot arrays of a
 * mixed batch are laid out env after env (robot_offset = prefix sum).
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t block_threads;     /* 64..256, multiple of 64; 0 = 256 */
  int32_t lanes_per_env[17]; /* indexed by N: power of two >= N, <= 16; 0 = smallest */
  int32_t qp_iters[17];      /* indexed by N: active-set iteration cap; 0 = 8N+32 */
  int32_t envs_per_wave[17]; /* indexed by N: envs sharing a wavefront, 1..64/lanes;
                                0 = 64/lanes (a wavefront runs the solver stages any
                                of its envs needs, so fewer envs per wavefront run
                                fewer of them per env, on more wavefronts) */
} rs_schedule;

rs_status rs_plan_create(rs_ctx *ctx, int32_t num_envs, const int32_t *robots_per_env,
                         const rs_schedule *schedule, rs_plan **out);
rs_status rs_plan_destroy(rs_plan *plan);
/* Total robots of the plan and the device prefix-sum array [E+1]. */
int64_t rs_plan_total_robots(const rs_plan *plan);
const int32_t *rs_plan_robot_offset(const rs_plan *plan);

/* env_reset for a mixed batch (FP32): b->robots is ignored; arrays use the
 * plan's robot offsets; reset definition as env_reset. The mask [E] (NULL =
 * all) is only read; the call allocates nothing. */
rs_status env_reset_mixed(rs_ctx *ctx, const rs_params *p, const rs_plan *plan,
                          const rs_batch *b, const uint8_t *mask, void *stream);

/* ---------------------------------------------------------------------------
 * env_run -- `steps` consecutive env_step calls with drawn actions for a mixed
 * batch in ONE persistent launch (FP32; RS_CTRL_DISCRETE, RS_CTRL_WAYPOINT or RS_CTRL_POSE,
 * action noise and scenario as set). Env e runs
 * steps_per_env ? min(steps, steps_per_env[e]) : steps steps, with stream time
 * t_start[e] + k (t_start NULL: t_global0 + k) at its k-th step. Outputs (each
 * may be NULL): reward_out/done_out [steps][E] (rows past an env's own count
 * untouched), reward_sum [E] (accumulated: += sum of the env's rewards),
 * obs_final: observation of the final state, env e's block of N_e x (2N_e+4)
 * floats starting at rs_plan_obs_offset(plan, e); qp_stats [E][RS_QPS_COUNT]
 * int32, accumulated certificate statistics. Results per env do not
 * depend on the other envs in the batch or on the schedule (as long as the
 * iteration cap is not reached: see rs_qp_failures and RS_QPS_CAPPED; and up
 * to rounding when two candidate rows of a three-row or second guess tie in
 * the top 15 bits of their scores, which the guess breaks by lane).
 * ------------------------------------------------------------------------- */
rs_status env_run(rs_ctx *ctx, const rs_params *p, const rs_plan *plan, const rs_batch *b,
                  int32_t steps, const int64_t *t_start, int64_t t_global0,
                  const int32_t *steps_per_env, float *reward_out, uint8_t *done_out,
                  float *reward_sum, float *obs_final, int32_t *qp_stats, void *stream);
/* Offset of env e's observation block in obs_final (host query). */
int64_t rs_plan_obs_offset(const rs_plan *plan, int32_t env);

/* ---------------------------------------------------------------------------
 * env_run_noalloc -- for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc). The same launch and results as env_run with a plan made from
 * the same robot counts (results do not depend on the schedule), but the work
 * list that a plan keeps in memory it allocates (robot and observation
 * offsets, env order, wavefront tiles) is built on `stream` by a small kernel
 * into one fixed device array of the library (RS_NOALLOC_SCRATCH_BYTES per
 * device, taken when the code is loaded and held until the process ends).
 * The call allocates nothing: no hipMalloc, hipFree or allocating library
 * routine.
 *  robots_per_env: DEVICE int32 [b->num_envs], each 2..16; b's robot arrays
 *    are laid out env after env (robot offset = prefix sum of the counts) and
 *    env e's block of obs_final starts at sum over e' < e of N_e'(2N_e'+4).
 *  b->num_envs: 1..RS_NOALLOC_MAX_ENVS, else RS_ERR_INVALID_ARG before any
 *    device work.
 *  bad_envs: DEVICE int32 [1] (may be NULL): set to the number of envs whose
 *    count is outside 2..16; when that is nonzero no env is stepped and no
 *    output is written.
 *  The schedule (lanes and envs per wavefront, iteration caps, block size) is
 *  the context's (rs_autotune); failures add to the context's counters. Other
 *  arguments as env_run.
 *  Every call on a device shares that device's array: calls that overlap on
 *  one device (two streams, or two host threads) race; order them on one
 *  stream.
 * ------------------------------------------------------------------------- */
#define RS_NOALLOC_MAX_ENVS 65536
#define RS_NOALLOC_SCRATCH_BYTES 2098176
rs_status env_run_noalloc(rs_ctx *ctx, const rs_params *p, const int32_t *robots_per_env,
                          const rs_batch *b, int32_t steps, const int64_t *t_start,
                          int64_t t_global0, const int32_t *steps_per_env, float *reward_out,
                          uint8_t *done_out, float *reward_sum, float *obs_final,
                          int32_t *qp_stats, int32_t *bad_envs, void *stream);

/* ---------------------------------------------------------------------------
 * Autotuner: builds the mixed workload of `envs` synthetic envs of every robot
 * count in `robots` (host [count], each 2..16; half drawn by the reset
 * sampler, half packed in a tight cluster so the certificate binds) and times
 * env_run over `steps` steps (best of 3) under candidate schedules, by
 * coordinate descent from the default schedule: block size in {64, 128, 256},
 * then per size lanes per env doubled, envs per wavefront in {1/2, 1/4, 1/8}
 * of a full tile (at least 1) and the active-set iteration cap in
 * {2N+4, 4N+8}. A change is kept when
 * no certificate solve of its run stopped at the iteration cap (so every
 * step reached the exact minimiser), every final position matches the
 * default-schedule, widest-cap reference within steps * dt * tol (tol in
 * m/s), and it is at least 2% faster, so the result is never slower than the
 * default on this workload. The tuning runs use the tuner's own failure
 * counters, not the context's. The schedule is
 * stored in the context (used by plans created afterwards with schedule NULL)
 * and returned in `out` (may be NULL). Allocates device scratch for the
 * workload; RS_ERR_OUT_OF_MEMORY if that fails.
 * ------------------------------------------------------------------------- */
rs_status rs_autotune(rs_ctx *ctx, const rs_params *p, const int32_t *robots, int32_t count,
                      int32_t envs, int32_t steps, double tol, rs_schedule *out);
/* The same search on the caller's own mixed batch (plan + b, FP32): every
 * candidate runs `steps` env_run steps from a copy of b's state, which is
 * left unchanged; the schedule is stored in the context and returned in out
 * (may be NULL). Allocates device scratch for the copy (RS_ERR_OUT_OF_MEMORY
 * if that fails). */
rs_status rs_autotune_batch(rs_ctx *ctx, const rs_params *p, const rs_plan *plan,
                            const rs_batch *b, int32_t steps, double tol, rs_schedule *out);
rs_status rs_get_schedule(rs_ctx *ctx, rs_schedule *out);
/* Sets the context's schedule (used by plans created afterwards with schedule
 * NULL, by env_run_noalloc and by the server), e.g. one an earlier
 * rs_autotune returned. Checked on the host: block_threads 0 or a multiple of
 * 64 up to 256; per robot count n = 2..16, lanes_per_env[n] 0 or a power of
 * two in n..16, envs_per_wave[n] 0..64/lanes, qp_iters[n] >= 0;
 * RS_ERR_INVALID_ARG otherwise, the schedule left unchanged. */
rs_status rs_set_schedule(rs_ctx *ctx, const rs_schedule *s);

/* ---------------------------------------------------------------------------
 * Serving loop (continuous batching of rollout requests).
 * A request is (envs, robots, horizon, seed): envs environments of `robots`
 * robots reset from the sampler (env ids = the request's id << 20 | e, episode
 * 0) and stepped `horizon` times with drawn actions; its result is the final
 * pose of every robot and the summed reward of every env. The server admits
 * queued requests in arrival order while their device bytes fit in the HBM
 * budget, keeps all admitted state device-resident, and advances every
 * admitted env `tick_steps` steps per tick with one persistent env_run launch
 * over all of them, so requests that arrive while others run join at the next
 * tick. Results of a request do not depend on what else is admitted.
 * ------------------------------------------------------------------------- */
typedef struct rs_server rs_server;
typedef struct {
  int64_t id;
  int32_t envs, robots, horizon;
  double submit_time, admit_time, finish_time; /* seconds, steady clock */
} rs_request_info;

rs_status rs_server_create(rs_ctx *ctx, const rs_params *p, int64_t hbm_budget_bytes,
                           int32_t tick_steps, rs_server **out);
rs_status rs_server_destroy(rs_server *s);
/* Device bytes a request needs while admitted. */
int64_t rs_request_bytes(int32_t envs, int32_t robots);
/* Queue a request; returns RS_ERR_BUDGET if it can never fit. The id keys the
 * request's streams (env id = id << 20 | env index), so ids are limited to
 * 0..4095 (RS_ERR_INVALID_ARG otherwise) and requests that run at the same
 * time need distinct ids; a long-running server recycles ids of finished
 * requests, whose results then repeat for equal (id, envs, robots, horizon). */
rs_status rs_server_submit(rs_server *s, int64_t id, int32_t envs, int32_t robots,
                           int32_t horizon);
/* Run one tick: admit, launch, retire finished requests. *busy = 1 while any
 * request is queued or running. */
rs_status rs_server_tick(rs_server *s, int32_t *busy);
/* Pop one finished request: copies its result to host arrays
 * final_xy [envs*robots*2] (x, y interleaved) and reward_sum [envs] (either
 * may be NULL). Returns RS_ERR_NOT_FOUND when none is finished. */
rs_status rs_server_poll(rs_server *s, rs_request_info *info, float *final_xy,
                         float *reward_sum);
typedef struct {
  int64_t submitted, admitted, finished, ticks;
  int64_t robot_steps;       /* total robot-steps executed */
  int64_t bytes_in_use, peak_bytes;
  int32_t queued, running;
} rs_server_stats;
rs_status rs_server_stats_get(rs_server *s, rs_server_stats *out);

#ifdef __cplusplus
}
#endif
#endif
