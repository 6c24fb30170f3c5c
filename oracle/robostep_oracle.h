/*
 * robostep_oracle.h -- plain FP64 CPU oracle of the batched Robotarium
 * environment step (JaxRobotarium, arXiv 2505.06771, Sec. 4.1 "Design":
 * unicycle GRITSBot model, single-integrator controllers, barrier-certificate
 * QP; Appendix "Navigation (MAPF)": observation of own position and goal
 * vector, reward -1 x distance to goal).
 *
 * TEST INFRASTRUCTURE ONLY. This library exists to check the HIP path. Only
 * the test-suite, the smoke check and the CPU-baseline leg of the benchmark
 * may load it. It shares no source, header, table or helper with the HIP
 * library and must never be used as a fallback for it.
 *
 * Everything is FP64 and written for clarity, not speed: dense matrices, no
 * blocking, no pruning. The paper gives no equations for the simulator, so the
 * constants and the readings of unspecified details are documented on each
 * function.
 */
#ifndef ROBOSTEP_ORACLE_H
#define ROBOSTEP_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Simulation constants. Units: metres, seconds, radians. */
typedef struct {
  double x_min, x_max, y_min, y_max; /* arena */
  double dt;                 /* fixed integration step */
  double proj_dist;          /* l: projection-point distance ahead of the axle */
  double barrier_gain;       /* gamma of the pairwise certificate */
  double safety_radius;      /* r_s */
  double boundary_gain_factor; /* c_b: wall rows use c_b * gamma */
  double v_max;              /* speed limit per coordinate and nominal norm */
  double action_speed;       /* speed of the discrete moves */
  double kp;                 /* proportional go-to-goal gain */
  double wheel_radius;       /* R; 0 disables wheel saturation */
  double base_length;        /* L (axle length) */
  double goal_radius;        /* <= 0 disables the all-at-goal termination */
  double reset_margin;       /* reset sampler keeps this far from the walls */
  double min_sep;            /* reset sampler minimum separation */
  double grid;               /* reset sampler lattice pitch */
  int32_t max_steps;         /* <= 0 disables the time limit */
  int32_t controller;        /* 0: discrete moves, 1: proportional go-to-goal,
                                2: waypoints followed by a unicycle position controller,
                                3: waypoint poses followed by a unicycle pose controller */
  uint64_t seed;             /* Philox key */
  double waypoint_step;      /* controller 2: distance of the waypoint a move action sets */
  double pos_gain;           /* controller 2: k_v, linear speed per metre of distance */
  double ang_gain;           /* controller 2: k_w, turn rate at a 90-degree bearing */
  double action_noise;       /* sigma of the uniform action noise; 0 disables it */
  double prey_speed;         /* scenario 1: prey speed (m/s) */
  double tag_radius;         /* scenario 1: a robot centre closer than this tags the prey */
  double tag_reward;         /* scenario 1: team reward of a step with a tag */
  int32_t scenario;          /* 0: Navigation, 1: Predator-Prey */
  double pose_gain_rho;      /* controller 3: k_rho (linear speed per metre) */
  double pose_gain_alpha;    /* controller 3: k_alpha (turn rate per radian of bearing) */
  double pose_gain_beta;     /* controller 3: k_beta (weight of the goal-heading error) */
} orc_params;

/* Philox4x32-10 block cipher (Salmon, Moraes, Dror, Shaw, SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Round an FP64 value to the nearest bfloat16 (ties to even); returned as FP64. */
double orc_bf16_round(double x);

/* Reset sampler on the integer lattice: X,Y,GX,GY are lattice indices. */
void orc_reset_lattice(const orc_params *p, uint64_t env_id, int32_t episode, int32_t n,
                       int64_t *X, int64_t *Y, int64_t *GX, int64_t *GY, uint32_t *heading_bits);
/* Reset one environment: poses, goals and headings (in metres / radians). */
void orc_reset_env(const orc_params *p, uint64_t env_id, int32_t episode, int32_t n,
                   double *x, double *y, double *th, double *gx, double *gy);

/* Discrete action of robot i drawn from the counter-based stream. */
int32_t orc_random_action(const orc_params *p, uint64_t env_id, int64_t t_global, int32_t i);

/* Per-coordinate bounds of the filtered command: speed box intersected with
 * the wall certificates of the projection point. */
void orc_bounds(const orc_params *p, int32_t n, const double *px, const double *py,
                double *lo_x, double *hi_x, double *lo_y, double *hi_y);

/* Barrier certificate: magnitude pre-clip of the nominal command, then the
 * exact projection onto {pairwise rows, bounds}. Returns 0 when solved,
 * 1 when the constraint set is empty (u is then the closed-form fallback),
 * 2 on a solver failure (KKT certificate not met). lambda (may be NULL) gets
 * the n(n-1)/2 pairwise multipliers for the objective ||u - u_nom||^2.
 * kkt (may be NULL) gets {stationarity, primal violation, dual infeasibility,
 * complementarity} residuals. */
int32_t orc_barrier_certificate(const orc_params *p, int32_t n, const double *px,
                                const double *py, const double *ux_nom, const double *uy_nom,
                                double *ux, double *uy, double *lambda, double *kkt,
                                double *max_violation);

/* Largest normalized violation of u against the rows and bounds at (px, py). */
double orc_max_violation(const orc_params *p, int32_t n, const double *px, const double *py,
                         const double *ux, const double *uy);

/* Unicycle position controller: (v, w) that drive a robot at (x, y, theta)
 * toward the waypoint (wx, wy). */
void orc_unicycle_position(const orc_params *p, double x, double y, double theta, double wx,
                           double wy, double *v, double *w);

/* Unicycle pose controller: (v, w) that drive a robot at (x, y, theta) to
 * the pose (wx, wy, wth). */
void orc_unicycle_pose(const orc_params *p, double x, double y, double theta, double wx,
                       double wy, double wth, double *v, double *w);

/* Unicycle command (v, w) -> velocity of the projection point. */
void orc_uni_to_si(const orc_params *p, double theta, double v, double w, double *ux,
                   double *uy);

/* Action noise of robot i at step t_global: one uniform draw per coordinate
 * in [-action_noise, action_noise). */
void orc_action_noise(const orc_params *p, uint64_t env_id, int64_t t_global, int32_t i,
                      double *nx, double *ny);

/* Nominal single-integrator command of every robot (before the magnitude
 * pre-clip): the controller's command plus the action noise. actions may be
 * NULL (drawn from the stream); the used actions go to actions_used (may be
 * NULL). */
void orc_nominal_command(const orc_params *p, int32_t n, uint64_t env_id, int64_t t_global,
                         const double *x, const double *y, const double *th, const double *gx,
                         const double *gy, const uint8_t *actions, uint8_t *actions_used,
                         double *unx, double *uny);

/* Predator-Prey: the prey's move from (qx, qy) given the robot centres (x, y):
 * writes the new position and, if scores is not NULL, the 17 candidate
 * scores (squared distance of each candidate to the closest robot); returns
 * the index of the chosen candidate (0 = stay, k = direction 2 pi (k-1)/16). */
int32_t orc_prey_move(const orc_params *p, int32_t n, const double *x, const double *y, double qx,
                      double qy, double *nqx, double *nqy, double *scores);
/* Predator-Prey: 1 when some robot centre is closer than tag_radius to the prey. */
int32_t orc_tagged(const orc_params *p, int32_t n, const double *x, const double *y, double qx,
                   double qy);

/* Single-integrator command at the projection point -> unicycle (v, w), then
 * optional wheel saturation. */
void orc_si_to_uni(const orc_params *p, double theta, double ux, double uy, double *v, double *w);

/* Observation of every robot: 2n+4 values each. */
void orc_observe(int32_t n, const double *x, const double *y, const double *th, const double *gx,
                 const double *gy, double *obs);

/* One environment step (all robots of one environment). actions may be NULL
 * (drawn from the stream). Writes the used actions (may be NULL), the post-step
 * (post-reset) observation, the team reward, the done flag, the infeasible flag
 * and the max violation. Returns the QP status (0 ok, 1 infeasible, 2 failure). */
int32_t orc_env_step(const orc_params *p, int32_t n, uint64_t env_id, int64_t t_global,
                     double *x, double *y, double *th, double *gx, double *gy, int32_t *step,
                     int32_t *episode, const uint8_t *actions, uint8_t *actions_used,
                     double *obs, double *reward, uint8_t *done, uint8_t *infeasible,
                     double *max_violation);

/* Policy MLP (in -> 64 -> 64 -> 5, ReLU) on bf16-rounded inputs and
 * activations with FP64 sums; weights are row-major [in][out] and already
 * bf16-valued. */
void orc_policy_logits(int32_t in_dim, const double *w1, const double *b1, const double *w2,
                       const double *b2, const double *w3, const double *b3, const double *obs,
                       double *logits);
/* Inverse-CDF draw of an action from logits with the 24-bit uniform of r. */
int32_t orc_sample_action(const double *logits, uint32_t r);
/* Sampling word of robot i for step t_global. */
uint32_t orc_policy_bits(const orc_params *p, uint64_t env_id, int64_t t_global, int32_t i);

/* Batched step over E environments of n robots with the discrete controller
 * (actions NULL => drawn). State arrays are [E*n] / [E]; obs [E*n*(2n+4)]. */
int32_t orc_env_step_batch(const orc_params *p, int32_t n, int32_t num_envs, uint64_t env_id_base,
                           int64_t t_global, double *x, double *y, double *th, double *gx,
                           double *gy, int32_t *step, int32_t *episode, const uint8_t *actions,
                           double *obs, double *reward, uint8_t *done, uint8_t *infeasible,
                           int32_t nthreads);

/* Rollout of `horizon` policy steps (observe, MLP, sample, step). Outputs are
 * [H][E][n][2n+4] obs (may be NULL), [H][E][n] actions, [H][E] reward/done. */
int32_t orc_rollout(const orc_params *p, int32_t n, int32_t num_envs, uint64_t env_id_base,
                    int64_t t_global0, const double *w1, const double *b1, const double *w2,
                    const double *b2, const double *w3, const double *b3, int32_t horizon,
                    double *x, double *y, double *th, double *gx, double *gy, int32_t *step,
                    int32_t *episode, double *obs, uint8_t *actions, double *reward,
                    uint8_t *done, int32_t nthreads);

#ifdef __cplusplus
}
#endif
#endif
