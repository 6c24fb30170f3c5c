// rs_lib.hip -- kernels and C-ABI entry points of the uniform-batch calls:
// env_reset, env_step, barrier_certificate (FP32 and FP64).
//
// Launch shape: 256-thread blocks; each block holds 256/G environments, one
// aligned group of G = next power of two >= N lanes per environment, lane i
// = robot i. State is structure-of-arrays in HBM (index e*N + i), so a group
// reads N consecutive elements of each field and a wavefront reads 64/G*N
// consecutive elements: the loads coalesce. The QP scratch of each group
// lives in LDS.
#include "rs_internal.hpp"

#include <cstddef>
#include "rs_step.hpp"

#include <cstring>

namespace rs {

static thread_local std::string g_error;

void set_error(const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_error = buf;
}
void clear_error() { g_error.clear(); }

rs_status check_params(const rs_params *p) {
  RS_CHECK_ARG(p != nullptr, "params is NULL");
  RS_CHECK_ARG(p->x_max > p->x_min && p->y_max > p->y_min, "empty arena");
  RS_CHECK_ARG(p->dt > 0 && p->proj_dist > 0 && p->v_max > 0, "dt, proj_dist, v_max must be > 0");
  RS_CHECK_ARG(p->barrier_gain > 0 && p->safety_radius > 0, "barrier gain, safety radius must be > 0");
  RS_CHECK_ARG(p->grid > 0, "grid must be > 0");
  RS_CHECK_ARG(p->dtype == RS_F32 || p->dtype == RS_F64, "dtype must be RS_F32 or RS_F64");
  RS_CHECK_ARG(p->controller == RS_CTRL_DISCRETE || p->controller == RS_CTRL_GOTO ||
                   p->controller == RS_CTRL_WAYPOINT || p->controller == RS_CTRL_POSE,
               "unknown controller %d", p->controller);
  RS_CHECK_ARG(p->waypoint_step >= 0 && p->pos_gain >= 0 && p->ang_gain >= 0,
               "waypoint step and controller gains must be >= 0");
  RS_CHECK_ARG((p->controller != RS_CTRL_WAYPOINT && p->controller != RS_CTRL_POSE) ||
                   p->waypoint_step > 0,
               "the waypoint and pose controllers need waypoint_step > 0");
  RS_CHECK_ARG(p->pose_gain_rho >= 0 && p->pose_gain_alpha >= 0 && p->pose_gain_beta >= 0,
               "pose controller gains must be >= 0");
  RS_CHECK_ARG(p->action_noise >= 0 && p->action_noise <= 1e3, "action_noise must be in [0, 1e3]");
  RS_CHECK_ARG(p->scenario == RS_SCN_NAVIGATION || p->scenario == RS_SCN_PREDATOR_PREY,
               "unknown scenario %d", p->scenario);
  RS_CHECK_ARG(p->prey_speed >= 0 && p->tag_radius >= 0,
               "prey_speed and tag_radius must be >= 0");
  RS_CHECK_ARG(p->qp_max_iters >= 0, "qp_max_iters must be >= 0");
  const double xlo = std::llround((p->x_min + p->reset_margin) / p->grid);
  const double xhi = std::llround((p->x_max - p->reset_margin) / p->grid);
  const double ylo = std::llround((p->y_min + p->reset_margin) / p->grid);
  const double yhi = std::llround((p->y_max - p->reset_margin) / p->grid);
  RS_CHECK_ARG(xhi >= xlo && yhi >= ylo, "reset margin leaves no room in the arena");
  RS_CHECK_ARG(xhi - xlo < 4.0e9 && yhi - ylo < 4.0e9, "reset lattice too fine for 32-bit draws");
  return RS_OK;
}

template <typename T> static bool aligned(const void *ptr) {
  return ((uintptr_t)ptr % sizeof(T)) == 0;
}

constexpr int kBlock = 256;
static_assert(kQPStats == RS_QPS_COUNT, "qp_stats layout of robostep.h");

// ---------------------------------------------------------------------------
// env_step
// ---------------------------------------------------------------------------
template <typename T> struct StepArgs {
  SimConst<T> C;
  int E, N;
  uint32_t env_base;
  uint32_t t_global;
  T *x, *y, *th, *gx, *gy;
  int32_t *step, *episode;
  const uint8_t *actions;
  T *obs, *reward;
  uint8_t *done, *infeasible;
  float *maxviol;
  int32_t *qp_stats;             // [E][kQPStats] accumulated (may be NULL)
  unsigned long long *qp_fail;   // the context's failure counters
};

template <typename T, int G, bool PP>
__global__ __launch_bounds__(kBlock) void k_env_step(StepArgs<T> A) {
  __shared__ QPScratch<T, G> qs[kBlock / G];
  const int lane = threadIdx.x & 63;
  const int i = threadIdx.x & (G - 1);
  const int e = blockIdx.x * (kBlock / G) + threadIdx.x / G;
  if (e >= A.E) return;  // whole group leaves together
  const int N = A.N;
  const bool on = i < N;
  const size_t r = (size_t)e * N + (on ? i : 0);
  T x = A.x[r], y = A.y[r], th = A.th[r], gx = A.gx[r], gy = A.gy[r];
  int step = A.step[e], episode = A.episode[e];
  const uint32_t env_id = A.env_base + (uint32_t)e;
  const ConstRef<T> K = kernarg_const<T>(offsetof(StepArgs<T>, C));
  int action = 0;
  if (A.C.controller != RS_CTRL_GOTO)
    action = A.actions ? (int)A.actions[r]
                       : drawn_action(K.get()->key0, K.get()->key1, env_id, A.t_global, i);
  T s, c;
  sincos_t(th, &s, &c);
  StepOut<T> out = env_step_group<T, G, PP>(K, A.C.qp_cap, &qs[threadIdx.x / G], lane, i, N, on,
                                        env_id, (uint32_t)A.t_global, action, x, y, th, c, s, gx, gy, step, episode,
                                        A.maxviol != nullptr);
  if (on) {
    A.x[r] = x; A.y[r] = y; A.th[r] = th; A.gx[r] = gx; A.gy[r] = gy;
  }
  if (A.obs) write_obs<T, G>(A.obs + r * (2 * N + 4), lane, i, N, on, x, y, c, s, gx, gy);
  if (i == 0) {
    A.step[e] = step;
    A.episode[e] = episode;
    if (A.reward) A.reward[e] = out.reward;
    if (A.done) A.done[e] = out.done ? 1 : 0;
    if (A.infeasible) A.infeasible[e] = (uint8_t)out.qp.status;
    if (A.maxviol) A.maxviol[e] = (float)out.maxviol;
    if (A.qp_stats) qp_stats_add(A.qp_stats + (size_t)e * kQPStats, out.qp);
    qp_fail_count(A.qp_fail, out.qp);
  }
}

// ---------------------------------------------------------------------------
// env_steps: `steps` env steps of a uniform batch in one launch, the state in
// registers between them (the persistent form of env_step, FP32 or FP64)
// ---------------------------------------------------------------------------
template <typename T> struct StepsArgs {
  SimConst<T> C;
  int E, N, steps;
  uint32_t env_base;
  uint32_t t0;
  T *x, *y, *th, *gx, *gy;
  int32_t *step, *episode;
  T *reward;                     // [steps][E] (may be NULL)
  uint8_t *done;                 // [steps][E] (may be NULL)
  T *obs;                        // final state [E*N][2N+4] (may be NULL)
  int32_t *qp_stats;             // [E][kQPStats] accumulated (may be NULL)
  unsigned long long *qp_fail;   // the context's failure counters
};

template <typename T, int G, bool PP>
__global__ __launch_bounds__(kBlock) void k_env_steps(StepsArgs<T> A) {
  __shared__ QPScratch<T, G> qs[kBlock / G];
  const int lane = threadIdx.x & 63;
  const int i = threadIdx.x & (G - 1);
  const int e = blockIdx.x * (kBlock / G) + threadIdx.x / G;
  if (e >= A.E) return;  // whole group leaves together
  const int N = A.N;
  const bool on = i < N;
  const size_t r = (size_t)e * N + (on ? i : 0);
  T x = A.x[r], y = A.y[r], th = A.th[r], gx = A.gx[r], gy = A.gy[r];
  int step = A.step[e], episode = A.episode[e];
  const uint32_t env_id = A.env_base + (uint32_t)e;
  const ConstRef<T> K = kernarg_const<T>(offsetof(StepsArgs<T>, C));
  // complete the state loads before the loop: an in-loop wait on them would
  // also wait for the loop's own stores
  __builtin_amdgcn_s_waitcnt(0);
  T s, c;
  sincos_t(th, &s, &c);
  for (int k = 0; k < A.steps; ++k) {
    const uint32_t t = A.t0 + (uint32_t)k;
    int action = 0;
    if (A.C.controller != RS_CTRL_GOTO)
      action = drawn_action(K.get()->key0, K.get()->key1, env_id, t, i);
    const StepOut<T> out = env_step_group<T, G, PP>(K, A.C.qp_cap, &qs[threadIdx.x / G], lane, i,
                                                    N, on, env_id, t, action, x, y, th, c, s, gx,
                                                    gy, step, episode, false);
    if (i == 0) {
      if (A.reward) A.reward[(size_t)k * A.E + e] = out.reward;
      if (A.done) A.done[(size_t)k * A.E + e] = out.done ? 1 : 0;
      if (A.qp_stats) qp_stats_add(A.qp_stats + (size_t)e * kQPStats, out.qp);
      qp_fail_count(A.qp_fail, out.qp);
    }
  }
  if (on) {
    A.x[r] = x; A.y[r] = y; A.th[r] = th; A.gx[r] = gx; A.gy[r] = gy;
  }
  if (A.obs) write_obs<T, G>(A.obs + r * (2 * N + 4), lane, i, N, on, x, y, c, s, gx, gy);
  if (i == 0) {
    A.step[e] = step;
    A.episode[e] = episode;
  }
}

// ---------------------------------------------------------------------------
// env_reset
// ---------------------------------------------------------------------------
template <typename T> struct ResetArgs {
  SimConst<T> C;
  int E, N;
  uint32_t env_base;
  T *x, *y, *th, *gx, *gy;
  int32_t *step, *episode;
  const uint8_t *mask;
  T *obs;
};

template <typename T, int G, bool PP>
__global__ __launch_bounds__(kBlock) void k_env_reset(ResetArgs<T> A) {
  const int lane = threadIdx.x & 63;
  const int i = threadIdx.x & (G - 1);
  const int e = blockIdx.x * (kBlock / G) + threadIdx.x / G;
  if (e >= A.E) return;
  if (A.mask && !A.mask[e]) return;
  const int N = A.N;
  const bool on = i < N;
  const size_t r = (size_t)e * N + (on ? i : 0);
  const int episode = A.episode[e];
  T x, y, th, gx, gy;
  reset_env<T, G, PP>(kernarg_const<T>(offsetof(ResetArgs<T>, C)), A.env_base + (uint32_t)e,
                  (uint32_t)episode, i, N, lane, x, y, th, gx, gy);
  if (on) {
    A.x[r] = x; A.y[r] = y; A.th[r] = th; A.gx[r] = gx; A.gy[r] = gy;
  }
  if (A.obs) {
    T s, c;
    sincos_t(th, &s, &c);
    write_obs<T, G>(A.obs + r * (2 * N + 4), lane, i, N, on, x, y, c, s, gx, gy);
  }
  if (i == 0) A.step[e] = 0;
}

// ---------------------------------------------------------------------------
// barrier_certificate
// ---------------------------------------------------------------------------
template <typename T> struct BarrierArgs {
  SimConst<T> C;
  int E, N;
  const T *px, *py, *uxn, *uyn;
  T *ux, *uy, *lambda;
  float *maxviol;
  uint8_t *infeasible;
  int32_t *qp_stats;
  unsigned long long *qp_fail;
};

template <typename T, int G>
__global__ __launch_bounds__(kBlock) void k_barrier(BarrierArgs<T> A) {
  __shared__ QPScratch<T, G> qs[kBlock / G];
  const int lane = threadIdx.x & 63;
  const int i = threadIdx.x & (G - 1);
  const int e = blockIdx.x * (kBlock / G) + threadIdx.x / G;
  if (e >= A.E) return;
  const int N = A.N;
  const bool on = i < N;
  const size_t r = (size_t)e * N + (on ? i : 0);
  const T px = A.px[r], py = A.py[r];
  T unx = A.uxn[r], uny = A.uyn[r];
  const ConstRef<T> K = kernarg_const<T>(offsetof(BarrierArgs<T>, C));
  preclip(*K.get(), unx, uny);
  T lox, hix, loy, hiy;
  wall_bounds(*K.get(), px, py, lox, hix, loy, hiy);
  QPScratch<T, G> *sh = &qs[threadIdx.x / G];
  T ux, uy;
  QPActive<T> act;
  const QPInfo info = qp_solve<T, G>(sh, K, A.C.qp_cap, lane, i, N, on, px, py, unx, uny, lox,
                                     hix, loy, hiy, ux, uy, &act);
  if (on) { A.ux[r] = ux; A.uy[r] = uy; }
  if (A.lambda) {
    // each lane writes the pairs it owns (i, i+k mod N); active rows come
    // from the register slots or, after a restart, from the LDS list
    const int P = N * (N - 1) / 2;
    T *lam = A.lambda + (size_t)e * P;
    for (int k = 1; k <= (N >> 1); ++k) {
      if (!on || (2 * k == N && i >= k)) continue;
      const int j = i + k >= N ? i + k - N : i + k;
      const int a = i < j ? i : j, b = i < j ? j : i;
      T val = T(0);
      if (act.rows_in_lds) {
        for (int s = 0; s < info.q; ++s)
          if (sh->act[s] == (a | (b << 8))) val = T(2) * sh->lam[s];
      } else {
        for (int s = 0; s < kQR; ++s)
          if (s < info.q && act.sa[s] == a && act.sb[s] == b) val = T(2) * act.slam[s];
      }
      lam[pair_index(a, b, N)] = val;
    }
  }
  if (A.maxviol) {
    const T mv = max_violation<T, G>(*K.get(), lane, i, N, on, px, py, ux, uy, lox, hix, loy,
                                      hiy);
    if (i == 0) A.maxviol[e] = (float)mv;
  }
  if (i == 0) {
    if (A.infeasible) A.infeasible[e] = (uint8_t)info.status;
    if (A.qp_stats) qp_stats_add(A.qp_stats + (size_t)e * kQPStats, info);
    qp_fail_count(A.qp_fail, info);
  }
}

template <typename K> static int blocks_for(int E, int G) {
  const int per = kBlock / G;
  return (E + per - 1) / per;
}

#define RS_DISPATCH_G(G, ...)                          \
  switch (G) {                                         \
    case 2: { constexpr int GG = 2; __VA_ARGS__; } break;   \
    case 4: { constexpr int GG = 4; __VA_ARGS__; } break;   \
    case 8: { constexpr int GG = 8; __VA_ARGS__; } break;   \
    default: { constexpr int GG = 16; __VA_ARGS__; } break; \
  }

static rs_status check_batch(const rs_batch *b, int dtype, bool need_state) {
  RS_CHECK_ARG(b != nullptr, "batch is NULL");
  RS_CHECK_ARG(b->num_envs >= 1, "num_envs must be >= 1 (got %d)", b->num_envs);
  RS_CHECK_ARG(b->robots >= 2 && b->robots <= RS_MAX_ROBOTS, "robots must be in 2..16 (got %d)",
               b->robots);
  if (need_state) {
    RS_CHECK_ARG(b->x && b->y && b->theta && b->goal_x && b->goal_y, "state pointer is NULL");
    RS_CHECK_ARG(b->step && b->episode, "step/episode pointer is NULL");
    const size_t a = dtype == RS_F64 ? 8 : 4;
    const void *ps[5] = {b->x, b->y, b->theta, b->goal_x, b->goal_y};
    for (const void *q : ps) RS_CHECK_ARG((uintptr_t)q % a == 0, "misaligned state array");
    RS_CHECK_ARG((uintptr_t)b->step % 4 == 0 && (uintptr_t)b->episode % 4 == 0,
                 "misaligned step/episode array");
  }
  return RS_OK;
}

static rs_status launch_status(const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error("%s launch failed: %s", what, hipGetErrorString(e));
    return RS_ERR_DEVICE;
  }
  return RS_OK;
}

template <typename T>
static rs_status do_env_step(rs_ctx *ctx, const rs_params *p, const rs_batch *b,
                             const uint8_t *actions, int64_t t_global, void *obs, void *reward,
                             uint8_t *done, float *maxviol, uint8_t *infeasible,
                             int32_t *qp_stats, hipStream_t st) {
  StepArgs<T> A;
  A.C = make_const<T>(*p);
  A.E = b->num_envs;
  A.N = b->robots;
  A.env_base = (uint32_t)b->env_id_base;
  A.t_global = (uint32_t)t_global;
  A.x = (T *)b->x; A.y = (T *)b->y; A.th = (T *)b->theta; A.gx = (T *)b->goal_x; A.gy = (T *)b->goal_y;
  A.step = b->step; A.episode = b->episode;
  A.actions = actions;
  A.obs = (T *)obs; A.reward = (T *)reward; A.done = done; A.infeasible = infeasible;
  A.maxviol = maxviol;
  A.qp_stats = qp_stats;
  A.qp_fail = ctx->qp_fail;
  const int G = pow2_group(A.N);
  if (p->scenario == RS_SCN_PREDATOR_PREY) {
    RS_DISPATCH_G(G, hipLaunchKernelGGL((k_env_step<T, GG, true>), dim3(blocks_for<T>(A.E, GG)),
                                        dim3(kBlock), 0, st, A));
  } else {
    RS_DISPATCH_G(G, hipLaunchKernelGGL((k_env_step<T, GG, false>), dim3(blocks_for<T>(A.E, GG)),
                                        dim3(kBlock), 0, st, A));
  }
  return launch_status("env_step");
}

template <typename T>
static rs_status do_env_steps(rs_ctx *ctx, const rs_params *p, const rs_batch *b, int32_t steps,
                              int64_t t_global0, void *reward, uint8_t *done, void *obs,
                              int32_t *qp_stats, hipStream_t st) {
  StepsArgs<T> A;
  A.C = make_const<T>(*p);
  A.E = b->num_envs;
  A.N = b->robots;
  A.steps = steps;
  A.env_base = (uint32_t)b->env_id_base;
  A.t0 = (uint32_t)t_global0;
  A.x = (T *)b->x; A.y = (T *)b->y; A.th = (T *)b->theta; A.gx = (T *)b->goal_x; A.gy = (T *)b->goal_y;
  A.step = b->step; A.episode = b->episode;
  A.reward = (T *)reward; A.done = done; A.obs = (T *)obs;
  A.qp_stats = qp_stats;
  A.qp_fail = ctx->qp_fail;
  const int G = pow2_group(A.N);
  if (p->scenario == RS_SCN_PREDATOR_PREY) {
    RS_DISPATCH_G(G, hipLaunchKernelGGL((k_env_steps<T, GG, true>), dim3(blocks_for<T>(A.E, GG)),
                                        dim3(kBlock), 0, st, A));
  } else {
    RS_DISPATCH_G(G, hipLaunchKernelGGL((k_env_steps<T, GG, false>), dim3(blocks_for<T>(A.E, GG)),
                                        dim3(kBlock), 0, st, A));
  }
  return launch_status("env_steps");
}

template <typename T>
static rs_status do_env_reset(const rs_params *p, const rs_batch *b, const uint8_t *mask,
                              void *obs, hipStream_t st) {
  ResetArgs<T> A;
  A.C = make_const<T>(*p);
  A.E = b->num_envs;
  A.N = b->robots;
  A.env_base = (uint32_t)b->env_id_base;
  A.x = (T *)b->x; A.y = (T *)b->y; A.th = (T *)b->theta; A.gx = (T *)b->goal_x; A.gy = (T *)b->goal_y;
  A.step = b->step; A.episode = b->episode;
  A.mask = mask;
  A.obs = (T *)obs;
  const int G = pow2_group(A.N);
  if (p->scenario == RS_SCN_PREDATOR_PREY) {
    RS_DISPATCH_G(G, hipLaunchKernelGGL((k_env_reset<T, GG, true>), dim3(blocks_for<T>(A.E, GG)),
                                        dim3(kBlock), 0, st, A));
  } else {
    RS_DISPATCH_G(G, hipLaunchKernelGGL((k_env_reset<T, GG, false>), dim3(blocks_for<T>(A.E, GG)),
                                        dim3(kBlock), 0, st, A));
  }
  return launch_status("env_reset");
}

template <typename T>
static rs_status do_barrier(rs_ctx *ctx, const rs_params *p, int E, int N, const void *px,
                            const void *py, const void *uxn, const void *uyn, void *ux, void *uy,
                            void *lambda, float *maxviol, uint8_t *infeasible, int32_t *qp_stats,
                            hipStream_t st) {
  BarrierArgs<T> A;
  A.C = make_const<T>(*p);
  A.E = E;
  A.N = N;
  A.px = (const T *)px; A.py = (const T *)py; A.uxn = (const T *)uxn; A.uyn = (const T *)uyn;
  A.ux = (T *)ux; A.uy = (T *)uy; A.lambda = (T *)lambda;
  A.maxviol = maxviol;
  A.infeasible = infeasible;
  A.qp_stats = qp_stats;
  A.qp_fail = ctx->qp_fail;
  const int G = pow2_group(N);
  RS_DISPATCH_G(G, hipLaunchKernelGGL((k_barrier<T, GG>), dim3(blocks_for<T>(E, GG)), dim3(kBlock),
                                      0, st, A));
  return launch_status("barrier_certificate");
}

}  // namespace rs

using namespace rs;

extern "C" {

void rs_params_default(rs_params *p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->x_min = -1.6; p->x_max = 1.6; p->y_min = -1.0; p->y_max = 1.0;
  p->dt = 0.033;
  p->proj_dist = 0.05;
  p->barrier_gain = 100.0;
  p->safety_radius = 0.17;
  p->boundary_gain_factor = 0.4;
  p->v_max = 0.2;
  p->action_speed = 0.2;
  p->kp = 1.0;
  p->wheel_radius = 0.016;
  p->base_length = 0.105;
  p->goal_radius = 0.05;
  p->reset_margin = 0.2;
  p->min_sep = 0.3;
  p->grid = 1e-4;
  p->max_steps = 500;
  p->controller = RS_CTRL_DISCRETE;
  p->dtype = RS_F32;
  p->qp_max_iters = 0;
  p->seed = 0;
  p->waypoint_step = 0.2;
  p->pos_gain = 0.8;
  p->ang_gain = 1.5707963267948966;
  p->action_noise = 0.0;
  p->prey_speed = 0.3;
  p->tag_radius = 0.25;
  p->tag_reward = 10.0;
  p->scenario = RS_SCN_NAVIGATION;
  p->pose_gain_rho = 0.8;
  p->pose_gain_alpha = 2.0;
  p->pose_gain_beta = 0.5;
}

rs_status rs_params_check(const rs_params *p) {
  clear_error();
  return check_params(p);
}

const char *rs_status_string(rs_status s) {
  switch (s) {
    case RS_OK: return "ok";
    case RS_ERR_INVALID_ARG: return "invalid argument";
    case RS_ERR_UNSUPPORTED: return "unsupported";
    case RS_ERR_OUT_OF_MEMORY: return "out of memory";
    case RS_ERR_DEVICE: return "device error";
    case RS_ERR_BUDGET: return "over budget";
    case RS_ERR_NOT_FOUND: return "not found";
  }
  return "unknown status";
}

const char *rs_last_error(void) { return g_error.c_str(); }

rs_status rs_create(int device, rs_ctx **out) {
  RS_CHECK_ARG(out != nullptr, "out is NULL");
  *out = nullptr;
  int count = 0;
  RS_CHECK_HIP(hipGetDeviceCount(&count));
  RS_CHECK_ARG(device >= 0 && device < count, "device %d out of range (%d devices)", device, count);
  RS_CHECK_HIP(hipSetDevice(device));
  hipDeviceProp_t prop;
  RS_CHECK_HIP(hipGetDeviceProperties(&prop, device));
  rs_ctx *c = new rs_ctx();
  c->device = device;
  c->num_cus = prop.multiProcessorCount;
  hipError_t he = hipMalloc((void **)&c->qp_fail, 2 * sizeof(unsigned long long));
  if (he == hipSuccess) he = hipMemset(c->qp_fail, 0, 2 * sizeof(unsigned long long));
  if (he == hipSuccess) he = rs::noalloc_setup(device);
  if (he != hipSuccess) {
    if (c->qp_fail) (void)hipFree(c->qp_fail);
    delete c;
    set_error("context allocation failed: %s", hipGetErrorString(he));
    return RS_ERR_DEVICE;
  }
  c->sched.block_threads = 256;
  for (int n = 0; n <= RS_MAX_ROBOTS; ++n) c->sched.lanes_per_env[n] = 0;
  *out = c;
  clear_error();
  return RS_OK;
}

rs_status rs_destroy(rs_ctx *ctx) {
  if (!ctx) return RS_OK;
  for (auto &kv : ctx->graphs) {
    (void)hipGraphExecDestroy(kv.second.exec);
    (void)hipGraphDestroy(kv.second.graph);
  }
  if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
  if (ctx->qp_fail) (void)hipFree(ctx->qp_fail);
  delete ctx;
  return RS_OK;
}

rs_status rs_qp_failures(rs_ctx *ctx, int64_t *infeasible, int64_t *capped, int32_t reset) {
  RS_CHECK_ARG(ctx != nullptr, "ctx is NULL");
  RS_CHECK_HIP(hipSetDevice(ctx->device));
  RS_CHECK_HIP(hipDeviceSynchronize());
  unsigned long long h[2] = {0, 0};
  RS_CHECK_HIP(hipMemcpy(h, ctx->qp_fail, sizeof(h), hipMemcpyDeviceToHost));
  if (infeasible) *infeasible = (int64_t)h[0];
  if (capped) *capped = (int64_t)h[1];
  if (reset) RS_CHECK_HIP(hipMemset(ctx->qp_fail, 0, sizeof(h)));
  return RS_OK;
}

rs_status env_step(rs_ctx *ctx, const rs_params *p, const rs_batch *b, const uint8_t *actions,
                   int64_t t_global, void *obs, void *reward, uint8_t *done, float *max_violation,
                   uint8_t *infeasible, int32_t *qp_stats, void *stream) {
  RS_CHECK_ARG(ctx != nullptr, "ctx is NULL");
  rs_status s = check_params(p);
  if (s != RS_OK) return s;
  s = check_batch(b, p->dtype, true);
  if (s != RS_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  if (p->dtype == RS_F64)
    return do_env_step<double>(ctx, p, b, actions, t_global, obs, reward, done, max_violation,
                               infeasible, qp_stats, st);
  return do_env_step<float>(ctx, p, b, actions, t_global, obs, reward, done, max_violation,
                            infeasible, qp_stats, st);
}

rs_status env_steps(rs_ctx *ctx, const rs_params *p, const rs_batch *b, int32_t steps,
                    int64_t t_global0, void *reward_out, uint8_t *done_out, void *obs_final,
                    int32_t *qp_stats, void *stream) {
  RS_CHECK_ARG(ctx != nullptr, "ctx is NULL");
  rs_status s = check_params(p);
  if (s != RS_OK) return s;
  s = check_batch(b, p->dtype, true);
  if (s != RS_OK) return s;
  RS_CHECK_ARG(steps >= 0, "steps must be >= 0 (got %d)", steps);
  RS_CHECK_ARG((int64_t)steps * b->num_envs <= INT32_MAX, "steps x num_envs must fit in int32");
  if (steps == 0) return RS_OK;
  hipStream_t st = (hipStream_t)stream;
  if (p->dtype == RS_F64)
    return do_env_steps<double>(ctx, p, b, steps, t_global0, reward_out, done_out, obs_final,
                                qp_stats, st);
  return do_env_steps<float>(ctx, p, b, steps, t_global0, reward_out, done_out, obs_final,
                             qp_stats, st);
}

rs_status env_reset(rs_ctx *ctx, const rs_params *p, const rs_batch *b, const uint8_t *mask,
                    void *obs, void *stream) {
  RS_CHECK_ARG(ctx != nullptr, "ctx is NULL");
  rs_status s = check_params(p);
  if (s != RS_OK) return s;
  s = check_batch(b, p->dtype, true);
  if (s != RS_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  if (p->dtype == RS_F64) return do_env_reset<double>(p, b, mask, obs, st);
  return do_env_reset<float>(p, b, mask, obs, st);
}

rs_status barrier_certificate(rs_ctx *ctx, const rs_params *p, int32_t num_envs, int32_t robots,
                              const void *px, const void *py, const void *ux_nom,
                              const void *uy_nom, void *ux, void *uy, void *lambda,
                              float *max_violation, uint8_t *infeasible, int32_t *qp_stats,
                              void *stream) {
  RS_CHECK_ARG(ctx != nullptr, "ctx is NULL");
  rs_status s = check_params(p);
  if (s != RS_OK) return s;
  RS_CHECK_ARG(num_envs >= 1, "num_envs must be >= 1 (got %d)", num_envs);
  RS_CHECK_ARG(robots >= 2 && robots <= RS_MAX_ROBOTS, "robots must be in 2..16 (got %d)", robots);
  RS_CHECK_ARG(px && py && ux_nom && uy_nom && ux && uy, "input/output pointer is NULL");
  const size_t a = p->dtype == RS_F64 ? 8 : 4;
  const void *ps[7] = {px, py, ux_nom, uy_nom, ux, uy, lambda};
  for (const void *q : ps) RS_CHECK_ARG((uintptr_t)q % a == 0, "misaligned array");
  hipStream_t st = (hipStream_t)stream;
  if (p->dtype == RS_F64)
    return do_barrier<double>(ctx, p, num_envs, robots, px, py, ux_nom, uy_nom, ux, uy, lambda,
                              max_violation, infeasible, qp_stats, st);
  return do_barrier<float>(ctx, p, num_envs, robots, px, py, ux_nom, uy_nom, ux, uy, lambda,
                           max_violation, infeasible, qp_stats, st);
}

}  // extern "C"
