// rs_mixed.hip -- persistent env_run kernel over mixed robot counts, plans,
// env_reset_mixed, env_run and the schedule autotuner.
//
// A plan sorts environments by lanes-per-env G (then by N) and cuts them into
// tiles of at most 64/G environments; each wavefront takes one tile and runs
// every step of the launch for it with the state in registers, so a launch
// covers envs of all sizes at once. G only changes how many envs share a
// wavefront: the arithmetic of an env is the same for every G (padding lanes
// add exact zeros), so results do not depend on the schedule.
#include "rs_run.hpp"
#include "rs_step.hpp"

#include <algorithm>
#include <chrono>
#include <cstddef>
#include <cstring>
#include <numeric>

namespace rs {

template <int G> constexpr int qp_bytes_per_wave() {
  return (64 / G) * (int)sizeof(QPScratch<float, G>);
}
constexpr int kMaxWaveLds =
    std::max(std::max(qp_bytes_per_wave<2>(), qp_bytes_per_wave<4>()),
             std::max(qp_bytes_per_wave<8>(), qp_bytes_per_wave<16>()));

// K: the launch's simulation constants in the kernel-argument segment, formed
// by the kernel (the segment pointer is only defined in a kernel's own body).
template <int G, bool PP>
__device__ __forceinline__ void run_tile(const RunArgs &A, ConstRef<float> K, char *wave_lds,
                                         int lane, int first, int count) {
  QPScratch<float, G> *sh = reinterpret_cast<QPScratch<float, G> *>(wave_lds) + lane / G;
  const int i = lane & (G - 1);
  const int grp = lane / G;
  if (grp >= count) return;  // whole group
  const int e = A.items[first + grp];
  const int N = A.nrob[e];
  const bool on = i < N;
  const size_t r = (size_t)A.offset[e] + (on ? i : 0);
  const uint32_t env_id = A.env_ids ? A.env_ids[e] : A.env_base + (uint32_t)e;
  const int qp_cap = A.qp_iters[N];

  float x = 0.f, y = 0.f, th = 0.f, gx = 0.f, gy = 0.f;
  int step = A.step[e], episode = A.episode[e];
  const bool consume = !A.reset_all && !A.reset_only && A.reset_mask && A.reset_mask[e];
  if (A.reset_all || (A.reset_only && A.reset_only[e]) || consume) {
    reset_env<float, G, PP>(K, env_id, (uint32_t)episode, i, N, lane, x, y, th, gx, gy);
    step = 0;
    if (consume && i == 0) A.reset_mask[e] = 0;
  } else if (on) {
    x = A.x[r]; y = A.y[r]; th = A.th[r]; gx = A.gx[r]; gy = A.gy[r];
  }
  int nsteps = A.steps;
  if (A.steps_per_env) nsteps = min(nsteps, A.steps_per_env[e]);
  const int64_t tb = A.t_start ? A.t_start[e] : (int64_t)A.t0;
  // complete the loads before the step loop (see k_rollout: the in-loop wait
  // would otherwise also wait for the loop's own stores)
  __builtin_amdgcn_s_waitcnt(0);
  float s, c;
  sincos_t(th, &s, &c);
  float rsum = 0.f;
  for (int k = 0; k < nsteps; ++k) {
    const auto *P = K.get();
    const int action = drawn_action(P->key0, P->key1, env_id, (uint32_t)(tb + k), i);
    const StepOut<float> so = env_step_group<float, G, PP>(K, qp_cap, sh, lane, i, N, on, env_id,
                                                       (uint32_t)(tb + k), action, x, y, th, c, s, gx, gy, step,
                                                       episode, false);
    rsum += so.reward;
    if (i == 0) {
      if (A.reward_out) A.reward_out[(size_t)k * A.E + e] = so.reward;
      if (A.done_out) A.done_out[(size_t)k * A.E + e] = so.done ? 1 : 0;
      if (A.qp_stats) qp_stats_add(A.qp_stats + (size_t)e * kQPStats, so.qp);
      qp_fail_count(A.qp_fail, so.qp);
    }
  }
  if (on) { A.x[r] = x; A.y[r] = y; A.th[r] = th; A.gx[r] = gx; A.gy[r] = gy; }
  if (A.obs_final)
    write_obs<float, G>(A.obs_final + A.obs_off[e] + (size_t)(on ? i : 0) * (2 * N + 4), lane, i,
                        N, on, x, y, c, s, gx, gy);
  if (i == 0) {
    A.step[e] = step;
    A.episode[e] = episode;
    if (A.reward_sum) A.reward_sum[e] += rsum;
    if (A.t_after) A.t_after[e] = tb + nsteps;
    if (A.steps_left_after && A.steps_per_env) A.steps_left_after[e] = A.steps_per_env[e] - nsteps;
  }
}

// PP: the Predator-Prey scenario (prey in the goal slots), a separate
// specialisation so that the Navigation kernel carries none of its code.
template <bool PP>
__global__ __launch_bounds__(256) void k_env_run(RunArgs A) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tile = blockIdx.x * (blockDim.x >> 6) + wave;
  if (tile >= A.num_tiles) return;
  if (A.num_tiles_dev && tile >= *A.num_tiles_dev) return;
  const int4 td = A.tiles[tile];
  char *mine = lds + (size_t)wave * kMaxWaveLds;
  const ConstRef<float> K = kernarg_const<float>(offsetof(RunArgs, C));
  switch (td.x) {
    case 2: run_tile<2, PP>(A, K, mine, lane, td.y, td.z); break;
    case 4: run_tile<4, PP>(A, K, mine, lane, td.y, td.z); break;
    case 8: run_tile<8, PP>(A, K, mine, lane, td.y, td.z); break;
    default: run_tile<16, PP>(A, K, mine, lane, td.y, td.z); break;
  }
}

hipError_t launch_run(const RunArgs &A, int block_threads, hipStream_t st) {
  const int waves = block_threads / 64;
  const int blocks = (A.num_tiles + waves - 1) / waves;
  if (blocks == 0) return hipSuccess;
  if (A.C.scenario == RS_SCN_PREDATOR_PREY)
    hipLaunchKernelGGL(k_env_run<true>, dim3(blocks), dim3(block_threads), waves * kMaxWaveLds, st,
                       A);
  else
    hipLaunchKernelGGL(k_env_run<false>, dim3(blocks), dim3(block_threads), waves * kMaxWaveLds, st,
                       A);
  return hipGetLastError();
}

int lanes_for(const rs_schedule &sched, int n) {
  const int g = sched.lanes_per_env[n];
  if (g >= n && g <= 16 && (g & (g - 1)) == 0 && g >= 2) return g;
  return pow2_group(n);
}

int envs_per_wave_for(const rs_schedule &sched, int n) {
  const int full = 64 / lanes_for(sched, n);
  const int c = sched.envs_per_wave[n];
  return (c >= 1 && c <= full) ? c : full;
}

void build_tiles(const std::vector<int32_t> &envs, const std::vector<int32_t> &nrob_of,
                 const rs_schedule &sched, std::vector<int32_t> &tiles,
                 std::vector<int32_t> &items) {
  // tiles hold envs of one (lanes, envs-per-wavefront) class, by robot count
  auto cls = [&](int32_t e) {
    const int n = nrob_of[e];
    return lanes_for(sched, n) * 128 + envs_per_wave_for(sched, n);
  };
  std::vector<int32_t> order(envs);
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    const int ca = cls(a), cb = cls(b);
    if (ca != cb) return ca < cb;
    return nrob_of[a] < nrob_of[b];
  });
  tiles.clear();
  items.clear();
  size_t k = 0;
  while (k < order.size()) {
    const int c0 = cls(order[k]);
    const int g = lanes_for(sched, nrob_of[order[k]]);
    const int cap = envs_per_wave_for(sched, nrob_of[order[k]]);
    const int first = (int)items.size();
    int count = 0;
    while (k < order.size() && count < cap && cls(order[k]) == c0) {
      items.push_back(order[k]);
      ++k;
      ++count;
    }
    tiles.push_back(g);
    tiles.push_back(first);
    tiles.push_back(count);
    tiles.push_back(0);
  }
}

static void default_schedule(rs_schedule &s) {
  std::memset(&s, 0, sizeof(s));
  s.block_threads = 256;
}

static rs_status plan_upload(rs_plan *pl) {
  std::vector<int32_t> envs(pl->num_envs);
  std::iota(envs.begin(), envs.end(), 0);
  std::vector<int32_t> tiles, items;
  build_tiles(envs, pl->robots_host, pl->sched, tiles, items);
  pl->num_tiles = (int32_t)(tiles.size() / 4);
  if (pl->tiles_dev) (void)hipFree(pl->tiles_dev);
  if (pl->items_dev) (void)hipFree(pl->items_dev);
  pl->tiles_dev = nullptr;
  pl->items_dev = nullptr;
  RS_CHECK_HIP(hipMalloc(&pl->tiles_dev, tiles.size() * sizeof(int32_t)));
  RS_CHECK_HIP(hipMalloc(&pl->items_dev, items.size() * sizeof(int32_t)));
  RS_CHECK_HIP(hipMemcpy(pl->tiles_dev, tiles.data(), tiles.size() * 4, hipMemcpyHostToDevice));
  RS_CHECK_HIP(hipMemcpy(pl->items_dev, items.data(), items.size() * 4, hipMemcpyHostToDevice));
  return RS_OK;
}

static RunArgs plan_args(const rs_plan *pl, const rs_params *p, const rs_batch *b) {
  RunArgs A;
  std::memset(&A, 0, sizeof(A));
  A.C = make_const<float>(*p);
  A.E = pl->num_envs;
  A.num_tiles = pl->num_tiles;
  A.env_base = (uint32_t)b->env_id_base;
  A.tiles = reinterpret_cast<const int4 *>(pl->tiles_dev);
  A.items = pl->items_dev;
  A.offset = pl->offset_dev;
  A.nrob = pl->nrob_dev;
  A.x = (float *)b->x; A.y = (float *)b->y; A.th = (float *)b->theta;
  A.gx = (float *)b->goal_x; A.gy = (float *)b->goal_y;
  A.step = b->step; A.episode = b->episode;
  A.qp_fail = pl->ctx->qp_fail;
  for (int n = 0; n <= RS_MAX_ROBOTS; ++n)
    A.qp_iters[n] = pl->sched.qp_iters[n] > 0 ? pl->sched.qp_iters[n] : p->qp_max_iters;
  return A;
}

static rs_status check_mixed(const rs_ctx *ctx, const rs_params *p, const rs_plan *plan,
                             const rs_batch *b) {
  RS_CHECK_ARG(ctx != nullptr && plan != nullptr && b != nullptr, "ctx/plan/batch is NULL");
  rs_status s = check_params(p);
  if (s != RS_OK) return s;
  RS_CHECK_ARG(p->dtype == RS_F32, "mixed batches run in FP32");
  RS_CHECK_ARG(action_driven(p->controller), "env_run draws actions: discrete, waypoint or pose controller");
  RS_CHECK_ARG(b->num_envs == plan->num_envs, "batch has %d envs, plan %d", b->num_envs,
               plan->num_envs);
  RS_CHECK_ARG(b->x && b->y && b->theta && b->goal_x && b->goal_y && b->step && b->episode,
               "state pointer is NULL");
  return RS_OK;
}

}  // namespace rs

using namespace rs;

extern "C" {

rs_status rs_plan_create(rs_ctx *ctx, int32_t num_envs, const int32_t *robots_per_env,
                         const rs_schedule *schedule, rs_plan **out) {
  RS_CHECK_ARG(ctx != nullptr && out != nullptr, "ctx/out is NULL");
  RS_CHECK_ARG(num_envs >= 1 && robots_per_env != nullptr, "need num_envs >= 1 and counts");
  *out = nullptr;
  rs_plan *pl = new rs_plan();
  pl->ctx = ctx;
  pl->num_envs = num_envs;
  pl->robots_host.assign(robots_per_env, robots_per_env + num_envs);
  pl->offset_host.resize(num_envs + 1);
  pl->obs_offset_host.resize(num_envs + 1);
  int64_t acc = 0, oacc = 0;
  for (int32_t e = 0; e < num_envs; ++e) {
    const int n = robots_per_env[e];
    if (n < 2 || n > RS_MAX_ROBOTS) {
      delete pl;
      set_error("robots_per_env[%d] = %d outside 2..16", e, n);
      return RS_ERR_INVALID_ARG;
    }
    pl->offset_host[e] = (int32_t)acc;
    pl->obs_offset_host[e] = oacc;
    acc += n;
    oacc += (int64_t)n * (2 * n + 4);
  }
  if (acc > INT32_MAX) {
    delete pl;
    set_error("too many robots in one plan");
    return RS_ERR_INVALID_ARG;
  }
  pl->offset_host[num_envs] = (int32_t)acc;
  pl->obs_offset_host[num_envs] = oacc;
  pl->total_robots = acc;
  pl->sched = schedule ? *schedule : ctx->sched;
  if (pl->sched.block_threads <= 0) pl->sched.block_threads = 256;
  if (pl->sched.block_threads % 64 != 0 || pl->sched.block_threads > 256) {
    delete pl;
    set_error("block_threads must be a multiple of 64 in 64..256");
    return RS_ERR_INVALID_ARG;
  }
  pl->block_threads = pl->sched.block_threads;
  auto fail = [&](hipError_t e) {
    set_error("plan allocation failed: %s", hipGetErrorString(e));
    rs_plan_destroy(pl);
    return RS_ERR_DEVICE;
  };
  hipError_t he;
  if ((he = hipMalloc(&pl->offset_dev, (num_envs + 1) * sizeof(int32_t))) != hipSuccess) return fail(he);
  if ((he = hipMalloc(&pl->nrob_dev, num_envs * sizeof(int32_t))) != hipSuccess) return fail(he);
  if ((he = hipMalloc(&pl->obs_off_dev, (num_envs + 1) * sizeof(int64_t))) != hipSuccess) return fail(he);
  if ((he = hipMemcpy(pl->offset_dev, pl->offset_host.data(), (num_envs + 1) * 4,
                      hipMemcpyHostToDevice)) != hipSuccess ||
      (he = hipMemcpy(pl->nrob_dev, pl->robots_host.data(), num_envs * 4,
                      hipMemcpyHostToDevice)) != hipSuccess ||
      (he = hipMemcpy(pl->obs_off_dev, pl->obs_offset_host.data(), (num_envs + 1) * 8,
                      hipMemcpyHostToDevice)) != hipSuccess)
    return fail(he);
  rs_status s = plan_upload(pl);
  if (s != RS_OK) {
    rs_plan_destroy(pl);
    return s;
  }
  *out = pl;
  return RS_OK;
}

rs_status rs_plan_destroy(rs_plan *pl) {
  if (!pl) return RS_OK;
  if (pl->offset_dev) (void)hipFree(pl->offset_dev);
  if (pl->nrob_dev) (void)hipFree(pl->nrob_dev);
  if (pl->obs_off_dev) (void)hipFree(pl->obs_off_dev);
  if (pl->tiles_dev) (void)hipFree(pl->tiles_dev);
  if (pl->items_dev) (void)hipFree(pl->items_dev);
  delete pl;
  return RS_OK;
}

int64_t rs_plan_total_robots(const rs_plan *plan) { return plan ? plan->total_robots : -1; }
const int32_t *rs_plan_robot_offset(const rs_plan *plan) { return plan ? plan->offset_dev : nullptr; }
int64_t rs_plan_obs_offset(const rs_plan *plan, int32_t env) {
  if (!plan || env < 0 || env > plan->num_envs) return -1;
  return plan->obs_offset_host[env];
}

rs_status env_reset_mixed(rs_ctx *ctx, const rs_params *p, const rs_plan *plan, const rs_batch *b,
                          const uint8_t *mask, void *stream) {
  rs_status s = check_mixed(ctx, p, plan, b);
  if (s != RS_OK) return s;
  RunArgs A = plan_args(plan, p, b);
  A.steps = 0;
  // the caller's mask is only read (no flag is consumed), so nothing is
  // allocated or copied
  A.reset_only = mask;
  A.reset_all = mask ? 0 : 1;
  hipError_t he = launch_run(A, plan->block_threads, (hipStream_t)stream);
  if (he != hipSuccess) {
    set_error("env_reset_mixed launch failed: %s", hipGetErrorString(he));
    return RS_ERR_DEVICE;
  }
  return RS_OK;
}

}  // extern "C"

namespace rs {

// env_run with the failure counters it adds to (the context's, or the
// autotuner's own).
static rs_status run_plan(rs_ctx *ctx, const rs_params *p, const rs_plan *plan, const rs_batch *b,
                          int32_t steps, const int64_t *t_start, int64_t t_global0,
                          const int32_t *steps_per_env, float *reward_out, uint8_t *done_out,
                          float *reward_sum, float *obs_final, int32_t *qp_stats,
                          unsigned long long *fail, void *stream) {
  rs_status s = check_mixed(ctx, p, plan, b);
  if (s != RS_OK) return s;
  RS_CHECK_ARG(steps >= 0, "steps must be >= 0");
  RunArgs A = plan_args(plan, p, b);
  A.qp_fail = fail;
  A.steps = steps;
  A.t0 = (uint32_t)t_global0;
  A.t_start = t_start;
  A.steps_per_env = steps_per_env;
  A.reward_out = reward_out;
  A.done_out = done_out;
  A.reward_sum = reward_sum;
  A.obs_final = obs_final;
  A.obs_off = plan->obs_off_dev;
  A.qp_stats = qp_stats;
  hipError_t he = launch_run(A, plan->block_threads, (hipStream_t)stream);
  if (he != hipSuccess) {
    set_error("env_run launch failed: %s", hipGetErrorString(he));
    return RS_ERR_DEVICE;
  }
  return RS_OK;
}

}  // namespace rs

extern "C" {

rs_status env_run(rs_ctx *ctx, const rs_params *p, const rs_plan *plan, const rs_batch *b,
                  int32_t steps, const int64_t *t_start, int64_t t_global0,
                  const int32_t *steps_per_env, float *reward_out, uint8_t *done_out,
                  float *reward_sum, float *obs_final, int32_t *qp_stats, void *stream) {
  if (ctx == nullptr) {
    set_error("ctx/plan/batch is NULL");
    return RS_ERR_INVALID_ARG;
  }
  return run_plan(ctx, p, plan, b, steps, t_start, t_global0, steps_per_env, reward_out,
                  done_out, reward_sum, obs_final, qp_stats, ctx->qp_fail, stream);
}

rs_status rs_get_schedule(rs_ctx *ctx, rs_schedule *out) {
  RS_CHECK_ARG(ctx != nullptr && out != nullptr, "ctx/out is NULL");
  *out = ctx->sched;
  return RS_OK;
}

rs_status rs_set_schedule(rs_ctx *ctx, const rs_schedule *sc) {
  RS_CHECK_ARG(ctx != nullptr && sc != nullptr, "ctx/schedule is NULL");
  RS_CHECK_ARG(sc->block_threads >= 0 && sc->block_threads <= 256 && sc->block_threads % 64 == 0,
               "block_threads %d: 0 or a multiple of 64 up to 256", sc->block_threads);
  for (int n = 2; n <= RS_MAX_ROBOTS; ++n) {
    const int g = sc->lanes_per_env[n];
    RS_CHECK_ARG(g == 0 || (g >= n && g <= RS_MAX_ROBOTS && (g & (g - 1)) == 0),
                 "lanes_per_env[%d] = %d: 0 or a power of two in %d..16", n, g, n);
    const int lanes = g ? g : pow2_group(n);
    RS_CHECK_ARG(sc->envs_per_wave[n] >= 0 && sc->envs_per_wave[n] <= 64 / lanes,
                 "envs_per_wave[%d] = %d: 0..%d", n, sc->envs_per_wave[n], 64 / lanes);
    RS_CHECK_ARG(sc->qp_iters[n] >= 0, "qp_iters[%d] = %d < 0", n, sc->qp_iters[n]);
  }
  ctx->sched = *sc;
  return RS_OK;
}

// ---------------------------------------------------------------------------
// Autotuner
// ---------------------------------------------------------------------------
}  // extern "C"

namespace rs {

// Schedule search over env_run launches of `steps` steps on a pristine state
// (the caller's batch `src`, or with src NULL the synthetic workload: the
// reset sampler for every other env, a tight cluster of pitch 0.2 m around the
// arena centre, where the certificate binds, for the rest). A candidate passes
// when no certificate of its first run stopped at the iteration cap (every
// step then reached the exact minimiser) and its final positions match the
// default-schedule, widest-cap reference within steps * dt * tol; it is kept
// when it is also at least 2% faster than the best so far.
static rs_status autotune_impl(rs_ctx *ctx, const rs_params *p, const std::vector<int32_t> &counts,
                               const rs_batch *src, int32_t steps, double tol, rs_schedule *out) {
  const int32_t E = (int32_t)counts.size();
  std::vector<int32_t> sizes;
  for (int32_t n : counts)
    if (std::find(sizes.begin(), sizes.end(), n) == sizes.end()) sizes.push_back(n);
  std::sort(sizes.begin(), sizes.end());
  size_t R = 0;
  for (int32_t e = 0; e < E; ++e) R += (size_t)counts[e];

  hipStream_t st;
  RS_CHECK_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  hipEvent_t ev0, ev1;
  (void)hipEventCreate(&ev0);
  (void)hipEventCreate(&ev1);
  float *dbuf = nullptr;
  int32_t *ibuf = nullptr;
  rs_status result = RS_OK;
  // dbuf: working state [5R] then the pristine copy [5R]; ibuf: working
  // step/episode [2E], pristine [2E], then the tuner's failure counters
  if (hipMalloc(&dbuf, 10 * R * sizeof(float)) != hipSuccess ||
      hipMalloc(&ibuf, (4 * (size_t)E + 4) * sizeof(int32_t)) != hipSuccess) {
    set_error("autotune allocation failed");
    result = RS_ERR_OUT_OF_MEMORY;
  }
  rs_batch b;
  std::memset(&b, 0, sizeof(b));
  float *init = dbuf ? dbuf + 5 * R : nullptr;
  int32_t *init_i = ibuf ? ibuf + 2 * E : nullptr;
  std::vector<float> rx(R), ry(R), cx(R), cy(R);
  auto restore = [&]() {
    (void)hipMemcpyAsync(dbuf, init, 5 * R * 4, hipMemcpyDeviceToDevice, st);
    (void)hipMemcpyAsync(ibuf, init_i, 2 * (size_t)E * sizeof(int32_t), hipMemcpyDeviceToDevice, st);
  };
  unsigned long long *fail = ibuf ? reinterpret_cast<unsigned long long *>(ibuf + 4 * E) : nullptr;
  auto measure = [&](const rs_schedule &sched, bool check, float &ms) -> bool {
    rs_plan *pl = nullptr;
    if (rs_plan_create(ctx, E, counts.data(), &sched, &pl) != RS_OK) return false;
    ms = 1e30f;
    bool ok = true;
    for (int rep = 0; rep < 3 && ok; ++rep) {
      restore();
      if (rep == 0) (void)hipMemsetAsync(fail, 0, 2 * sizeof(unsigned long long), st);
      (void)hipEventRecord(ev0, st);
      if (run_plan(ctx, p, pl, &b, steps, nullptr, 0, nullptr, nullptr, nullptr, nullptr, nullptr,
                   nullptr, fail, st) != RS_OK) {
        ok = false;
        break;
      }
      (void)hipEventRecord(ev1, st);
      (void)hipEventSynchronize(ev1);
      float t = 0.f;
      (void)hipEventElapsedTime(&t, ev0, ev1);
      ms = std::min(ms, t);
      if (rep == 0) {
        unsigned long long h[2] = {0, 0};
        (void)hipMemcpy(h, fail, sizeof(h), hipMemcpyDeviceToHost);
        ok = h[1] == 0;
      }
      if (ok && rep == 0 && check) {
        (void)hipMemcpy(cx.data(), b.x, R * 4, hipMemcpyDeviceToHost);
        (void)hipMemcpy(cy.data(), b.y, R * 4, hipMemcpyDeviceToHost);
        const double bound = steps * p->dt * tol;
        double worst = 0.0;
        for (size_t q = 0; q < R; ++q)
          worst = std::max(worst, (double)std::max(std::fabs(cx[q] - rx[q]), std::fabs(cy[q] - ry[q])));
        ok = worst <= bound;
      }
    }
    rs_plan_destroy(pl);
    return ok;
  };

  rs_schedule best;
  default_schedule(best);
  if (result == RS_OK) {
    float *f = dbuf;
    b.num_envs = E;
    b.robots = 0;
    b.x = f; b.y = f + R; b.theta = f + 2 * R; b.goal_x = f + 3 * R; b.goal_y = f + 4 * R;
    b.step = ibuf;
    b.episode = ibuf + E;
    if (src) {
      const void *fs[5] = {src->x, src->y, src->theta, src->goal_x, src->goal_y};
      for (int k = 0; k < 5; ++k)
        (void)hipMemcpyAsync(init + k * R, fs[k], R * 4, hipMemcpyDeviceToDevice, st);
      (void)hipMemcpyAsync(init_i, src->step, (size_t)E * 4, hipMemcpyDeviceToDevice, st);
      (void)hipMemcpyAsync(init_i + E, src->episode, (size_t)E * 4, hipMemcpyDeviceToDevice, st);
      (void)hipStreamSynchronize(st);
    } else {
      rs_plan *ref_plan = nullptr;
      result = rs_plan_create(ctx, E, counts.data(), &best, &ref_plan);
      if (result == RS_OK) {
        (void)hipMemsetAsync(ibuf, 0, 2 * (size_t)E * sizeof(int32_t), st);
        result = env_reset_mixed(ctx, p, ref_plan, &b, nullptr, st);
        (void)hipStreamSynchronize(st);
        std::vector<float> hx(R), hy(R);
        (void)hipMemcpy(hx.data(), b.x, R * 4, hipMemcpyDeviceToHost);
        (void)hipMemcpy(hy.data(), b.y, R * 4, hipMemcpyDeviceToHost);
        size_t off = 0;
        for (int32_t e = 0; e < E; ++e) {
          const int n = counts[e];
          if (e & 1) {
            const int side = (int)std::ceil(std::sqrt((double)n));
            for (int i = 0; i < n; ++i) {
              hx[off + i] = -0.3f + 0.2f * (float)(i % side);
              hy[off + i] = -0.3f + 0.2f * (float)(i / side);
            }
          }
          off += (size_t)n;
        }
        (void)hipMemcpy(b.x, hx.data(), R * 4, hipMemcpyHostToDevice);
        (void)hipMemcpy(b.y, hy.data(), R * 4, hipMemcpyHostToDevice);
        (void)hipMemcpy(init, dbuf, 5 * R * 4, hipMemcpyDeviceToDevice);
        (void)hipMemcpy(init_i, ibuf, 2 * (size_t)E * 4, hipMemcpyDeviceToDevice);
        rs_plan_destroy(ref_plan);
      }
    }
    // reference positions: the default schedule with the widest iteration cap
    rs_schedule ref = best;
    for (int32_t n : sizes) ref.qp_iters[n] = 8 * n + 32;
    float ref_ms = 0.f;
    if (result == RS_OK && measure(ref, false, ref_ms)) {
      (void)hipMemcpy(rx.data(), b.x, R * 4, hipMemcpyDeviceToHost);
      (void)hipMemcpy(ry.data(), b.y, R * 4, hipMemcpyDeviceToHost);
    } else if (result == RS_OK) {
      set_error("autotune: the reference run failed or a certificate reached the widest "
                "iteration cap (8N+32)");
      result = RS_ERR_DEVICE;
    }
    // coordinate descent from the default schedule: block size, then per
    // size lanes per env, envs per wavefront and the iteration cap
    float best_ms = 0.f;
    if (result == RS_OK && !measure(best, true, best_ms)) result = RS_ERR_DEVICE;
    auto consider = [&](const rs_schedule &cand) {
      float ms = 0.f;
      if (measure(cand, true, ms) && ms < 0.98f * best_ms) {
        best = cand;
        best_ms = ms;
      }
    };
    if (result == RS_OK) {
      for (int blk = 64; blk <= 256; blk *= 2) {
        if (blk == best.block_threads) continue;
        rs_schedule c = best;
        c.block_threads = blk;
        consider(c);
      }
      for (int32_t n : sizes) {
        const int g0 = pow2_group(n);
        if (2 * g0 <= 16) {
          rs_schedule c = best;
          c.lanes_per_env[n] = 2 * g0;
          consider(c);
        }
        const int full = 64 / lanes_for(best, n);
        for (int div = 2; div <= 8; div *= 2) {
          if (full / div < 1) break;
          rs_schedule c = best;
          c.envs_per_wave[n] = full / div;
          consider(c);
        }
        const int caps[2] = {2 * n + 4, 4 * n + 8};
        for (int ci = 0; ci < 2; ++ci) {
          rs_schedule c = best;
          c.qp_iters[n] = caps[ci];
          consider(c);
        }
      }
      // report the effective values for the tuned sizes
      for (int32_t n : sizes) {
        best.lanes_per_env[n] = lanes_for(best, n);
        best.envs_per_wave[n] = envs_per_wave_for(best, n);
        if (best.qp_iters[n] <= 0) best.qp_iters[n] = 8 * n + 32;
      }
      ctx->sched = best;
    }
  }
  if (dbuf) (void)hipFree(dbuf);
  if (ibuf) (void)hipFree(ibuf);
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);
  (void)hipStreamDestroy(st);
  if (out) *out = ctx->sched;
  return result;
}

}  // namespace rs

extern "C" {

rs_status rs_autotune(rs_ctx *ctx, const rs_params *p, const int32_t *robots, int32_t count,
                      int32_t envs, int32_t steps, double tol, rs_schedule *out) {
  RS_CHECK_ARG(ctx != nullptr && robots != nullptr && count >= 1, "ctx/robots invalid");
  RS_CHECK_ARG(envs >= 1 && steps >= 1 && tol > 0, "envs, steps, tol must be > 0");
  rs_status s = check_params(p);
  if (s != RS_OK) return s;
  RS_CHECK_ARG(p->dtype == RS_F32 && action_driven(p->controller),
               "autotune runs the FP32 path of an action-driven controller");
  for (int32_t k = 0; k < count; ++k)
    RS_CHECK_ARG(robots[k] >= 2 && robots[k] <= RS_MAX_ROBOTS, "robots[%d] = %d outside 2..16",
                 k, robots[k]);
  // the mixed workload: `envs` envs of every listed size, interleaved
  const int64_t E64 = (int64_t)envs * count;
  RS_CHECK_ARG(E64 < (1 << 24), "envs * count too large for the autotuner");
  std::vector<int32_t> counts((size_t)E64);
  for (int64_t e = 0; e < E64; ++e) counts[(size_t)e] = robots[e % count];
  return autotune_impl(ctx, p, counts, nullptr, steps, tol, out);
}

rs_status rs_autotune_batch(rs_ctx *ctx, const rs_params *p, const rs_plan *plan,
                            const rs_batch *b, int32_t steps, double tol, rs_schedule *out) {
  rs_status s = check_mixed(ctx, p, plan, b);
  if (s != RS_OK) return s;
  RS_CHECK_ARG(steps >= 1 && tol > 0, "steps and tol must be > 0");
  return autotune_impl(ctx, p, plan->robots_host, b, steps, tol, out);
}

}  // extern "C"
