// rs_noalloc.hip -- env_run_noalloc: the env_run launch for callers that
// cannot allocate device memory (code under HIP graph capture, serving loops
// and harnesses that forbid hipMalloc).
//
// env_run reads its work list (robot and observation offsets, the env order
// and the wavefront tiles) from memory that rs_plan_create allocates. Here a
// one-workgroup kernel builds the same kind of list on the stream, from a
// device array of robot counts, into one file-scope device array of fixed
// size; the persistent kernel of env_run then runs from it. Every call on a
// device shares that device's array.
#include "rs_run.hpp"

#include <algorithm>
#include <cstring>
#include <mutex>

namespace rs {

namespace {

constexpr size_t al256(size_t b) { return (b + 255) & ~size_t(255); }
constexpr int kMaxEnvs = RS_NOALLOC_MAX_ENVS;
constexpr int kMaxTiles = kMaxEnvs + RS_MAX_ROBOTS;  // at most E + one partial tile per count
// byte layout of the array
constexpr size_t kHdr = 0;                                      // int32 {tiles, bad envs}
constexpr size_t kOffset = 256;                                 // int32 [E+1] robot offsets
constexpr size_t kObsOff = kOffset + al256(4 * (size_t)(kMaxEnvs + 1));  // int64 [E+1]
constexpr size_t kItems = kObsOff + al256(8 * (size_t)(kMaxEnvs + 1));   // int32 [E]
constexpr size_t kTiles = kItems + al256(4 * (size_t)kMaxEnvs);          // int4 [tiles]
constexpr size_t kScratchBytes = kTiles + al256(16 * (size_t)kMaxTiles);

// Host code may not use this name as a device address: the address of each
// device's copy comes from hipGetSymbolAddress (noalloc_setup).
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static_assert(kScratchBytes == RS_NOALLOC_SCRATCH_BYTES, "header states the array size");

constexpr int kDevices = 64;
std::mutex g_mu;
unsigned char *g_scratch[kDevices] = {};

constexpr int kPlanThreads = 1024;
constexpr int kPlanWaves = kPlanThreads / 64;

struct PlanArgs {
  const int32_t *nrob;  // [E] robot counts (device)
  int32_t *bad_out;     // [1] (may be NULL)
  unsigned char *s;     // this device's array
  int E;
  int32_t lanes[RS_MAX_ROBOTS + 1];  // lanes per env, by robot count
  int32_t epw[RS_MAX_ROBOTS + 1];    // envs per wavefront tile, by robot count
};

template <typename T> __device__ T wave_incl_scan(T v, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const T u = __shfl_up(v, d, 64);
    if (lane >= d) v += u;
  }
  return v;
}

template <typename T> __device__ T wave_sum(T v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// Work list of E envs: robot offsets (prefix sum of the counts in env order),
// observation offsets (prefix sum of N (2N + 4)), env indices grouped by robot
// count (env order within a count) and, per count, tiles of envs-per-wavefront
// envs. Wavefront w takes the envs [w seg, (w+1) seg) in rounds of 64, one
// env per lane, in two passes: totals per wavefront, then positions.
__global__ __launch_bounds__(kPlanThreads) void k_noalloc_plan(PlanArgs P) {
  __shared__ int32_t w_rob[kPlanWaves];
  __shared__ int64_t w_obs[kPlanWaves];
  __shared__ int32_t w_cnt[kPlanWaves][RS_MAX_ROBOTS + 1];  // per count, then start position
  __shared__ int32_t w_bad[kPlanWaves];
  __shared__ int32_t total[RS_MAX_ROBOTS + 1], item_base[RS_MAX_ROBOTS + 1],
      tile_base[RS_MAX_ROBOTS + 1];
  __shared__ int32_t bad;
  int32_t *hdr = reinterpret_cast<int32_t *>(P.s + kHdr);
  int32_t *offset = reinterpret_cast<int32_t *>(P.s + kOffset);
  int64_t *obs_off = reinterpret_cast<int64_t *>(P.s + kObsOff);
  int32_t *items = reinterpret_cast<int32_t *>(P.s + kItems);
  int4 *tiles = reinterpret_cast<int4 *>(P.s + kTiles);

  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int seg = ((P.E + kPlanWaves - 1) / kPlanWaves + 63) & ~63;
  const int lo = min(P.E, w * seg), hi = min(P.E, lo + seg);

  // pass 1: per-wavefront robots, observation floats, counts and bad envs
  int32_t r = 0, nbad = 0, cnt = 0;  // cnt: lane m counts envs of m robots
  int64_t o = 0;
  for (int base = lo; base < hi; base += 64) {
    const int e = base + lane;
    const int n = e < hi ? P.nrob[e] : 0;
    const bool ok = n >= 2 && n <= RS_MAX_ROBOTS;
    if (e < hi && !ok) ++nbad;
    const int nn = ok ? n : 0;
    r += nn;
    o += (int64_t)nn * (2 * nn + 4);
#pragma unroll
    for (int m = 2; m <= RS_MAX_ROBOTS; ++m) {
      const int c = __popcll(__ballot(nn == m));
      if (lane == m) cnt += c;
    }
  }
  r = wave_sum(r);
  o = wave_sum(o);
  nbad = wave_sum(nbad);
  if (lane == 0) {
    w_rob[w] = r;
    w_obs[w] = o;
    w_bad[w] = nbad;
  }
  if (lane <= RS_MAX_ROBOTS) w_cnt[w][lane] = cnt;
  __syncthreads();

  // bases across wavefronts, counts and tiles (one thread: 16 x 15 values)
  if (threadIdx.x == 0) {
    int32_t nb = 0;
    for (int k = 0; k < kPlanWaves; ++k) nb += w_bad[k];
    bad = nb;
    if (P.bad_out) P.bad_out[0] = nb;
    if (nb) {
      hdr[0] = 0;
      hdr[1] = nb;
    } else {
      int32_t ra = 0;
      int64_t oa = 0;
      for (int k = 0; k < kPlanWaves; ++k) {
        const int32_t rk = w_rob[k];
        const int64_t okk = w_obs[k];
        w_rob[k] = ra;
        w_obs[k] = oa;
        ra += rk;
        oa += okk;
      }
      offset[P.E] = ra;
      obs_off[P.E] = oa;
      int32_t ib = 0, tb = 0;
      for (int m = 2; m <= RS_MAX_ROBOTS; ++m) {
        int32_t c = 0;
        for (int k = 0; k < kPlanWaves; ++k) {
          const int32_t ck = w_cnt[k][m];
          w_cnt[k][m] = ib + c;
          c += ck;
        }
        total[m] = c;
        item_base[m] = ib;
        tile_base[m] = tb;
        ib += c;
        tb += (c + P.epw[m] - 1) / P.epw[m];
      }
      hdr[0] = tb;
      hdr[1] = 0;
    }
  }
  __syncthreads();
  if (bad) return;

  // pass 2: offsets in env order, env indices by count (stable)
  int32_t rb = w_rob[w];
  int64_t ob = w_obs[w];
  int32_t pos = (lane >= 2 && lane <= RS_MAX_ROBOTS) ? w_cnt[w][lane] : 0;
  const uint64_t below = (1ull << lane) - 1ull;
  for (int base = lo; base < hi; base += 64) {
    const int e = base + lane;
    const int n = e < hi ? P.nrob[e] : 0;
    const int64_t on = (int64_t)n * (2 * n + 4);
    const int32_t ri = wave_incl_scan<int32_t>(n, lane);
    const int64_t oi = wave_incl_scan<int64_t>(on, lane);
    int32_t at = 0;
#pragma unroll
    for (int m = 2; m <= RS_MAX_ROBOTS; ++m) {
      const uint64_t bm = __ballot(n == m);
      const int32_t pm = __builtin_amdgcn_readlane(pos, m);
      if (n == m) at = pm + __popcll(bm & below);
      if (lane == m) pos += __popcll(bm);
    }
    if (e < hi) {
      offset[e] = rb + ri - n;
      obs_off[e] = ob + oi - on;
      items[at] = e;
    }
    rb += __shfl(ri, 63, 64);
    ob += __shfl(oi, 63, 64);
  }

  // tiles, count after count
  for (int m = 2; m <= RS_MAX_ROBOTS; ++m) {
    const int c = total[m], cap = P.epw[m];
    const int nt = (c + cap - 1) / cap;
    for (int k = threadIdx.x; k < nt; k += kPlanThreads)
      tiles[tile_base[m] + k] = make_int4(P.lanes[m], item_base[m] + k * cap, min(cap, c - k * cap), 0);
  }
}

}  // namespace

hipError_t noalloc_setup(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (device < 0 || device >= kDevices) return hipErrorInvalidDevice;
  if (g_scratch[device]) return hipSuccess;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch[device] = static_cast<unsigned char *>(p);
  return hipSuccess;
}

static unsigned char *noalloc_scratch(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  return (device >= 0 && device < kDevices) ? g_scratch[device] : nullptr;
}

}  // namespace rs

using namespace rs;

extern "C" {

rs_status env_run_noalloc(rs_ctx *ctx, const rs_params *p, const int32_t *robots_per_env,
                          const rs_batch *b, int32_t steps, const int64_t *t_start,
                          int64_t t_global0, const int32_t *steps_per_env, float *reward_out,
                          uint8_t *done_out, float *reward_sum, float *obs_final,
                          int32_t *qp_stats, int32_t *bad_envs, void *stream) {
  RS_CHECK_ARG(ctx != nullptr && b != nullptr && robots_per_env != nullptr,
               "ctx/batch/robots_per_env is NULL");
  rs_status s = check_params(p);
  if (s != RS_OK) return s;
  RS_CHECK_ARG(p->dtype == RS_F32, "mixed batches run in FP32");
  RS_CHECK_ARG(action_driven(p->controller), "env_run draws actions: discrete, waypoint or pose controller");
  RS_CHECK_ARG(b->num_envs >= 1 && b->num_envs <= kMaxEnvs,
               "num_envs %d outside 1..%d (the fixed work-list size of env_run_noalloc)",
               b->num_envs, kMaxEnvs);
  RS_CHECK_ARG(b->x && b->y && b->theta && b->goal_x && b->goal_y && b->step && b->episode,
               "state pointer is NULL");
  RS_CHECK_ARG(steps >= 0, "steps must be >= 0");
  unsigned char *sc = noalloc_scratch(ctx->device);
  if (sc == nullptr) {
    set_error("env_run_noalloc: no work-list array for device %d", ctx->device);
    return RS_ERR_DEVICE;
  }
  const rs_schedule &sched = ctx->sched;
  const int block_threads = sched.block_threads > 0 ? sched.block_threads : 256;
  RS_CHECK_ARG(block_threads % 64 == 0 && block_threads <= 256,
               "block_threads must be a multiple of 64 in 64..256");
  const int E = b->num_envs;

  PlanArgs P;
  std::memset(&P, 0, sizeof(P));
  P.nrob = robots_per_env;
  P.bad_out = bad_envs;
  P.s = sc;
  P.E = E;
  int epw_min = 64;
  for (int n = 2; n <= RS_MAX_ROBOTS; ++n) {
    P.lanes[n] = lanes_for(sched, n);
    P.epw[n] = envs_per_wave_for(sched, n);
    epw_min = std::min(epw_min, (int)P.epw[n]);
  }
  const hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_noalloc_plan, dim3(1), dim3(kPlanThreads), 0, st, P);
  hipError_t he = hipGetLastError();
  if (he != hipSuccess) {
    set_error("env_run_noalloc work-list launch failed: %s", hipGetErrorString(he));
    return RS_ERR_DEVICE;
  }

  RunArgs A;
  std::memset(&A, 0, sizeof(A));
  A.C = make_const<float>(*p);
  A.E = E;
  // grid for the most tiles any counts can need; the kernel reads the real
  // number from the work list
  A.num_tiles = (E + epw_min - 1) / epw_min + (RS_MAX_ROBOTS - 1);
  A.num_tiles_dev = reinterpret_cast<const int32_t *>(sc + kHdr);
  A.env_base = (uint32_t)b->env_id_base;
  A.tiles = reinterpret_cast<const int4 *>(sc + kTiles);
  A.items = reinterpret_cast<const int32_t *>(sc + kItems);
  A.offset = reinterpret_cast<const int32_t *>(sc + kOffset);
  A.nrob = robots_per_env;
  A.obs_off = reinterpret_cast<const int64_t *>(sc + kObsOff);
  A.x = (float *)b->x; A.y = (float *)b->y; A.th = (float *)b->theta;
  A.gx = (float *)b->goal_x; A.gy = (float *)b->goal_y;
  A.step = b->step; A.episode = b->episode;
  A.qp_fail = ctx->qp_fail;
  for (int n = 0; n <= RS_MAX_ROBOTS; ++n)
    A.qp_iters[n] = sched.qp_iters[n] > 0 ? sched.qp_iters[n] : p->qp_max_iters;
  A.steps = steps;
  A.t0 = (uint32_t)t_global0;
  A.t_start = t_start;
  A.steps_per_env = steps_per_env;
  A.reward_out = reward_out;
  A.done_out = done_out;
  A.reward_sum = reward_sum;
  A.obs_final = obs_final;
  A.qp_stats = qp_stats;
  he = launch_run(A, block_threads, st);
  if (he != hipSuccess) {
    set_error("env_run_noalloc launch failed: %s", hipGetErrorString(he));
    return RS_ERR_DEVICE;
  }
  return RS_OK;
}

}  // extern "C"
