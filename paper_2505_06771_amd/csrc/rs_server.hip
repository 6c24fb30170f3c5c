// rs_server.hip -- continuous-batching server for rollout requests.
//
// Memory: one device pool sized by the HBM budget holds the robot state of
// every admitted request (five float fields, each a contiguous range of the
// request's robots), and a slot table holds the per-env metadata. Both are
// carved with first-fit range allocators; a request is admitted, in arrival
// order, when its bytes fit the budget and both ranges can be carved.
//
// Ticks: every admitted env advances up to `tick_steps` steps per tick in ONE
// persistent env_run launch over all admitted envs (newly admitted envs are
// reset inside the same launch). The work list of the next tick is built on
// the host while the current one runs; at most two ticks are in flight. The
// host knows each request's remaining steps, so a request whose last step is
// in tick k is retired as soon as tick k's event completes: its final poses
// and summed rewards are copied out and its ranges are freed. Admission and
// retirement allocate no device or pinned memory and create no events: slot
// metadata is staged in a pinned table indexed like the slot table, and a
// request only remembers the index of its last tick.
//
// Determinism: an env's stream id is (request id << 20 | env index) and its
// stream time is its own step count, so a request's result does not depend on
// which other requests share its ticks.
#include "rs_run.hpp"

#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <memory>

namespace rs {

static double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over [0, capacity) with coalescing of free ranges.
class RangeAlloc {
 public:
  void init(int64_t cap) {
    free_.clear();
    if (cap > 0) free_[0] = cap;
  }
  int64_t alloc(int64_t len) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= len) {
        const int64_t start = it->first, rest = it->second - len;
        free_.erase(it);
        if (rest > 0) free_[start + len] = rest;
        return start;
      }
    }
    return -1;
  }
  void release(int64_t start, int64_t len) {
    auto it = free_.emplace(start, len).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<int64_t, int64_t> free_;
};

struct Request {
  int64_t id = 0;
  int32_t envs = 0, robots = 0, horizon = 0;
  int32_t remaining = 0;  // steps not yet launched
  int64_t robot_off = -1;
  int64_t slot_off = -1;
  int64_t bytes = 0;
  double submit_t = 0, admit_t = 0, finish_t = 0;
  int64_t last_tick = -1;  // index of the tick holding its last step
  std::vector<float> xy, rsum;
};

}  // namespace rs

using namespace rs;

struct rs_server {
  rs_ctx *ctx = nullptr;
  rs_params p{};
  int64_t budget = 0, in_use = 0, peak = 0;
  int32_t tick_steps = 0;
  int64_t cap_robots = 0, cap_slots = 0;
  // device pool
  float *x = nullptr, *y = nullptr, *th = nullptr, *gx = nullptr, *gy = nullptr;
  int32_t *step = nullptr, *episode = nullptr, *nrob = nullptr, *offset = nullptr;
  int32_t *steps_left = nullptr;
  uint32_t *env_ids = nullptr;
  int64_t *t_next = nullptr;
  float *rsum = nullptr;
  uint8_t *reset_mask = nullptr;
  int4 *tiles_dev[2] = {nullptr, nullptr};
  int32_t *items_dev[2] = {nullptr, nullptr};
  int32_t *tiles_host[2] = {nullptr, nullptr};  // pinned staging
  int32_t *items_host[2] = {nullptr, nullptr};
  int32_t *meta_host = nullptr;  // pinned [4][cap_slots]: nrob, offset, steps, env id per slot
  hipEvent_t staging_free[2] = {nullptr, nullptr};
  int cur = 0;
  std::vector<int32_t> nrob_of;  // host mirror of nrob per slot
  RangeAlloc robots_alloc, slots_alloc;
  std::deque<std::unique_ptr<Request>> queue;
  std::vector<std::unique_ptr<Request>> running;
  std::deque<std::unique_ptr<Request>> finished;
  hipEvent_t tick_ev[2] = {nullptr, nullptr};  // event of tick k in slot k & 1
  int64_t ticks_launched = 0;
  int64_t ticks_done = 0;  // ticks 0 .. ticks_done - 1 are known complete
  hipStream_t stream = nullptr, copy_stream = nullptr;
  rs_server_stats stats{};
};

namespace rs {

static const int64_t kEnvBytes = 4 * 4 + 8 + 4 + 4 + 1;  // slot metadata per env
static const int64_t kRobotBytes = 5 * 4;

static void free_server(rs_server *s) {
  void *ptrs[] = {s->x, s->y, s->th, s->gx, s->gy, s->step, s->episode, s->nrob, s->offset,
                  s->steps_left, s->env_ids, s->t_next, s->rsum, s->reset_mask,
                  s->tiles_dev[0], s->tiles_dev[1], s->items_dev[0], s->items_dev[1]};
  for (void *q : ptrs)
    if (q) (void)hipFree(q);
  for (int k = 0; k < 2; ++k) {
    if (s->tiles_host[k]) (void)hipHostFree(s->tiles_host[k]);
    if (s->items_host[k]) (void)hipHostFree(s->items_host[k]);
    if (s->staging_free[k]) (void)hipEventDestroy(s->staging_free[k]);
  }
  for (hipEvent_t e : s->tick_ev)
    if (e) (void)hipEventDestroy(e);
  if (s->meta_host) (void)hipHostFree(s->meta_host);
  if (s->stream) (void)hipStreamDestroy(s->stream);
  if (s->copy_stream) (void)hipStreamDestroy(s->copy_stream);
  delete s;
}

// Whether tick k has completed (ticks complete in launch order on the one
// stream). The event of tick k stays in slot k & 1 until tick k + 2 is
// launched, and launching tick k + 2 first waits for tick k.
static bool tick_complete(rs_server *s, int64_t k, bool wait) {
  if (k < s->ticks_done) return true;
  if (k >= s->ticks_launched) return false;
  hipEvent_t ev = s->tick_ev[k & 1];
  if ((wait ? hipEventSynchronize(ev) : hipEventQuery(ev)) != hipSuccess) return false;
  s->ticks_done = k + 1;
  return true;
}

// Retire requests whose last tick has completed.
static rs_status retire(rs_server *s, bool wait) {
  for (size_t k = 0; k < s->running.size();) {
    Request *r = s->running[k].get();
    const bool ready = r->remaining == 0 && r->last_tick >= 0 && tick_complete(s, r->last_tick, wait);
    if (!ready) { ++k; continue; }
    const int64_t R = (int64_t)r->envs * r->robots;
    std::vector<float> hx(R), hy(R);
    RS_CHECK_HIP(hipMemcpyAsync(hx.data(), s->x + r->robot_off, R * 4, hipMemcpyDeviceToHost, s->copy_stream));
    RS_CHECK_HIP(hipMemcpyAsync(hy.data(), s->y + r->robot_off, R * 4, hipMemcpyDeviceToHost, s->copy_stream));
    r->rsum.resize(r->envs);
    RS_CHECK_HIP(hipMemcpyAsync(r->rsum.data(), s->rsum + r->slot_off, (size_t)r->envs * 4,
                                hipMemcpyDeviceToHost, s->copy_stream));
    RS_CHECK_HIP(hipStreamSynchronize(s->copy_stream));
    r->xy.resize(2 * R);
    for (int64_t q = 0; q < R; ++q) { r->xy[2 * q] = hx[q]; r->xy[2 * q + 1] = hy[q]; }
    r->finish_t = now_s();
    s->robots_alloc.release(r->robot_off, R);
    s->slots_alloc.release(r->slot_off, r->envs);
    s->in_use -= r->bytes;
    s->stats.finished++;
    s->finished.push_back(std::move(s->running[k]));
    s->running.erase(s->running.begin() + k);
  }
  return RS_OK;
}

static rs_status admit(rs_server *s) {
  while (!s->queue.empty()) {
    Request *r = s->queue.front().get();
    if (s->in_use + r->bytes > s->budget) break;
    const int64_t R = (int64_t)r->envs * r->robots;
    const int64_t ro = s->robots_alloc.alloc(R);
    if (ro < 0) break;
    const int64_t so = s->slots_alloc.alloc(r->envs);
    if (so < 0) {
      s->robots_alloc.release(ro, R);
      break;
    }
    r->robot_off = ro;
    r->slot_off = so;
    r->admit_t = now_s();
    r->remaining = r->horizon;
    s->in_use += r->bytes;
    s->peak = std::max(s->peak, s->in_use);
    // slot metadata: nrob, offset, steps_left, env_ids (4 int32 per env),
    // staged in the pinned table at the request's slots. A slot range is
    // handed out again only after its previous request retired, i.e. after
    // the tick holding its last step completed, which the copies below of
    // that request preceded on the same stream.
    const int64_t S = s->cap_slots;
    int32_t *m0 = s->meta_host + so, *m1 = m0 + S, *m2 = m1 + S, *m3 = m2 + S;
    for (int32_t e = 0; e < r->envs; ++e) {
      m0[e] = r->robots;
      m1[e] = (int32_t)(ro + (int64_t)e * r->robots);
      m2[e] = r->horizon;
      m3[e] = (int32_t)(((uint32_t)r->id << 20) | (uint32_t)e);
      s->nrob_of[so + e] = r->robots;
    }
    const size_t nb = (size_t)r->envs * 4;
    RS_CHECK_HIP(hipMemcpyAsync(s->nrob + so, m0, nb, hipMemcpyHostToDevice, s->stream));
    RS_CHECK_HIP(hipMemcpyAsync(s->offset + so, m1, nb, hipMemcpyHostToDevice, s->stream));
    RS_CHECK_HIP(hipMemcpyAsync(s->steps_left + so, m2, nb, hipMemcpyHostToDevice, s->stream));
    RS_CHECK_HIP(hipMemcpyAsync(s->env_ids + so, m3, nb, hipMemcpyHostToDevice, s->stream));
    RS_CHECK_HIP(hipMemsetAsync(s->t_next + so, 0, (size_t)r->envs * 8, s->stream));
    RS_CHECK_HIP(hipMemsetAsync(s->step + so, 0, nb, s->stream));
    RS_CHECK_HIP(hipMemsetAsync(s->episode + so, 0, nb, s->stream));
    RS_CHECK_HIP(hipMemsetAsync(s->rsum + so, 0, nb, s->stream));
    RS_CHECK_HIP(hipMemsetAsync(s->reset_mask + so, 1, (size_t)r->envs, s->stream));
    s->stats.admitted++;
    s->running.push_back(std::move(s->queue.front()));
    s->queue.pop_front();
  }
  return RS_OK;
}

static rs_status launch_tick(rs_server *s) {
  std::vector<int32_t> envs;
  for (auto &r : s->running) {
    if (r->remaining <= 0) continue;
    for (int32_t e = 0; e < r->envs; ++e) envs.push_back((int32_t)(r->slot_off + e));
  }
  if (envs.empty()) return RS_OK;
  // at most two ticks in flight: wait for tick k-2 before launching tick k
  const int slot = (int)(s->ticks_launched & 1);
  if (s->ticks_launched >= 2 && !tick_complete(s, s->ticks_launched - 2, true)) {
    set_error("serving: waiting for tick %lld failed", (long long)(s->ticks_launched - 2));
    return RS_ERR_DEVICE;
  }
  std::vector<int32_t> tiles, items;
  build_tiles(envs, s->nrob_of, s->ctx->sched, tiles, items);
  const int k = s->cur;
  s->cur ^= 1;
  RS_CHECK_HIP(hipEventSynchronize(s->staging_free[k]));
  std::memcpy(s->tiles_host[k], tiles.data(), tiles.size() * 4);
  std::memcpy(s->items_host[k], items.data(), items.size() * 4);
  RS_CHECK_HIP(hipMemcpyAsync(s->tiles_dev[k], s->tiles_host[k], tiles.size() * 4,
                              hipMemcpyHostToDevice, s->stream));
  RS_CHECK_HIP(hipMemcpyAsync(s->items_dev[k], s->items_host[k], items.size() * 4,
                              hipMemcpyHostToDevice, s->stream));
  RS_CHECK_HIP(hipEventRecord(s->staging_free[k], s->stream));
  RunArgs A;
  std::memset(&A, 0, sizeof(A));
  A.C = make_const<float>(s->p);
  A.E = (int)s->cap_slots;
  A.steps = s->tick_steps;
  A.num_tiles = (int)(tiles.size() / 4);
  A.tiles = s->tiles_dev[k];
  A.items = s->items_dev[k];
  A.offset = s->offset;
  A.nrob = s->nrob;
  A.env_ids = s->env_ids;
  A.t_start = s->t_next;
  A.t_after = s->t_next;
  A.steps_per_env = s->steps_left;
  A.steps_left_after = s->steps_left;
  A.reset_mask = s->reset_mask;
  A.x = s->x; A.y = s->y; A.th = s->th; A.gx = s->gx; A.gy = s->gy;
  A.step = s->step; A.episode = s->episode;
  A.reward_sum = s->rsum;
  A.qp_fail = s->ctx->qp_fail;
  // the iteration cap of env_run's plans: the schedule's, else the parameters'
  for (int n = 0; n <= RS_MAX_ROBOTS; ++n)
    A.qp_iters[n] = s->ctx->sched.qp_iters[n] > 0 ? s->ctx->sched.qp_iters[n] : s->p.qp_max_iters;
  const int blk = s->ctx->sched.block_threads > 0 ? s->ctx->sched.block_threads : 256;
  hipError_t he = launch_run(A, blk, s->stream);
  if (he != hipSuccess) {
    set_error("serving tick launch failed: %s", hipGetErrorString(he));
    return RS_ERR_DEVICE;
  }
  RS_CHECK_HIP(hipEventRecord(s->tick_ev[slot], s->stream));
  const int64_t this_tick = s->ticks_launched++;
  for (auto &r : s->running) {
    if (r->remaining <= 0) continue;
    const int32_t adv = std::min(r->remaining, s->tick_steps);
    s->stats.robot_steps += (int64_t)adv * r->envs * r->robots;
    r->remaining -= adv;
    if (r->remaining == 0) r->last_tick = this_tick;
  }
  s->stats.ticks++;
  return RS_OK;
}

}  // namespace rs

extern "C" {

int64_t rs_request_bytes(int32_t envs, int32_t robots) {
  if (envs <= 0 || robots <= 0) return 0;
  const int64_t b = (int64_t)envs * robots * kRobotBytes + (int64_t)envs * kEnvBytes;
  return (b + 255) & ~(int64_t)255;
}

rs_status rs_server_create(rs_ctx *ctx, const rs_params *p, int64_t hbm_budget_bytes,
                           int32_t tick_steps, rs_server **out) {
  RS_CHECK_ARG(ctx != nullptr && out != nullptr, "ctx/out is NULL");
  rs_status st = check_params(p);
  if (st != RS_OK) return st;
  RS_CHECK_ARG(p->dtype == RS_F32 && action_driven(p->controller),
               "the server runs the FP32 path of an action-driven controller");

  RS_CHECK_ARG(hbm_budget_bytes >= 4096, "budget too small");
  RS_CHECK_ARG(tick_steps >= 1, "tick_steps must be >= 1");
  *out = nullptr;
  rs_server *s = new rs_server();
  s->ctx = ctx;
  s->p = *p;
  s->budget = hbm_budget_bytes;
  s->tick_steps = tick_steps;
  // every admitted byte set fits: robots need >= 20 B each, envs >= 49 B
  s->cap_robots = hbm_budget_bytes / kRobotBytes;
  // slot table: as many envs as the budget can hold (2 robots each), at most
  // 2^21; the work-list buffers are sized by it
  s->cap_slots = std::min<int64_t>(hbm_budget_bytes / (kEnvBytes + 2 * kRobotBytes), 1 << 21);
  s->nrob_of.assign(s->cap_slots, 2);
  s->robots_alloc.init(s->cap_robots);
  s->slots_alloc.init(s->cap_slots);
  auto fail = [&](const char *what) {
    set_error("server allocation failed (%s)", what);
    free_server(s);
    return RS_ERR_OUT_OF_MEMORY;
  };
  const size_t R = (size_t)s->cap_robots, S = (size_t)s->cap_slots;
  if (hipMalloc(&s->x, R * 4) || hipMalloc(&s->y, R * 4) || hipMalloc(&s->th, R * 4) ||
      hipMalloc(&s->gx, R * 4) || hipMalloc(&s->gy, R * 4))
    return fail("robot pool");
  if (hipMalloc(&s->step, S * 4) || hipMalloc(&s->episode, S * 4) || hipMalloc(&s->nrob, S * 4) ||
      hipMalloc(&s->offset, S * 4) || hipMalloc(&s->steps_left, S * 4) ||
      hipMalloc(&s->env_ids, S * 4) || hipMalloc(&s->t_next, S * 8) || hipMalloc(&s->rsum, S * 4) ||
      hipMalloc(&s->reset_mask, S))
    return fail("slot table");
  for (int k = 0; k < 2; ++k) {
    if (hipMalloc(&s->tiles_dev[k], S * 16) || hipMalloc(&s->items_dev[k], S * 4)) return fail("work list");
    if (hipHostMalloc((void **)&s->tiles_host[k], S * 16, hipHostMallocDefault) ||
        hipHostMalloc((void **)&s->items_host[k], S * 4, hipHostMallocDefault))
      return fail("pinned staging");
    if (hipEventCreateWithFlags(&s->staging_free[k], hipEventDisableTiming)) return fail("event");
  }
  if (hipHostMalloc((void **)&s->meta_host, 4 * S * sizeof(int32_t), hipHostMallocDefault))
    return fail("pinned metadata table");
  if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) ||
      hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking))
    return fail("streams");
  if (hipEventCreateWithFlags(&s->tick_ev[0], hipEventDisableTiming) ||
      hipEventCreateWithFlags(&s->tick_ev[1], hipEventDisableTiming))
    return fail("events");
  *out = s;
  return RS_OK;
}

rs_status rs_server_destroy(rs_server *s) {
  if (!s) return RS_OK;
  (void)hipStreamSynchronize(s->stream);
  (void)hipStreamSynchronize(s->copy_stream);
  free_server(s);
  return RS_OK;
}

rs_status rs_server_submit(rs_server *s, int64_t id, int32_t envs, int32_t robots,
                           int32_t horizon) {
  RS_CHECK_ARG(s != nullptr, "server is NULL");
  RS_CHECK_ARG(envs >= 1 && envs < (1 << 20), "envs must be in 1..2^20-1");
  RS_CHECK_ARG(robots >= 2 && robots <= RS_MAX_ROBOTS, "robots must be in 2..16");
  RS_CHECK_ARG(horizon >= 1, "horizon must be >= 1");
  RS_CHECK_ARG(id >= 0 && id < (1 << 12), "request id must be in 0..4095 (12-bit stream field)");
  auto r = std::make_unique<Request>();
  r->id = id;
  r->envs = envs;
  r->robots = robots;
  r->horizon = horizon;
  r->bytes = rs_request_bytes(envs, robots);
  r->submit_t = now_s();
  if (r->bytes > s->budget || (int64_t)envs > s->cap_slots ||
      (int64_t)envs * robots > s->cap_robots) {
    set_error("request %lld needs %lld bytes, budget %lld", (long long)id, (long long)r->bytes,
              (long long)s->budget);
    return RS_ERR_BUDGET;
  }
  s->queue.push_back(std::move(r));
  s->stats.submitted++;
  return RS_OK;
}

rs_status rs_server_tick(rs_server *s, int32_t *busy) {
  RS_CHECK_ARG(s != nullptr, "server is NULL");
  rs_status st = retire(s, false);
  if (st != RS_OK) return st;
  st = admit(s);
  if (st != RS_OK) return st;
  st = launch_tick(s);
  if (st != RS_OK) return st;
  if (busy) *busy = (s->queue.empty() && s->running.empty()) ? 0 : 1;
  // when every running request has launched all its steps, wait for them so
  // the caller's loop ends with results available
  bool all_launched = !s->running.empty();
  for (auto &r : s->running) all_launched = all_launched && r->remaining == 0;
  if (all_launched && s->queue.empty()) {
    st = retire(s, true);
    if (st != RS_OK) return st;
    if (busy) *busy = s->running.empty() ? 0 : 1;
  }
  return RS_OK;
}

rs_status rs_server_poll(rs_server *s, rs_request_info *info, float *final_xy, float *reward_sum) {
  RS_CHECK_ARG(s != nullptr, "server is NULL");
  if (s->finished.empty()) return RS_ERR_NOT_FOUND;
  Request *r = s->finished.front().get();
  if (info) {
    info->id = r->id;
    info->envs = r->envs;
    info->robots = r->robots;
    info->horizon = r->horizon;
    info->submit_time = r->submit_t;
    info->admit_time = r->admit_t;
    info->finish_time = r->finish_t;
  }
  if (final_xy) std::memcpy(final_xy, r->xy.data(), r->xy.size() * 4);
  if (reward_sum) std::memcpy(reward_sum, r->rsum.data(), r->rsum.size() * 4);
  s->finished.pop_front();
  return RS_OK;
}

rs_status rs_server_stats_get(rs_server *s, rs_server_stats *out) {
  RS_CHECK_ARG(s != nullptr && out != nullptr, "server/out is NULL");
  *out = s->stats;
  out->bytes_in_use = s->in_use;
  out->peak_bytes = s->peak;
  out->queued = (int32_t)s->queue.size();
  out->running = (int32_t)s->running.size();
  return RS_OK;
}

}  // extern "C"
