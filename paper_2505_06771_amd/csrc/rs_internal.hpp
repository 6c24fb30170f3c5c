// rs_internal.hpp -- host-side internals shared by the library's translation
// units: context, error reporting, parameter conversion.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "robostep.h"
#include "rs_device.hpp"

namespace rs {

void set_error(const char *fmt, ...);
void clear_error();

struct GraphKey {
  std::vector<uintptr_t> words;
  bool operator<(const GraphKey &o) const { return words < o.words; }
};

// A captured single-kernel launch; `args` holds the argument block the
// instantiated graph currently carries.
struct CachedGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraphNode_t node = nullptr;
  std::vector<char> args;
};

}  // namespace rs

struct rs_ctx {
  int device = 0;
  int num_cus = 256;
  rs_schedule sched{};           // autotuned schedule table
  std::map<rs::GraphKey, rs::CachedGraph> graphs;  // rollout graph cache
  hipStream_t capture_stream = nullptr;
  // certificate failures counted by the kernels: [0] infeasible, [1] capped
  unsigned long long *qp_fail = nullptr;
};

struct rs_plan {
  rs_ctx *ctx = nullptr;
  int32_t num_envs = 0;
  int64_t total_robots = 0;
  std::vector<int32_t> robots_host;      // [E]
  std::vector<int32_t> offset_host;      // [E+1]
  std::vector<int64_t> obs_offset_host;  // [E+1]
  // device arrays
  int32_t *offset_dev = nullptr;   // [E+1] robot offsets
  int32_t *nrob_dev = nullptr;     // [E] robots per env
  int64_t *obs_off_dev = nullptr;  // [E+1] observation offsets
  int32_t *tiles_dev = nullptr;    // [num_tiles * 4]: G, first item, count, N
  int32_t *items_dev = nullptr;    // [E] env indices sorted by tile
  int32_t num_tiles = 0;
  int32_t block_threads = 256;
  rs_schedule sched{};
};

namespace rs {

#define RS_CHECK_ARG(cond, ...)        \
  do {                                 \
    if (!(cond)) {                     \
      ::rs::set_error(__VA_ARGS__);    \
      return RS_ERR_INVALID_ARG;       \
    }                                  \
  } while (0)

#define RS_CHECK_HIP(call)                                                        \
  do {                                                                            \
    hipError_t _e = (call);                                                       \
    if (_e != hipSuccess) {                                                       \
      ::rs::set_error("%s failed: %s", #call, hipGetErrorString(_e));             \
      return RS_ERR_DEVICE;                                                       \
    }                                                                             \
  } while (0)

rs_status check_params(const rs_params *p);

// Looks up this device's copy of env_run_noalloc's work-list array (once per
// device, with the device current; called by rs_create).
hipError_t noalloc_setup(int device);

// Controllers whose nominal command comes from a per-robot action.
inline bool action_driven(int controller) {
  return controller == RS_CTRL_DISCRETE || controller == RS_CTRL_WAYPOINT ||
         controller == RS_CTRL_POSE;
}

template <typename T> SimConst<T> make_const(const rs_params &p) {
  SimConst<T> C;
  C.xwl = (T)(p.x_min + 0.5 * p.safety_radius);
  C.xwh = (T)(p.x_max - 0.5 * p.safety_radius);
  C.ywl = (T)(p.y_min + 0.5 * p.safety_radius);
  C.ywh = (T)(p.y_max - 0.5 * p.safety_radius);
  C.dt = (T)p.dt;
  C.l = (T)p.proj_dist;
  C.inv_l = (T)(1.0 / p.proj_dist);
  C.gamma = (T)p.barrier_gain;
  C.rs2 = (T)(p.safety_radius * p.safety_radius);
  C.kb = (T)(p.boundary_gain_factor * p.barrier_gain);
  C.vmax = (T)p.v_max;
  C.vmax4 = (T)(4.0 * p.v_max);
  C.aspeed = (T)p.action_speed;
  C.kp = (T)p.kp;
  C.wstep = (T)p.waypoint_step;
  C.kv = (T)p.pos_gain;
  C.kw = (T)p.ang_gain;
  C.krho = (T)p.pose_gain_rho;
  C.kalpha = (T)p.pose_gain_alpha;
  C.noise = (T)p.action_noise;
  C.prey_step = (T)(p.prey_speed * p.dt);
  C.tag_r = (T)p.tag_radius;
  C.tag_reward = (T)p.tag_reward;
  const bool sat = p.wheel_radius > 0.0 && p.base_length > 0.0;
  C.R = sat ? (T)p.wheel_radius : T(0);
  C.halfL = sat ? (T)(0.5 * p.base_length) : T(0);
  C.wheel_lim = sat ? (T)(p.v_max / p.wheel_radius) : T(0);
  C.inv_R = sat ? (T)(1.0 / p.wheel_radius) : T(0);
  C.R_over_L = sat ? (T)(p.wheel_radius / p.base_length) : T(0);
  C.goal_r = (T)p.goal_radius;
  const bool f32 = sizeof(T) == 4;
  C.tol_add = f32 ? (T)2e-6 : (T)1e-12;
  C.eps_z = f32 ? (T)1e-9 : (T)1e-20;
  C.eps_r = f32 ? (T)1e-6 : (T)1e-13;
  C.max_steps = p.max_steps;
  C.controller = p.controller;
  C.scenario = p.scenario;
  C.qp_cap = p.qp_max_iters;
  C.key0 = (uint32_t)p.seed;
  C.key1 = (uint32_t)(p.seed >> 32);
  C.xlo = llround((p.x_min + p.reset_margin) / p.grid);
  C.xhi = llround((p.x_max - p.reset_margin) / p.grid);
  C.ylo = llround((p.y_min + p.reset_margin) / p.grid);
  C.yhi = llround((p.y_max - p.reset_margin) / p.grid);
  C.wx = C.xhi - C.xlo + 1;
  C.wy = C.yhi - C.ylo + 1;
  const int64_t s = llround(p.min_sep / p.grid);
  C.sep2 = s * s;
  C.grid = p.grid;
  return C;
}

inline int pow2_group(int n) {
  int g = 2;
  while (g < n) g <<= 1;
  return g;
}

}  // namespace rs
