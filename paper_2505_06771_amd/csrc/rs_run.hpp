// rs_run.hpp -- the persistent multi-step kernel over a work list of
// environments with mixed robot counts (used by env_run, env_reset_mixed, the
// autotuner and the serving loop).
#pragma once

#include "rs_internal.hpp"

namespace rs {

// Device view of one launch of the persistent kernel. Every per-env array is
// indexed by the env index e that the work list names.
struct RunArgs {
  SimConst<float> C;
  int E;           // rows of reward_out/done_out
  int steps;       // step budget of this launch
  int num_tiles;           // tiles of the launch (an upper bound when num_tiles_dev is set)
  const int32_t *num_tiles_dev;  // device tile count written by an earlier kernel (may be NULL)
  uint32_t env_base;
  uint32_t t0;
  const int4 *tiles;       // {G, first item, count, unused}
  const int32_t *items;    // env indices, tile after tile
  const int32_t *offset;   // [E] first robot of env e
  const int32_t *nrob;     // [E] robots of env e
  const uint32_t *env_ids; // [E] stream id of env e (NULL: env_base + e)
  const int64_t *t_start;  // [E] stream time of the env's first step (NULL: t0)
  int64_t *t_after;        // [E] written: t_start + steps run (may be NULL)
  const int32_t *steps_per_env;  // [E] step budget (NULL: steps)
  int32_t *steps_left_after;     // [E] written: budget - steps run (may be NULL)
  uint8_t *reset_mask;     // [E] reset (and clear) flagged envs first (may be NULL)
  const uint8_t *reset_only;  // [E] reset flagged envs, flags left as they are (may be NULL)
  int reset_all;           // reset every env first
  float *x, *y, *th, *gx, *gy;
  int32_t *step, *episode;
  float *reward_out;       // [steps][E] (may be NULL)
  uint8_t *done_out;       // [steps][E] (may be NULL)
  float *reward_sum;       // [E] accumulated (may be NULL)
  float *obs_final;        // (may be NULL)
  const int64_t *obs_off;  // [E] offsets into obs_final
  int32_t *qp_stats;       // [E][kQPStats] accumulated (may be NULL)
  unsigned long long *qp_fail;  // the context's failure counters
  int32_t qp_iters[17];
};

// Launch the persistent kernel: one wavefront per tile.
hipError_t launch_run(const RunArgs &A, int block_threads, hipStream_t st);

// Build tiles/items for the envs `envs` (indices) with robot counts `nrob_of`
// (indexed by env index), grouping by lanes-per-env from `sched`.
void build_tiles(const std::vector<int32_t> &envs, const std::vector<int32_t> &nrob_of,
                 const rs_schedule &sched, std::vector<int32_t> &tiles,
                 std::vector<int32_t> &items);

int lanes_for(const rs_schedule &sched, int n);
// Envs per wavefront tile for robot count n (1 .. 64 / lanes_for).
int envs_per_wave_for(const rs_schedule &sched, int n);

}  // namespace rs
