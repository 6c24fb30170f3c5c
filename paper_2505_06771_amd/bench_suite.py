"""Secondary benchmarks of the batched Robotarium step (one MI355X).

  single_env_f64   1 env x 4 robots, go-to-goal, FP64, 1000 steps: per-step
                   env_step launches, plain and hipGraph-captured, and one
                   persistent env_steps launch (us/step)
  uniform_4096x4   4096 envs x 4 robots, random moves, 1000 steps: per-step
                   env_step launches (plain, graph) and one persistent env_run
  uneven_8192      8192 envs, N in {2,4,6,8,12} (0.1/0.3/0.3/0.2/0.1), 1000
                   steps: one persistent env_run launch (default and autotuned
                   schedule) vs per-size env_step launches (5 per step)
  rollout_waypoint_noise
                   the fused 16384 x 8 x 128 policy rollout with waypoint
                   actions (unicycle position controller) and with waypoint
                   poses (unicycle pose controller), both with action noise,
                   beside the same rollout with discrete moves and no noise
                   (kernel ms per launch from HIP events, robot-steps/s)
  rollout_predator_prey
                   Predator-Prey rollouts (waypoint actions, 100-step
                   episodes): 16384 envs x 8 robots and 43690 envs x 3
  serving          Poisson rollout requests (64-4096 envs log-uniform, N in
                   3..16, horizon 50-500): continuous batching vs plain
                   per-request per-step launches; p50/p99 latency + robot-steps/s

Every number is measured with inputs resident on the device; results are
written as JSON lines to the output file and echoed on stderr.
"""
from __future__ import annotations

import json
import math
import sys
import time

import numpy as np


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _sync():
    import torch

    torch.cuda.synchronize()


def _graph_of(fn):
    """Capture fn() (a sequence of library launches on the current stream)."""
    import torch

    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()  # warm-up outside capture
    torch.cuda.current_stream().wait_stream(s)
    _sync()
    with torch.cuda.graph(g):
        fn()
    _sync()
    return g


def launch_floor_us(reps=2000):
    import torch

    torch.cuda._sleep(1)
    _sync()
    t0 = time.perf_counter()
    for _ in range(reps):
        torch.cuda._sleep(1)
    _sync()
    return (time.perf_counter() - t0) / reps * 1e6


def single_env_f64(R, ctx, seed=0, steps=1000):
    import torch

    p = R.params(controller=R.RS_CTRL_GOTO, goal_radius=0.0, max_steps=0, dtype=R.RS_F64,
                 seed=seed)
    b = R.Batch.empty(1, 4, dtype=torch.float64)
    R.env_reset(ctx, p, b)
    _sync()
    t0 = time.perf_counter()
    for t in range(steps):
        R.env_step(ctx, p, b, t_global=t)
    _sync()
    plain = (time.perf_counter() - t0) / steps * 1e6
    g = _graph_of(lambda: [R.env_step(ctx, p, b, t_global=t) for t in range(100)])
    t0 = time.perf_counter()
    for _ in range(steps // 100):
        g.replay()
    _sync()
    graph = (time.perf_counter() - t0) / steps * 1e6
    R.env_steps(ctx, p, b, 10, t_global0=2 * steps)  # warm-up
    _sync()
    t0 = time.perf_counter()
    R.env_steps(ctx, p, b, steps, t_global0=3 * steps)
    _sync()
    persistent = (time.perf_counter() - t0) / steps * 1e6
    return {"config": "single_env_f64", "envs": 1, "robots": 4, "steps": steps,
            "us_per_step_plain": plain, "us_per_step_graph": graph,
            "us_per_step_persistent": persistent,
            "robot_steps_per_s_graph": 4 / (graph * 1e-6),
            "robot_steps_per_s_persistent": 4 / (persistent * 1e-6)}


def uniform_4096x4(R, ctx, seed=0, steps=1000):
    import torch

    E, n = 4096, 4
    p = R.params(seed=seed)
    b = R.Batch.empty(E, n)
    R.env_reset(ctx, p, b)
    obs = torch.empty(E * n * (2 * n + 4), device="cuda")
    rew = torch.empty(E, device="cuda")
    done = torch.empty(E, dtype=torch.uint8, device="cuda")
    step = lambda t: R.env_step(ctx, p, b, t_global=t, obs=obs, reward=rew, done=done)
    step(0)
    _sync()
    t0 = time.perf_counter()
    for t in range(steps):
        step(t)
    _sync()
    plain = (time.perf_counter() - t0) / steps
    g = _graph_of(lambda: [step(t) for t in range(100)])
    t0 = time.perf_counter()
    for _ in range(steps // 100):
        g.replay()
    _sync()
    graph = (time.perf_counter() - t0) / steps
    plan = R.Plan(ctx, np.full(E, n, np.int32))
    R.env_run(ctx, p, plan, b, 10)
    _sync()
    t0 = time.perf_counter()
    R.env_run(ctx, p, plan, b, steps, t_global0=0)
    _sync()
    persist = (time.perf_counter() - t0) / steps
    rs = E * n
    return {"config": "uniform_4096x4", "envs": E, "robots": n, "steps": steps,
            "us_per_step_plain": plain * 1e6, "us_per_step_graph": graph * 1e6,
            "us_per_step_env_run": persist * 1e6, "launch_floor_us": launch_floor_us(),
            "robot_steps_per_s_plain": rs / plain, "robot_steps_per_s_graph": rs / graph,
            "robot_steps_per_s_env_run": rs / persist}


def uneven_8192(R, ctx, seed=0, steps=1000, autotune=True):
    import torch

    from paper_2505_06771_amd import synth

    counts = synth.uneven_sizes(seed, 8192)
    robots = int(counts.sum())
    p = R.params(seed=seed)
    out = {"config": "uneven_8192", "envs": 8192, "robots_total": robots, "steps": steps}

    def persistent(schedule, label):
        plan = R.Plan(ctx, counts, schedule)
        b = R.Batch.empty(8192, 0, total_robots=plan.total_robots)
        R.env_reset_mixed(ctx, p, plan, b)
        R.env_run(ctx, p, plan, b, 5)
        _sync()
        ctx.qp_failures(reset=True)
        t0 = time.perf_counter()
        R.env_run(ctx, p, plan, b, steps, t_global0=0)
        _sync()
        dt = time.perf_counter() - t0
        out[f"robot_steps_per_s_{label}"] = robots * steps / dt
        out[f"ms_{label}"] = dt * 1e3
        # certificate solves of the timed run that were infeasible or stopped
        # at the schedule's iteration cap (a capped solve is not exact)
        out[f"qp_infeasible_{label}"], out[f"qp_capped_{label}"] = ctx.qp_failures(reset=True)

    persistent(None, "persistent_default")
    if autotune:
        # tuned on the benchmark's own batch (the reset state), 50 steps
        plan = R.Plan(ctx, counts)
        b = R.Batch.empty(8192, 0, total_robots=plan.total_robots)
        R.env_reset_mixed(ctx, p, plan, b)
        t0 = time.perf_counter()
        s = R.autotune_batch(ctx, p, plan, b, steps=50, tol=1e-4)
        out["autotune_s"] = time.perf_counter() - t0
        out["schedule"] = {"block_threads": s.block_threads,
                           "lanes_per_env": {n: s.lanes_per_env[n] for n in (2, 4, 6, 8, 12)},
                           "envs_per_wave": {n: s.envs_per_wave[n] for n in (2, 4, 6, 8, 12)},
                           "qp_iters": {n: s.qp_iters[n] for n in (2, 4, 6, 8, 12)}}
        persistent(s, "persistent_autotuned")
    # plain: one uniform batch per size, 5 env_step launches per step
    batches = []
    base = 0
    for n in sorted(set(counts.tolist())):
        k = int((counts == n).sum())
        bb = R.Batch.empty(k, n, env_id_base=base)
        R.env_reset(ctx, p, bb)
        batches.append(bb)
        base += k
    for bb in batches:
        R.env_step(ctx, p, bb, t_global=0)
    _sync()
    t0 = time.perf_counter()
    for t in range(steps):
        for bb in batches:
            R.env_step(ctx, p, bb, t_global=t)
    _sync()
    dt = time.perf_counter() - t0
    out["robot_steps_per_s_plain_per_size"] = robots * steps / dt
    out["ms_plain_per_size"] = dt * 1e3
    return out


def serving(R, ctx, seed=0, count=2000, skip=200, budget=64 << 30, stress_budget=2 << 20,
            tick=32, rate=None, plain_count=120):
    """Continuous batching vs plain per-request launches on the same Poisson
    arrival process. `rate` defaults to 0.7 x the saturated capacity of the
    served path (measured first on a burst) / mean request work. The served
    path runs twice: at the nominal HBM budget and at `stress_budget`, small
    enough that admission queues requests (2 MiB holds one request of the
    largest size, 4096 envs x 16 robots, 1.45 MB). Two plain forms serve the
    same stream in arrival order, one request at a time: every request in one
    persistent env_run launch (all requests; its saturated capacity is
    measured on the same burst as the served path's), and every step as its
    own env_step launch (only the first `plain_count` requests: about a third
    of a second each)."""
    import torch

    from paper_2505_06771_amd import synth

    p = R.params(seed=seed)
    probe = synth.request_stream(seed + 1, 64, 1.0)
    # saturated capacity: all requests at once
    srv = R.Server(ctx, p, budget, tick)
    t0 = time.perf_counter()
    for r in probe:
        srv.submit(r["id"], r["envs"], r["robots"], r["horizon"])
    while srv.tick():
        while srv.poll() is not None:
            pass
    while srv.poll() is not None:
        pass
    cap = srv.stats().robot_steps / (time.perf_counter() - t0)
    srv.close()
    mean_work = np.mean([r["envs"] * r["robots"] * r["horizon"] for r in probe])
    if rate is None:
        rate = 0.7 * cap / mean_work
    reqs = synth.request_stream(seed, count, rate)

    def run_served(budget):
        srv = R.Server(ctx, p, budget, tick)
        lat, late = {}, {}
        start = time.perf_counter()
        k = 0
        while len(lat) < count:
            now = time.perf_counter() - start
            while k < count and reqs[k]["arrival"] <= now:
                r = reqs[k]
                srv.submit(r["id"], r["envs"], r["robots"], r["horizon"])
                late[r["id"]] = (time.perf_counter() - start) - r["arrival"]
                k += 1
            busy = srv.tick()
            while True:
                info = srv.poll()
                if info is None:
                    break
                # completion - arrival: server clock from submission to
                # completion plus the load generator's own delay in submitting
                lat[info.id] = (info.finish_time - info.submit_time) + late[info.id]
            if not busy and k < count:
                time.sleep(max(0.0, min(1e-3, reqs[k]["arrival"] - (time.perf_counter() - start))))
        wall = time.perf_counter() - start
        st = srv.stats()
        srv.close()
        return lat, wall, st.robot_steps, st.peak_bytes

    def run_plain(n_req):
        """FIFO, one request at a time, reset + one env_step launch per step."""
        lat = {}
        start = time.perf_counter()
        work = 0
        for r in reqs[:n_req]:
            now = time.perf_counter() - start
            if now < r["arrival"]:
                time.sleep(r["arrival"] - now)
            b = R.Batch.empty(r["envs"], r["robots"], env_id_base=r["id"] << 20)
            R.env_reset(ctx, p, b)
            for t in range(r["horizon"]):
                R.env_step(ctx, p, b, t_global=t)
            _sync()
            lat[r["id"]] = time.perf_counter() - start - r["arrival"]
            work += r["envs"] * r["robots"] * r["horizon"]
        return lat, time.perf_counter() - start, work

    # plain but fair: FIFO, each request alone in ONE persistent env_run
    # launch (no per-step launches). Per robot count a 4096-env plan and
    # state are made up front, so nothing is allocated per request; a
    # request resets and runs its first `envs` envs (the others take 0 steps)
    # with the served path's env ids and stream times.
    import torch as _t

    pre = {}
    for n in range(3, 17):
        pl = R.Plan(ctx, np.full(4096, n, np.int32))
        pre[n] = (pl, R.Batch.empty(4096, 0, total_robots=pl.total_robots))
    mask = _t.zeros(4096, dtype=_t.uint8, device="cuda")
    spe = _t.zeros(4096, dtype=_t.int32, device="cuda")

    def plain_one(r):
        pl, bb = pre[r["robots"]]
        bb.env_id_base = r["id"] << 20
        bb.step.zero_()
        bb.episode.zero_()
        mask.zero_()
        mask[:r["envs"]] = 1
        spe.zero_()
        spe[:r["envs"]] = r["horizon"]
        R.env_reset_mixed(ctx, p, pl, bb, mask=mask)
        R.env_run(ctx, p, pl, bb, r["horizon"], t_global0=0, steps_per_env=spe)

    def run_plain_persistent(rs, honour_arrivals=True):
        lat = {}
        start = time.perf_counter()
        work = 0
        for r in rs:
            now = time.perf_counter() - start
            if honour_arrivals and now < r["arrival"]:
                time.sleep(r["arrival"] - now)
            plain_one(r)
            _sync()
            lat[r["id"]] = time.perf_counter() - start - r["arrival"]
            work += r["envs"] * r["robots"] * r["horizon"]
        return lat, time.perf_counter() - start, work

    # saturated capacity of the plain persistent form on the same burst
    _, wall_pc, work_pc = run_plain_persistent(probe, honour_arrivals=False)
    cap_plain = work_pc / wall_pc

    lat_s, wall_s, work_s, _ = run_served(budget)
    ls = np.array([lat_s[i] for i in range(skip, count)])
    lat_q, wall_q, work_q, peak_q = run_served(stress_budget)
    lq = np.array([lat_q[i] for i in range(skip, count)])
    lat_pp, wall_pp, work_pp = run_plain_persistent(reqs)
    lpp = np.array([lat_pp[i] for i in range(skip, count)])
    n_plain = min(plain_count, count)
    lat_p, wall_p, work_p = run_plain(n_plain)
    lp = np.array([lat_p[i] for i in range(min(skip, n_plain // 2), n_plain)])
    return {"config": "serving", "requests": count, "excluded_warmup": skip,
            "arrival_rate_hz": rate, "saturated_capacity_robot_steps_per_s": cap,
            "mean_request_robot_steps": mean_work, "tick_steps": tick, "budget_bytes": budget,
            "served_p50_ms": float(np.percentile(ls, 50) * 1e3),
            "served_p99_ms": float(np.percentile(ls, 99) * 1e3),
            "served_robot_steps_per_s": work_s / wall_s,
            "stress_budget_bytes": stress_budget, "stress_peak_bytes": peak_q,
            "stress_p50_ms": float(np.percentile(lq, 50) * 1e3),
            "stress_p99_ms": float(np.percentile(lq, 99) * 1e3),
            "stress_robot_steps_per_s": work_q / wall_q,
            "plain_persistent_capacity_robot_steps_per_s": cap_plain,
            "plain_persistent_requests": count,
            "plain_persistent_p50_ms": float(np.percentile(lpp, 50) * 1e3),
            "plain_persistent_p99_ms": float(np.percentile(lpp, 99) * 1e3),
            "plain_persistent_robot_steps_per_s": work_pp / wall_pp,
            "plain_requests": n_plain,
            "plain_p50_ms": float(np.percentile(lp, 50) * 1e3),
            "plain_p99_ms": float(np.percentile(lp, 99) * 1e3),
            "plain_robot_steps_per_s": work_p / wall_p}


def _time_rollout(R, ctx, p, E, n, H, launches, seed):
    """Median kernel time (ms, HIP events on the launch stream) of `launches`
    rollout launches after two warm-ups, from a fresh reset."""
    import torch

    from paper_2505_06771_amd import synth

    D = 2 * n + 4
    w = synth.policy_weights(seed, D)
    bf = lambda a: torch.from_numpy(a).to(torch.bfloat16).cuda().contiguous()
    fl = lambda a: torch.from_numpy(a).float().cuda().contiguous()
    pol = R.Policy(bf(w["w1"]), fl(w["b1"]), bf(w["w2"]), fl(w["b2"]), bf(w["w3"]), fl(w["b3"]))
    obs = torch.empty(H * E * n * D, device="cuda")
    act = torch.empty(H * E * n, dtype=torch.uint8, device="cuda")
    rew = torch.empty(H * E, device="cuda")
    done = torch.empty(H * E, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    b = R.Batch.empty(E, n)
    R.env_reset(ctx, p, b)
    for k in range(2):
        R.rollout(ctx, p, b, pol, H, k * H, obs, act, rew, done, stream=stream)
    _sync()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(launches)]
    for k in range(launches):
        ev[k][0].record(stream)
        R.rollout(ctx, p, b, pol, H, (2 + k) * H, obs, act, rew, done, stream=stream)
        ev[k][1].record(stream)
    _sync()
    ms = sorted(a.elapsed_time(z) for a, z in ev)
    return ms[len(ms) // 2], float(rew.sum().item())


def _rollout_bytes(E, n, H):
    """HBM bytes per launch: obs + action per robot-step, reward + done per
    env-step, state in and out once, weights once."""
    D = 2 * n + 4
    return (H * (E * n * (4 * D + 1) + E * 5) + 2 * (E * n * 20 + E * 8)
            + 2 * (D * 64 + 64 * 64 + 64 * 5) + 4 * (64 + 64 + 5))


def rollout_waypoint_noise(R, ctx, seed=0, launches=10, E=16384, n=8, H=128, sigma=0.05):
    algo = _rollout_bytes(E, n, H)
    res = {"config": "rollout_waypoint_noise", "envs": E, "robots": n, "horizon": H,
           "launches": launches, "action_noise": sigma}
    for name, kw in (("discrete", {}),
                     ("waypoint_noise", {"controller": R.RS_CTRL_WAYPOINT, "action_noise": sigma}),
                     ("pose_noise", {"controller": R.RS_CTRL_POSE, "action_noise": sigma})):
        med, _ = _time_rollout(R, ctx, R.params(seed=seed, **kw), E, n, H, launches, seed)
        res[f"kernel_ms_median_{name}"] = med
        res[f"robot_steps_per_s_{name}"] = E * n * H / (med * 1e-3)
        res[f"hbm_frac_{name}"] = algo / (med * 1e-3) / 8e12
    res["algorithmic_bytes_per_launch"] = algo
    return res


def rollout_predator_prey(R, ctx, seed=0, launches=10, H=128):
    """Predator-Prey rollouts with waypoint actions and 100-step episodes: the
    headline shape (16384 envs x 8 robots) and the paper's team size (3
    robots) on the same number of robots."""
    res = {"config": "rollout_predator_prey", "horizon": H, "launches": launches,
           "controller": "waypoint", "max_steps": 100}
    for E, n in ((16384, 8), (43690, 3)):
        p = R.params(seed=seed, scenario=R.RS_SCN_PREDATOR_PREY,
                     controller=R.RS_CTRL_WAYPOINT, max_steps=100)
        med, tags = _time_rollout(R, ctx, p, E, n, H, launches, seed)
        algo = _rollout_bytes(E, n, H)
        key = f"{E}x{n}"
        res[f"kernel_ms_median_{key}"] = med
        res[f"robot_steps_per_s_{key}"] = E * n * H / (med * 1e-3)
        res[f"hbm_frac_{key}"] = algo / (med * 1e-3) / 8e12
        res[f"tag_reward_last_launch_{key}"] = tags
    return res


def run_all(path, seed=0, which=("single_env_f64", "uniform_4096x4", "uneven_8192",
                                 "rollout_waypoint_noise", "rollout_predator_prey", "serving")):
    import os

    import torch

    from paper_2505_06771_amd import robostep as R

    torch.cuda.init()  # torch first: its tensors and the library share the device
    ctx = R.Context(0)
    os.makedirs(os.path.dirname(path), exist_ok=True)
    fns = {"single_env_f64": single_env_f64, "uniform_4096x4": uniform_4096x4,
           "uneven_8192": uneven_8192, "rollout_waypoint_noise": rollout_waypoint_noise,
           "rollout_predator_prey": rollout_predator_prey, "serving": serving}
    with open(path, "w") as f:
        for name in which:
            _log(f"[suite] {name} ...")
            res = fns[name](R, ctx, seed=seed)
            _log(f"[suite] {json.dumps(res)}")
            f.write(json.dumps(res) + "\n")
            f.flush()
    ctx.close()


if __name__ == "__main__":
    import argparse

    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default="results/bench_suite.json")
    ap.add_argument("--only", nargs="*")
    a = ap.parse_args()
    run_all(a.out, which=tuple(a.only) if a.only else
            ("single_env_f64", "uniform_4096x4", "uneven_8192", "rollout_waypoint_noise",
             "rollout_predator_prey", "serving"))
