#!/usr/bin/env python3
"""Benchmark of the batched Robotarium step on one MI355X.

Default (the headline line): the fused policy rollout, 16384 envs x 8 robots x
128 steps per launch (observation, bf16 MLP on MFMA, sampling, barrier QP,
unicycle step, reward, reset), state resident in HBM. One "step" of the
contract is one rollout launch. Prints ONE JSON line with robot-steps/s, the
roofline of the rollout kernel (HBM-bound: algorithmic bytes / measured kernel
time) and the FP64 CPU oracle timed on a bounded sample of the same workload.

--suite additionally measures the other configurations (single env FP64,
4096 x 4 env_step, mixed-size persistent launch vs per-size launches, serving
vs plain per-request launches) and writes them to --suite-out.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "robot-steps/sec at N=8x16384 envs"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def rollout_algorithmic_bytes(E, N, H):
    """HBM bytes one rollout launch must move: per step the observation
    (2N+4 floats) and action (1 byte) of every robot and reward (4 B) + done
    (1 B) of every env; once per launch the state read and written back
    (5 floats per robot, step and episode per env) and the bf16 weights."""
    D = 2 * N + 4
    per_step = E * N * (4 * D + 1) + E * 5
    state = 2 * (E * N * 20 + E * 8)
    weights = 2 * (D * 64 + 64 * 64 + 64 * 5) + 4 * (64 + 64 + 5)
    return H * per_step + state + weights


def kernel_source_hash():
    """First 16 hex digits of the sha256 of the kernel sources and of the
    build script that holds their compiler flags."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2505_06771_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    with open(os.path.join(ROOT, "paper_2505_06771_amd", "build.py"), "rb") as f:
        h.update(b"build.py")
        h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(E, N, H):
    """HBM bytes per rollout launch from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel calibration),
    if it was taken on the current kernel source and this shape."""
    path = os.path.join(ROOT, "profiles", "rollout_16384x8x128_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != kernel_source_hash() or d.get("shape") != [E, N, H]:
        return None
    return d.get("bytes_per_launch")


def make_policy(R, torch, w):
    bf = lambda a: torch.from_numpy(a).to(torch.bfloat16).cuda().contiguous()
    fl = lambda a: torch.from_numpy(a).float().cuda().contiguous()
    return R.Policy(bf(w["w1"]), fl(w["b1"]), bf(w["w2"]), fl(w["b2"]), bf(w["w3"]), fl(w["b3"]))


def bench_rollout(args):
    import torch

    from paper_2505_06771_amd import robostep as R
    from paper_2505_06771_amd import synth

    E, N, H = args.envs, args.robots, args.horizon
    D = 2 * N + 4
    ctx = R.Context(0)
    p = R.params(seed=args.seed)
    b = R.Batch.empty(E, N)
    R.env_reset(ctx, p, b)
    pol = make_policy(R, torch, synth.policy_weights(args.seed, D))
    obs = torch.empty(H * E * N * D, device="cuda")
    act = torch.empty(H * E * N, dtype=torch.uint8, device="cuda")
    rew = torch.empty(H * E, device="cuda")
    done = torch.empty(H * E, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    for k in range(args.warmup):
        R.rollout(ctx, p, b, pol, H, k * H, obs, act, rew, done, stream=stream)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record(stream)
        R.rollout(ctx, p, b, pol, H, (args.warmup + k) * H, obs, act, rew, done, stream=stream)
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern_ms = [a.elapsed_time(z) for a, z in ev]
    wall = t1 - t0
    robot_steps = E * N * H * args.steps
    avg_ms = sum(kern_ms) / len(kern_ms)
    algo = rollout_algorithmic_bytes(E, N, H)
    achieved = algo / (avg_ms * 1e-3) / 1e9
    traffic = measured_traffic(E, N, H)
    resets = int(done.sum().item())
    log(f"rollout {E}x{N}x{H}: wall {wall * 1e3 / args.steps:.3f} ms/launch, kernel avg "
        f"{avg_ms:.3f} ms (min {min(kern_ms):.3f}), {robot_steps / wall / 1e9:.2f} G robot-steps/s, "
        f"{achieved:.0f} GB/s algorithmic, dones in last launch {resets}")
    ctx.close()
    return {
        "value": robot_steps / wall,
        "ms_per_step": wall * 1e3 / args.steps,
        "kernel_ms": avg_ms,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic},
    }


def cpu_baseline(args):
    """The FP64 oracle on a bounded sample of the same workload (by default
    `cpu_envs` = 4096 of its 16384 envs, 8 robots, all 128 policy steps: about
    20 s of CPU work), threads over envs; the rate is robot-steps per second."""
    import numpy as np

    import oracle as O
    from paper_2505_06771_amd import synth

    N, H, E = args.robots, args.horizon, args.cpu_envs
    threads = min(len(os.sched_getaffinity(0)), 16)
    po = O.Params(seed=args.seed)
    st = {k: np.zeros(E * N) for k in ("x", "y", "th", "gx", "gy")}
    for e in range(E):
        x, y, th, gx, gy = O.reset_env(po, e, 0, N)
        for k, v in zip(("x", "y", "th", "gx", "gy"), (x, y, th, gx, gy)):
            st[k][e * N:(e + 1) * N] = v
    st["step"] = np.zeros(E, np.int32)
    st["episode"] = np.zeros(E, np.int32)
    w = {k: v.astype(np.float64) for k, v in synth.policy_weights(args.seed, 2 * N + 4).items()}
    t0 = time.perf_counter()
    O.rollout(po, N, st, 0, 0, w, H, want_obs=True, nthreads=threads)
    dt = time.perf_counter() - t0
    rate = E * N * H / dt
    log(f"cpu oracle: {E} envs x {N} x {H} steps in {dt:.2f} s on {threads} threads "
        f"-> {rate:.3g} robot-steps/s")
    return {"value": rate, "unit": "robot-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{E} envs x {N} robots x {H} policy steps (FP64), {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--envs", type=int, default=16384)
    ap.add_argument("--robots", type=int, default=8)
    ap.add_argument("--horizon", type=int, default=128)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-envs", type=int, default=4096)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--suite", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--suite-out", default=os.path.join(ROOT, "results", "bench_suite.json"))
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus} GPUs, world size {world}); "
              "environments are independent, so N GPUs would each run this one-GPU workload "
              "on their own share of the envs", file=sys.stderr)
        sys.exit(2)
    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    from paper_2505_06771_amd import robostep as R

    R.lib()  # raises if the HIP library is not built
    res = bench_rollout(args)
    if args.calib_copy:
        src = torch.ones(1 << 28, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: 3 x 1 GiB device-to-device")
    if args.suite:
        from paper_2505_06771_amd import bench_suite

        bench_suite.run_all(args.suite_out, seed=args.seed)
    cpu = None if args.no_cpu else cpu_baseline(args)
    line = {
        "metric": METRIC,
        "value": res["value"],
        "unit": "robot-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"fused policy rollout, {args.envs} envs x {args.robots} robots x "
                               f"{args.horizon} steps per launch (FP32 state, bf16 MLP "
                               f"{2 * args.robots + 4}-64-64-5 on MFMA, exact barrier QP)",
                   "envs": args.envs, "robots": args.robots, "horizon": args.horizon,
                   "parallelism": "single GPU"},
        "roofline": res["roofline"],
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
