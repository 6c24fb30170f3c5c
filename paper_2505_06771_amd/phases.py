"""Where the fused rollout's time goes, per phase of its step loop.

    python -m paper_2505_06771_amd.build --phase-timers   # librobostep_timers.so
    python -m paper_2505_06771_amd.phases [--launches 8] [--envs 16384] [--robots 8] [--horizon 128]
    python -m paper_2505_06771_amd.phases --stages   # certificate stages, product library

Runs the policy rollout of the benchmark (seeded synthetic weights, discrete
moves, all envs reset together at the start) with the diagnostic library,
whose step loop reads the shader clock at its phase boundaries and adds each
phase's cycles to per-wavefront counters. Per launch it prints the launch
time, the mean cycles per wavefront-step of each phase, the spread of the
wavefronts' totals and the least-squares slope of a wavefront's total on its
number of steps with an active-set loop solve (the cost of such a step);
then one JSON line over all launches. The product library carries none of
this code.

With --stages it runs the same launches with the product library instead and
its in-kernel certificate counters (the qp_stats output of the rollout, a
separately compiled counting variant of the kernel): the share of env-steps
whose command each stage of the certificate produced, and the active-set
iterations per loop solve.
"""
from __future__ import annotations

import argparse
import json
import os
import sys

NAMES = ["obs", "mlp", "sample", "pre", "qp", "post", "loop_steps", "total"]


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--launches", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--envs", type=int, default=16384)
    ap.add_argument("--robots", type=int, default=8)
    ap.add_argument("--horizon", type=int, default=128)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--stages", action="store_true")
    args = ap.parse_args(argv)

    import numpy as np
    import torch

    from paper_2505_06771_amd import build as B
    from paper_2505_06771_amd import robostep as R
    from paper_2505_06771_amd import synth

    if not args.stages:
        if not os.path.exists(B.LIB_TIMERS):
            raise RuntimeError(f"{B.LIB_TIMERS} is missing: build it with "
                               "python -m paper_2505_06771_amd.build --phase-timers")
        R.use_library(B.LIB_TIMERS)
    assert torch.cuda.is_available(), "the phase timers need a GPU"
    E, n, H = args.envs, args.robots, args.horizon
    if not 2 <= n <= 14:
        raise SystemExit("the rollout takes 2..14 robots")
    G = 1 << (n - 1).bit_length()  # lanes per env
    if E * G % 256:
        raise SystemExit("envs x lanes per env must fill whole 256-lane blocks")
    waves = E * G // 64
    D = 2 * n + 4
    ctx = R.Context(0)
    p = R.params(seed=args.seed)
    b = R.Batch.empty(E, n)
    R.env_reset(ctx, p, b)
    w = synth.policy_weights(args.seed, D)
    bf = lambda a: torch.from_numpy(a).to(torch.bfloat16).cuda().contiguous()
    fl = lambda a: torch.from_numpy(a).float().cuda().contiguous()
    pol = R.Policy(bf(w["w1"]), fl(w["b1"]), bf(w["w2"]), fl(w["b2"]), bf(w["w3"]), fl(w["b3"]))
    obs = torch.empty(H * E * n * D, device="cuda")
    act = torch.empty(H * E * n, dtype=torch.uint8, device="cuda")
    rew = torch.empty(H * E, device="cuda")
    done = torch.empty(H * E, dtype=torch.uint8, device="cuda")
    for k in range(args.warmup):
        R.rollout(ctx, p, b, pol, H, k * H, obs, act, rew, done)
    torch.cuda.synchronize()
    if args.stages:
        return stages(R, ctx, p, b, pol, obs, act, rew, done, args)
    allP, ms = [], []
    for k in range(args.launches):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        R.rollout(ctx, p, b, pol, H, (args.warmup + k) * H, obs, act, rew, done)
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
        P = ctx.phase_cycles(waves).astype(np.float64)
        allP.append(P)
        tot, ls = P[:, 7], P[:, 6]
        slope = np.polyfit(ls, tot, 1)[0] if ls.std() > 0 else float("nan")
        mean = P.mean(axis=0) / H
        print(f"launch {k}: {ms[-1]:.3f} ms | per wavefront-step "
              + " ".join(f"{nm} {mean[j]:.0f}" for j, nm in enumerate(NAMES) if j != 6)
              + f" | slowest total / mean {tot.max() / tot.mean():.2f}"
              + f" | loop-solve steps per wavefront mean {ls.mean():.2f} max {ls.max():.0f}"
              + f" | total = a + {slope:.0f} x loop-solve steps", flush=True)
    P = np.concatenate(allP)
    tot = P[:, 7]
    q = np.quantile(tot, [0.5, 0.9, 0.99, 1.0]) / tot.mean()
    mean = P.mean(axis=0) / H
    summary = {
        "envs": E, "robots": n, "horizon": H, "launches": args.launches, "warmup": args.warmup,
        "ms_mean": float(np.mean(ms)),
        "cycles_per_wavefront_step": {nm: round(float(mean[j])) for j, nm in enumerate(NAMES) if j != 6},
        "share": {nm: round(float(mean[j] / mean[7]), 3) for j, nm in enumerate(NAMES) if j not in (6, 7)},
        "wavefront_total_over_mean_p50_p90_p99_max": [round(float(x), 3) for x in q],
        "loop_solve_steps_per_wavefront_mean": round(float(P[:, 6].mean()), 2),
        "loop_solve_steps_per_wavefront_max": int(P[:, 6].max()),
    }
    print(json.dumps(summary), flush=True)
    ctx.close()


STAGES = ["box", "one_row", "two_rows", "shared_robot", "active_set", "general", "infeasible",
          "capped"]


def stages(R, ctx, p, b, pol, obs, act, rew, done, args):
    """Certificate stage shares over the launches, from the in-kernel counters."""
    import numpy as np
    import torch

    E, H = args.envs, args.horizon
    qs = torch.zeros((E, R.QPS_COUNT), dtype=torch.int32, device="cuda")
    per_launch = []
    for k in range(args.launches):
        qs.zero_()
        R.rollout(ctx, p, b, pol, H, (args.warmup + k) * H, obs, act, rew, done, qp_stats=qs)
        torch.cuda.synchronize()
        q = qs.cpu().numpy().astype(np.int64)
        per_launch.append(q)
        tot = q[:, :8].sum()
        loops = q[:, R.QPS_ACTIVE_SET].sum() + q[:, R.QPS_GENERAL].sum()
        per_env = q[:, R.QPS_ACTIVE_SET] + q[:, R.QPS_GENERAL]
        per_wave = per_env.reshape(-1, 64 // (1 << (args.robots - 1).bit_length())).sum(axis=1)
        print(f"launch {k}: env-steps {tot} | " + " ".join(
            f"{nm} {q[:, j].sum() / tot:.4%}" for j, nm in enumerate(STAGES))
            + f" | loop solves {loops}, per env max {int(per_env.max())}"
            + f", summed over the envs of a wavefront max {int(per_wave.max())}", flush=True)
    Q = np.concatenate(per_launch)
    tot = Q[:, :8].sum()
    loops = Q[:, R.QPS_ACTIVE_SET].sum() + Q[:, R.QPS_GENERAL].sum()
    summary = {
        "envs": E, "robots": args.robots, "horizon": H, "launches": args.launches,
        "warmup": args.warmup, "env_steps": int(tot),
        "share": {nm: float(Q[:, j].sum() / tot) for j, nm in enumerate(STAGES)},
        "loop_solves_per_launch": float(loops / args.launches),
        "iterations_per_loop_solve": float(Q[:, R.QPS_ITERATIONS].sum() / max(loops, 1)),
    }
    print(json.dumps(summary), flush=True)
    ctx.close()


if __name__ == "__main__":
    sys.exit(main())
