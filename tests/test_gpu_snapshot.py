"""GPU: checkpoint and resume. Running 1000 steps is bit-identical to running
500, taking a snapshot, restoring it into a fresh batch and running 500 more
(the stream is counter based, so the snapshot holds the whole state); the
snapshot buffer round-trips a mixed-size batch too."""
import numpy as np
import pytest

from tests.gpu_util import banner, ctx_and_lib, host

pytestmark = pytest.mark.gpu


def _run(R, ctx, p, b, t0, t1, rewards):
    import torch

    E = b.num_envs
    for t in range(t0, t1):
        rew = torch.zeros(E, device="cuda", dtype=b.x.dtype)
        done = torch.zeros(E, dtype=torch.uint8, device="cuda")
        R.env_step(ctx, p, b, t_global=t, reward=rew, done=done)
        rewards.append((host(rew).copy(), host(done).copy()))


@pytest.mark.parametrize("prec,extra", [
    ("f32", {}), ("f64", {}),
    # Predator-Prey with waypoints and action noise: the prey lives in the goal
    # slots and the noise is keyed by the stream time, so the same arrays resume it
    ("f32", {"scenario": 1, "controller": 2, "action_noise": 0.05}),
], ids=["f32", "f64", "f32-predator-prey"])
def test_resume_is_bit_identical(prec, extra):
    import torch

    R, ctx = ctx_and_lib()
    dt = torch.float32 if prec == "f32" else torch.float64
    E, n = 64, 4
    p = R.params(seed=11, dtype=R.RS_F32 if prec == "f32" else R.RS_F64, max_steps=300, **extra)
    banner(f"snapshot {prec} E={E} n={n} {extra}")
    a = R.Batch.empty(E, n, dtype=dt)
    R.env_reset(ctx, p, a)
    b = R.Batch.empty(E, n, dtype=dt)
    R.env_reset(ctx, p, b)
    ra, rb = [], []
    _run(R, ctx, p, a, 0, 1000, ra)
    _run(R, ctx, p, b, 0, 500, rb)
    snap = R.snapshot(ctx, b)
    c = R.Batch.empty(E, n, dtype=dt)
    R.restore(ctx, c, snap)
    _run(R, ctx, p, c, 500, 1000, rb)
    for k in ("x", "y", "theta", "goal_x", "goal_y", "step", "episode"):
        np.testing.assert_array_equal(host(getattr(a, k)), host(getattr(c, k)), err_msg=k)
    assert len(ra) == len(rb)
    for (r1, d1), (r2, d2) in zip(ra, rb):
        np.testing.assert_array_equal(r1, r2)
        np.testing.assert_array_equal(d1, d2)
    assert sum(int(d.sum()) for _, d in ra) > 0  # resets happened across the cut


def test_snapshot_round_trip_mixed_batch():
    R, ctx = ctx_and_lib()
    from paper_2505_06771_amd import synth

    counts = synth.uneven_sizes(3, 96)
    plan = R.Plan(ctx, counts, None)
    p = R.params(seed=4)
    banner("snapshot mixed")
    b = R.Batch.empty(96, 0, total_robots=plan.total_robots)
    R.env_reset_mixed(ctx, p, plan, b)
    R.env_run(ctx, p, plan, b, 37)
    snap = R.snapshot(ctx, b)
    c = R.Batch.empty(96, 0, total_robots=plan.total_robots)
    R.restore(ctx, c, snap)
    for k in ("x", "y", "theta", "goal_x", "goal_y", "step", "episode"):
        np.testing.assert_array_equal(host(getattr(b, k)), host(getattr(c, k)), err_msg=k)
    R.env_run(ctx, p, plan, b, 20, t_global0=37)
    R.env_run(ctx, p, plan, c, 20, t_global0=37)
    np.testing.assert_array_equal(host(b.x), host(c.x))
