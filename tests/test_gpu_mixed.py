"""GPU tests of mixed-size batches: env_reset_mixed, env_run (one persistent
launch over envs with different robot counts), schedule independence and the
autotuner.

Parity: one env_run step is compared with the FP64 oracle teacher-forced
(tolerances as in test_gpu_step); a k-step env_run equals k one-step launches
bit for bit; results are identical under every schedule (lanes per env,
block size) and for an env alone or inside a mixed batch.
"""
import ctypes

import numpy as np
import pytest

from paper_2505_06771_amd import synth
from tests.gpu_util import angle_diff, banner, ctx_and_lib, dev, host, pose_band

pytestmark = pytest.mark.gpu


def _mixed_batch(R, ctx, counts, seed, env_id_base=0, schedule=None):
    import torch

    plan = R.Plan(ctx, counts, schedule)
    b = R.Batch.empty(len(counts), 0, env_id_base=env_id_base, total_robots=plan.total_robots)
    b.robots = 0
    R.env_reset_mixed(ctx, R.params(seed=seed), plan, b)
    return plan, b


def _offsets(counts):
    return np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)


def test_reset_mixed_matches_oracle(orc):
    import torch

    R, ctx = ctx_and_lib()
    counts = synth.uneven_sizes(1, 157)
    banner("reset mixed")
    plan, b = _mixed_batch(R, ctx, counts, seed=4, env_id_base=10)
    torch.cuda.synchronize()
    off = _offsets(counts)
    x, th = host(b.x), host(b.theta)
    po = orc.Params(seed=4)
    for e, n in enumerate(counts):
        ox, oy, oth, ogx, ogy = orc.reset_env(po, 10 + e, 0, int(n))
        np.testing.assert_array_equal(x[off[e]:off[e + 1]], ox.astype(np.float32))
        assert angle_diff(th[off[e]:off[e + 1]], oth).max() <= 1e-6


@pytest.mark.parametrize("extra", [{}, {"controller": 2, "action_noise": 0.05},
                                   {"controller": 3, "action_noise": 0.05}],
                         ids=["discrete", "waypoint_noise", "pose_noise"])
def test_env_run_one_step_teacher_forced(orc, extra):
    import torch

    R, ctx = ctx_and_lib()
    counts = synth.uneven_sizes(2, 211)
    E = len(counts)
    plan, b = _mixed_batch(R, ctx, counts, seed=6)
    # push the step counters near the time limit so resets happen
    b.step.copy_(torch.from_numpy(np.random.default_rng(0).integers(490, 500, E).astype(np.int32)).cuda())
    off = _offsets(counts)
    po = orc.Params(seed=6, **extra)
    p = R.params(seed=6, **extra)
    rew = torch.zeros(E, device="cuda")
    done = torch.zeros(E, dtype=torch.uint8, device="cuda")
    total_obs = sum(int(n) * (2 * int(n) + 4) for n in counts)
    obs = torch.zeros(total_obs, device="cuda")
    banner("env_run teacher forced")
    resets = 0
    for t in range(15):
        before = {k: host(getattr(b, a)).astype(np.float64) for k, a in
                  (("x", "x"), ("y", "y"), ("th", "theta"), ("gx", "goal_x"), ("gy", "goal_y"))}
        st0, ep0 = host(b.step).copy(), host(b.episode).copy()
        R.env_run(ctx, p, plan, b, 1, t_global0=300 + t, reward_out=rew, done_out=done,
                  obs_final=obs)
        torch.cuda.synchronize()
        gx_, gy_, gth = host(b.x), host(b.y), host(b.theta)
        gob, grw, gdn = host(obs), host(rew), host(done)
        for e, n in enumerate(counts):
            n = int(n)
            sl = slice(off[e], off[e + 1])
            one = {k: v[sl].copy() for k, v in before.items()}
            one["step"], one["episode"] = int(st0[e]), int(ep0[e])
            acts = [orc.random_action(po, e, 300 + t, i) for i in range(n)]
            if pose_band(po, one["th"], acts).any():
                continue  # pose controller: goal bearing at +-pi
            out = orc.env_step(po, one, e, 300 + t)
            assert out["status"] != 2
            assert out["done"] == gdn[e]
            resets += out["done"]
            assert np.abs(one["x"] - gx_[sl]).max() <= 1e-5
            assert np.abs(one["y"] - gy_[sl]).max() <= 1e-5
            assert angle_diff(one["th"], gth[sl]).max() <= 6.6e-5
            assert abs(out["reward"] - grw[e]) <= n * 1e-5
            o0 = plan.obs_offset(e)
            np.testing.assert_allclose(gob[o0:o0 + n * (2 * n + 4)].reshape(n, 2 * n + 4),
                                       out["obs"], atol=1e-5, rtol=0)
    assert resets > E // 2


def _run_steps(R, ctx, counts, seed, steps, schedule=None, chunks=1, env_id_base=0):
    import torch

    plan, b = _mixed_batch(R, ctx, counts, seed, env_id_base=env_id_base, schedule=schedule)
    p = R.params(seed=seed)
    E = len(counts)
    rsum = torch.zeros(E, device="cuda")
    per = steps // chunks
    for k in range(chunks):
        R.env_run(ctx, p, plan, b, per, t_global0=k * per, reward_sum=rsum)
    torch.cuda.synchronize()
    return host(b.x).copy(), host(b.theta).copy(), host(rsum).copy(), plan


def test_multi_step_equals_single_steps():
    R, ctx = ctx_and_lib()
    counts = synth.uneven_sizes(3, 300)
    banner("env_run chunking")
    a = _run_steps(R, ctx, counts, 9, 40, chunks=1)
    b = _run_steps(R, ctx, counts, 9, 40, chunks=40)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    np.testing.assert_allclose(a[2], b[2], rtol=1e-6, atol=1e-5)  # summation order differs


def test_schedule_independence():
    R, ctx = ctx_and_lib()
    counts = synth.uneven_sizes(4, 260)
    banner("schedules")
    ref = _run_steps(R, ctx, counts, 12, 25)
    for blk, wide, div in [(64, False, 1), (128, True, 1), (256, True, 1), (256, False, 4),
                           (128, False, 64)]:
        s = R.RsSchedule()
        s.block_threads = blk
        for n in range(2, 17):
            g = 2
            while g < n:
                g *= 2
            s.lanes_per_env[n] = min(16, 2 * g) if wide else g
            s.envs_per_wave[n] = max(1, (64 // s.lanes_per_env[n]) // div)
        got = _run_steps(R, ctx, counts, 12, 25, schedule=s)
        np.testing.assert_array_equal(got[0], ref[0])
        np.testing.assert_array_equal(got[1], ref[1])
        np.testing.assert_array_equal(got[2], ref[2])


def test_env_alone_equals_env_in_mix():
    R, ctx = ctx_and_lib()
    mix = synth.uneven_sizes(5, 120)
    # last 20 envs have 8 robots: run them alone with the same env ids
    counts = np.concatenate([mix, np.full(20, 8, np.int32)])
    banner("alone vs mix")
    a = _run_steps(R, ctx, counts, 21, 30)
    alone = _run_steps(R, ctx, np.full(20, 8, np.int32), 21, 30, env_id_base=len(mix))
    off = int(np.sum(mix))
    np.testing.assert_array_equal(a[0][off:], alone[0])
    np.testing.assert_array_equal(a[2][len(mix):], alone[2])


def test_autotune_returns_valid_schedule():
    R, ctx = ctx_and_lib()
    banner("autotune")
    s = R.autotune(ctx, R.params(), [4, 8], envs=512, steps=20, tol=1e-4)
    for n in (4, 8):
        g = s.lanes_per_env[n]
        assert g >= n and g in (4, 8, 16)
        assert s.qp_iters[n] in (2 * n + 4, 4 * n + 8, 8 * n + 32)
        assert 1 <= s.envs_per_wave[n] <= 64 // g
    assert s.block_threads in (64, 128, 256)


def test_autotuned_schedule_matches_oracle(orc):
    """The schedule the autotuner picks (its candidates are rejected when a
    certificate reaches the iteration cap) steps stressed mixed batches like
    the oracle: one env_run step at a time, teacher-forced, commands exact to
    the tolerances of the env_step tests, no capped solve."""
    import torch

    R, ctx = ctx_and_lib()
    sizes = [4, 8, 12]
    banner("autotune vs oracle")
    s = R.autotune(ctx, R.params(), sizes, envs=256, steps=20, tol=1e-4)
    counts = np.array([sizes[k % 3] for k in range(150)], np.int32)
    plan = R.Plan(ctx, counts, s)
    E = len(counts)
    off = _offsets(counts)
    b = R.Batch.empty(E, 0, env_id_base=0, total_robots=plan.total_robots)
    b.robots = 0
    fields = {k: np.zeros(plan.total_robots) for k in ("x", "y", "th", "gx", "gy")}
    for e, n in enumerate(counts):
        kind = "cluster" if e % 2 else "mixed"
        st = synth.stressed_states(500 + e, 1, int(n), kind)
        for k in fields:
            fields[k][off[e]:off[e + 1]] = st[k][0]
    for k, a in (("x", "x"), ("y", "y"), ("th", "theta"), ("gx", "goal_x"), ("gy", "goal_y")):
        getattr(b, a).copy_(torch.from_numpy(fields[k].astype(np.float32)).cuda())
    po = orc.Params(seed=4)
    p = R.params(seed=4)
    qs = torch.zeros((E, R.QPS_COUNT), dtype=torch.int32, device="cuda")
    ctx.qp_failures(reset=True)
    for t in range(6):
        before = {k: host(getattr(b, a)).astype(np.float64) for k, a in
                  (("x", "x"), ("y", "y"), ("th", "theta"), ("gx", "goal_x"), ("gy", "goal_y"))}
        st0, ep0 = host(b.step).copy(), host(b.episode).copy()
        R.env_run(ctx, p, plan, b, 1, t_global0=t, qp_stats=qs)
        torch.cuda.synchronize()
        gx_, gy_, gth = host(b.x), host(b.y), host(b.theta)
        for e, n in enumerate(counts):
            sl = slice(off[e], off[e + 1])
            one = {k: v[sl].copy() for k, v in before.items()}
            one["step"], one["episode"] = int(st0[e]), int(ep0[e])
            out = orc.env_step(po, one, e, t)
            assert out["status"] != 2
            assert np.abs(one["x"] - gx_[sl]).max() <= 1e-5
            assert np.abs(one["y"] - gy_[sl]).max() <= 1e-5
            assert angle_diff(one["th"], gth[sl]).max() <= 6.6e-5
    q = host(qs)
    assert q[:, R.QPS_CAPPED].sum() == 0 and ctx.qp_failures()[1] == 0
    assert q[:, R.QPS_ACTIVE_SET:R.QPS_GENERAL + 1].sum() > 0
    print("tuned schedule:", {n: (s.lanes_per_env[n], s.qp_iters[n]) for n in sizes},
          "block", s.block_threads, "stages", q[:, :R.QPS_ITERATIONS].sum(axis=0).tolist())


def test_autotune_on_the_callers_batch_leaves_it_unchanged():
    import torch

    R, ctx = ctx_and_lib()
    counts = synth.uneven_sizes(7, 400)
    banner("autotune_batch")
    plan, b = _mixed_batch(R, ctx, counts, seed=3)
    before = [host(getattr(b, a)).copy() for a in ("x", "y", "theta", "step", "episode")]
    s = R.autotune_batch(ctx, R.params(seed=3), plan, b, steps=20, tol=1e-4)
    torch.cuda.synchronize()
    after = [host(getattr(b, a)) for a in ("x", "y", "theta", "step", "episode")]
    for u, v in zip(before, after):
        np.testing.assert_array_equal(u, v)
    for n in sorted(set(counts.tolist())):
        g = s.lanes_per_env[n]
        assert g >= n and g in (2, 4, 8, 16)
        assert 1 <= s.envs_per_wave[n] <= 64 // g
        assert s.qp_iters[n] in (2 * n + 4, 4 * n + 8, 8 * n + 32)
    got = R.RsSchedule()
    R.lib().rs_get_schedule(ctx.handle, ctypes.byref(got))
    assert got.block_threads == s.block_threads
