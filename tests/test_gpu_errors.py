"""Argument errors of the entry points on a live GPU context: every call below
is refused by the entry point's own host-side checks, with a message naming
the problem, before any kernel is launched, and leaves the batch untouched.
Each refused call is otherwise well formed (buffers sized for what it names),
so the test depends only on the checks, not on what a kernel would do."""
import numpy as np
import pytest

from paper_2505_06771_amd import synth
from tests.gpu_util import banner, ctx_and_lib, host

pytestmark = pytest.mark.gpu


def _snap(b):
    return [host(a).copy() for a in (b.x, b.y, b.theta, b.goal_x, b.goal_y, b.step, b.episode)]


def _same(b, before):
    for a, z in zip(_snap(b), before):
        np.testing.assert_array_equal(a, z)


def _policy(R, torch, dim):
    w = synth.policy_weights(0, dim)
    bf = lambda a: torch.from_numpy(a).to(torch.bfloat16).cuda().contiguous()
    fl = lambda a: torch.from_numpy(a).float().cuda().contiguous()
    return R.Policy(bf(w["w1"]), fl(w["b1"]), bf(w["w2"]), fl(w["b2"]), bf(w["w3"]), fl(w["b3"]))


def _rollout_buffers(torch, E, n, H):
    D = 2 * n + 4
    return (torch.zeros(H * E * n * D, device="cuda"),
            torch.zeros(H * E * n, dtype=torch.uint8, device="cuda"),
            torch.zeros(H * E, device="cuda"), torch.zeros(H * E, dtype=torch.uint8, device="cuda"))


def test_env_step_refuses_empty_and_out_of_range_batches():
    R, ctx = ctx_and_lib()
    p = R.params()
    banner("errors env_step batch")
    for E, n, msg in [(0, 4, "num_envs"), (3, 1, "robots"), (3, 17, "robots")]:
        b = R.Batch.empty(E, n)
        with pytest.raises(R.RobostepError, match=msg):
            R.env_step(ctx, p, b, t_global=0)
        with pytest.raises(R.RobostepError, match=msg):
            R.env_reset(ctx, p, b)


def test_env_step_refuses_bad_parameters_and_leaves_the_state():
    R, ctx = ctx_and_lib()
    b = R.Batch.empty(5, 4)
    R.env_reset(ctx, R.params(seed=2), b)
    before = _snap(b)
    banner("errors env_step params")
    for kw, msg in [({"dt": -1.0}, "dt"), ({"v_max": 0.0}, "v_max"),
                    ({"controller": 7}, "controller"), ({"dtype": 5}, "dtype")]:
        with pytest.raises(R.RobostepError, match=msg):
            R.env_step(ctx, R.params(**kw), b, t_global=0)
    _same(b, before)


def test_rollout_refuses_unsupported_configurations():
    import torch

    R, ctx = ctx_and_lib()
    H = 4
    banner("errors rollout")
    # 15 robots: 34 observation features exceed the 32-wide first MLP layer
    b15 = R.Batch.empty(2, 15)
    R.env_reset(ctx, R.params(), b15)
    before = _snap(b15)
    with pytest.raises(R.RobostepError, match="2\\*robots\\+4 <= 32"):
        R.rollout(ctx, R.params(), b15, _policy(R, torch, 34), H, 0,
                  *_rollout_buffers(torch, 2, 15, H))
    _same(b15, before)
    # FP64 parameters, the go-to-goal controller and a policy of the wrong width
    b = R.Batch.empty(3, 8)
    R.env_reset(ctx, R.params(), b)
    before = _snap(b)
    pol = _policy(R, torch, 20)
    for p, msg in [(R.params(dtype=R.RS_F64), "FP32"),
                   (R.params(controller=R.RS_CTRL_GOTO), "samples actions")]:
        with pytest.raises(R.RobostepError, match=msg):
            R.rollout(ctx, p, b, pol, H, 0, *_rollout_buffers(torch, 3, 8, H))
    with pytest.raises(R.RobostepError, match="in_dim"):
        R.rollout(ctx, R.params(), b, _policy(R, torch, 16), H, 0,
                  *_rollout_buffers(torch, 3, 8, H))
    with pytest.raises(R.RobostepError, match="horizon"):
        R.rollout(ctx, R.params(), b, pol, 0, 0, *_rollout_buffers(torch, 3, 8, 1))
    _same(b, before)


def test_env_run_refuses_fp64_and_non_sampling_controllers():
    R, ctx = ctx_and_lib()
    counts = np.array([2, 5, 3, 8], np.int32)
    plan = R.Plan(ctx, counts, None)
    b = R.Batch.empty(len(counts), 0, total_robots=plan.total_robots)
    b.robots = 0
    R.env_reset_mixed(ctx, R.params(seed=4), plan, b)
    before = _snap(b)
    banner("errors env_run")
    with pytest.raises(R.RobostepError, match="FP32"):
        R.env_run(ctx, R.params(dtype=R.RS_F64), plan, b, 3)
    with pytest.raises(R.RobostepError, match="draws actions"):
        R.env_run(ctx, R.params(controller=R.RS_CTRL_GOTO), plan, b, 3)
    _same(b, before)
