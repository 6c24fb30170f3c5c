"""GPU tests of env_steps, the persistent form of env_step (Sec. 4.1, the
step of every robot; several steps per launch with the state held on chip):
equal to the same number of env_step calls bit for bit in both precisions and
scenarios, resets included, and a single FP64 env on the oracle's trajectory.
"""
import numpy as np
import pytest

from paper_2505_06771_amd import synth
from tests.gpu_util import banner, batch_from_states, ctx_and_lib, host

pytestmark = pytest.mark.gpu


def _states(seed, E, n):
    a = synth.random_states(seed, E - E // 2, n)
    b = synth.stressed_states(seed + 1, E // 2, n, "mixed")
    return {k: np.concatenate([a[k], b[k]]) for k in a}


@pytest.mark.parametrize("kind,n,scenario,controller", [
    ("f32", 4, 0, 0), ("f32", 8, 0, 0), ("f32", 12, 0, 2), ("f32", 3, 1, 2), ("f32", 8, 1, 2),
    ("f64", 2, 0, 0), ("f64", 4, 0, 1), ("f64", 8, 0, 3)])
def test_env_steps_equals_repeated_env_step(kind, n, scenario, controller):
    import torch

    R, ctx = ctx_and_lib()
    tdt = torch.float32 if kind == "f32" else torch.float64
    E, K, t0 = 200, 40, 100
    st = _states(20 + n, E, n)
    max_steps = 100 if scenario == R.RS_SCN_PREDATOR_PREY else 500
    # step counters close to the limit: resets fall inside the window
    step0 = np.random.default_rng(n).integers(max_steps - 30, max_steps, E).astype(np.int32)
    kw = dict(seed=5, scenario=scenario, controller=controller, max_steps=max_steps,
              dtype=R.RS_F64 if kind == "f64" else R.RS_F32)
    if controller == R.RS_CTRL_WAYPOINT:
        kw["action_noise"] = 0.05
    p = R.params(**kw)
    b1 = batch_from_states(R, st, n, tdt, env_id_base=7, step=step0)
    b2 = batch_from_states(R, st, n, tdt, env_id_base=7, step=step0)
    D = 2 * n + 4
    rew1 = torch.zeros((K, E), dtype=tdt, device="cuda")
    done1 = torch.zeros((K, E), dtype=torch.uint8, device="cuda")
    obs1 = torch.zeros(E * n * D, dtype=tdt, device="cuda")
    qs1 = torch.zeros((E, R.QPS_COUNT), dtype=torch.int32, device="cuda")
    banner(f"env_steps {kind} n={n} scenario={scenario} controller={controller}")
    R.env_steps(ctx, p, b1, K, t_global0=t0, reward=rew1, done=done1, obs_final=obs1,
                qp_stats=qs1)
    rew2 = torch.zeros((K, E), dtype=tdt, device="cuda")
    done2 = torch.zeros((K, E), dtype=torch.uint8, device="cuda")
    obs2 = torch.zeros(E * n * D, dtype=tdt, device="cuda")
    qs2 = torch.zeros((E, R.QPS_COUNT), dtype=torch.int32, device="cuda")
    for k in range(K):
        R.env_step(ctx, p, b2, t_global=t0 + k, obs=obs2, reward=rew2[k], done=done2[k],
                   qp_stats=qs2)
    torch.cuda.synchronize()
    assert int(host(done1).sum()) > 0, "the window should contain resets"
    for a1, a2 in ((b1.x, b2.x), (b1.y, b2.y), (b1.theta, b2.theta), (b1.goal_x, b2.goal_x),
                   (b1.goal_y, b2.goal_y), (b1.step, b2.step), (b1.episode, b2.episode),
                   (rew1, rew2), (done1, done2), (obs1, obs2), (qs1, qs2)):
        np.testing.assert_array_equal(host(a1), host(a2))


def test_env_steps_single_env_f64_on_the_oracle_trajectory(orc):
    """1 env, N = 4, proportional go-to-goal controller, FP64, 1000 steps in
    one launch without resets: the final poses stay on the oracle's."""
    import torch

    R, ctx = ctx_and_lib()
    n = 4
    po = orc.Params(controller=1, goal_radius=0.0, max_steps=0, seed=0)
    x, y, th, gx, gy = orc.reset_env(po, 0, 0, n)
    st = {"x": x[None].copy(), "y": y[None].copy(), "th": th[None].copy(),
          "gx": gx[None].copy(), "gy": gy[None].copy()}
    b = batch_from_states(R, st, n, torch.float64)
    p = R.params(controller=R.RS_CTRL_GOTO, goal_radius=0.0, max_steps=0, dtype=R.RS_F64)
    ref = {"x": x.copy(), "y": y.copy(), "th": th.copy(), "gx": gx.copy(), "gy": gy.copy(),
           "step": 0, "episode": 0}
    rew = torch.zeros((1000, 1), dtype=torch.float64, device="cuda")
    banner("env_steps goto f64 1000 steps")
    R.env_steps(ctx, p, b, 1000, t_global0=0, reward=rew)
    rref = np.zeros(1000)
    for t in range(1000):
        out = orc.env_step(po, ref, 0, t)
        rref[t] = out["reward"]
    torch.cuda.synchronize()
    gap = max(np.abs(host(b.x) - ref["x"]).max(), np.abs(host(b.y) - ref["y"]).max())
    print(f"env_steps f64 worst final position gap {gap:.3g}")
    assert gap < 1e-9
    assert int(host(b.step)[0]) == 1000
    np.testing.assert_allclose(host(rew)[:, 0], rref, atol=4e-9, rtol=0)


def test_env_steps_arguments():
    import torch

    R, ctx = ctx_and_lib()
    b = R.Batch.empty(4, 4)
    R.env_reset(ctx, R.params(), b)
    before = host(b.x).copy()
    R.env_steps(ctx, R.params(), b, 0)  # nothing to do
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host(b.x), before)
    with pytest.raises(R.RobostepError):
        R.env_steps(ctx, R.params(), b, -1)
    with pytest.raises(R.RobostepError):
        R.env_steps(ctx, R.params(dt=-1.0), b, 3)
    with pytest.raises(R.RobostepError):
        R.env_steps(ctx, R.params(), R.Batch.empty(4, 17), 3)
