"""GPU parity of the Predator-Prey scenario (env_reset, env_step, the
mixed-size env_reset_mixed / env_run and, in test_gpu_rollout, the fused
rollout) against the FP64 oracle, teacher-forced: every step starts both sides
from the GPU's state.

Tolerances as in the Navigation tests (FP32: positions 1e-5 m, heading
6.6e-5 rad, observations 1e-5; FP64: 1e-9). Decisions taken in floating
point are exact outside a band: the prey's choice may differ only where the
GPU's candidate scores within 1e-5 m^2 of the oracle's best (a near-tie), and
the tag reward only where some centre is within 1e-5 m of the tag radius;
band cases must stay rare. Episode ends (step limit) and reset draws are
exact.
"""
import numpy as np
import pytest

from paper_2505_06771_amd import synth
from tests.gpu_util import angle_diff, banner, batch_from_states, ctx_and_lib, host, \
    oracle_state, prey_band, tag_band

pytestmark = pytest.mark.gpu


def _pp_states(seed, E, n):
    a = synth.random_states(seed, E - E // 2, n)
    b = synth.stressed_states(seed + 1, E // 2, n, "mixed")
    st = {k: np.concatenate([a[k], b[k]]) for k in a}
    # one prey per env, in every goal slot: near the robots for half the envs
    rng = np.random.default_rng(seed + 2)
    qx = np.where(np.arange(E) % 2 == 0, st["x"][:, 0] + rng.uniform(-0.3, 0.3, E),
                  rng.uniform(-1.4, 1.4, E))
    qy = np.where(np.arange(E) % 2 == 0, st["y"][:, 0] + rng.uniform(-0.3, 0.3, E),
                  rng.uniform(-0.85, 0.85, E))
    st["gx"] = np.repeat(np.clip(qx, -1.5, 1.5)[:, None], n, axis=1)
    st["gy"] = np.repeat(np.clip(qy, -0.9, 0.9)[:, None], n, axis=1)
    return st


@pytest.mark.parametrize("kind", ["f32", "f64"])
@pytest.mark.parametrize("n", [3, 8])
def test_pp_reset_parity(orc, n, kind):
    import torch

    R, ctx = ctx_and_lib()
    tdt, ndt = (torch.float32, np.float32) if kind == "f32" else (torch.float64, np.float64)
    E = 120
    b = R.Batch.empty(E, n, dtype=tdt, env_id_base=300)
    b.episode.copy_(torch.arange(E, dtype=torch.int32, device="cuda") % 4)
    p = R.params(scenario=R.RS_SCN_PREDATOR_PREY, seed=21,
                 dtype=R.RS_F64 if kind == "f64" else R.RS_F32)
    po = orc.Params(scenario=1, seed=21)
    banner(f"pp reset n={n} {kind}")
    R.env_reset(ctx, p, b)
    torch.cuda.synchronize()
    gx, gy, x = (host(a).reshape(E, n) for a in (b.goal_x, b.goal_y, b.x))
    for e in range(E):
        ox, oy, oth, ogx, ogy = orc.reset_env(po, 300 + e, e % 4, n)
        np.testing.assert_array_equal(x[e], ox.astype(ndt))
        np.testing.assert_array_equal(gx[e], ogx.astype(ndt))
        np.testing.assert_array_equal(gy[e], ogy.astype(ndt))
        assert (gx[e] == gx[e, 0]).all()


def _pp_step_compare(orc, po, R, ctx, p, b, n, steps, t0, tol):
    import torch

    E = b.num_envs
    tdt = b.x.dtype
    obs = torch.zeros(E * n * (2 * n + 4), dtype=tdt, device="cuda")
    rew = torch.zeros(E, dtype=tdt, device="cuda")
    done = torch.zeros(E, dtype=torch.uint8, device="cuda")
    stats = {"tags": 0, "resets": 0, "band_prey": 0, "band_tag": 0, "decisions": 0}
    for t in range(steps):
        before = oracle_state(b)
        R.env_step(ctx, p, b, t_global=t0 + t, obs=obs, reward=rew, done=done)
        torch.cuda.synchronize()
        after = oracle_state(b)
        ref = {k: v.copy() for k, v in before.items()}
        out = orc.env_step_batch(po, n, ref, b.env_id_base, t0 + t, want_obs=True)
        assert out["status"] != 2
        np.testing.assert_array_equal(host(done), out["done"])  # step limit: exact
        np.testing.assert_array_equal(after["step"], ref["step"])
        np.testing.assert_array_equal(after["episode"], ref["episode"])
        grw = host(rew).astype(np.float64)
        gob = host(obs).reshape(E, n, 2 * n + 4).astype(np.float64)
        stats["resets"] += int(out["done"].sum())
        for e in range(E):
            sl = slice(e * n, (e + 1) * n)
            stats["decisions"] += 1
            dxy = max(np.abs(after["x"][sl] - ref["x"][sl]).max(),
                      np.abs(after["y"][sl] - ref["y"][sl]).max())
            assert dxy <= tol["xy"], f"t={t} e={e}: robot gap {dxy}"
            assert angle_diff(after["th"][sl], ref["th"][sl]).max() <= tol["th"]
            gq = (after["gx"][e * n], after["gy"][e * n])
            assert (after["gx"][sl] == gq[0]).all() and (after["gy"][sl] == gq[1]).all()
            dq = max(abs(gq[0] - ref["gx"][e * n]), abs(gq[1] - ref["gy"][e * n]))
            if dq > tol["xy"]:
                assert not out["done"][e], f"t={t} e={e}: reset prey differs"
                assert prey_band(orc, po, before["x"][sl], before["y"][sl], before["gx"][e * n],
                                 before["gy"][e * n], *gq), f"t={t} e={e}: prey gap {dq}"
                stats["band_prey"] += 1
                continue
            if grw[e] != out["reward"][e]:
                assert not out["done"][e]
                assert tag_band(po, ref["x"][sl], ref["y"][sl], ref["gx"][e * n],
                                ref["gy"][e * n]), f"t={t} e={e}: tag reward differs"
                stats["band_tag"] += 1
            stats["tags"] += int(out["reward"][e] > 0)
            assert np.abs(gob[e] - out["obs"][e]).max() <= tol["obs"], f"t={t} e={e}: obs"
    return stats


@pytest.mark.parametrize("kind,n,controller", [("f32", 3, 2), ("f32", 8, 2), ("f32", 8, 0),
                                               ("f64", 5, 2)])
def test_pp_env_step_teacher_forced(orc, kind, n, controller):
    import torch

    R, ctx = ctx_and_lib()
    tdt = torch.float32 if kind == "f32" else torch.float64
    E = 97
    st = _pp_states(400 + n, E, n)
    rng = np.random.default_rng(n)
    step0 = rng.integers(80, 100, E).astype(np.int32)  # 100-step episodes end in the run
    b = batch_from_states(R, st, n, tdt, env_id_base=700, step=step0,
                          episode=rng.integers(0, 3, E).astype(np.int32))
    kw = dict(scenario=1, controller=controller, max_steps=100, seed=5)
    p = R.params(dtype=R.RS_F64 if kind == "f64" else R.RS_F32, **kw)
    po = orc.Params(**kw)
    tol = ({"xy": 1e-5, "th": 6.6e-5, "obs": 1e-5} if kind == "f32"
           else {"xy": 1e-9, "th": 1e-9, "obs": 1e-9})
    banner(f"pp env_step {kind} n={n} controller={controller}")
    s = _pp_step_compare(orc, po, R, ctx, p, b, n, steps=30, t0=10, tol=tol)
    print(s)
    assert s["resets"] >= E // 2 and s["tags"] > 0
    assert s["band_prey"] + s["band_tag"] <= max(2, 0.005 * s["decisions"])


def test_pp_prey_flees_on_the_gpu(orc):
    """Hand-built: one tagger due west of the prey, robots standing still; the
    prey steps due east by prey_speed * dt every step."""
    import torch

    R, ctx = ctx_and_lib()
    n, E = 2, 4
    x = np.tile([[-0.5, -1.2]], (E, 1))
    y = np.tile([[0.0, 0.8]], (E, 1))
    st = {"x": x, "y": y, "th": np.zeros((E, n)), "gx": np.full((E, n), 0.0),
          "gy": np.full((E, n), 0.0)}
    b = batch_from_states(R, st, n, torch.float64)
    p = R.params(scenario=R.RS_SCN_PREDATOR_PREY, max_steps=0, dtype=R.RS_F64)
    acts = torch.zeros(E * n, dtype=torch.uint8, device="cuda")
    banner("pp flee")
    for t in range(5):
        R.env_step(ctx, p, b, actions=acts, t_global=t)
    torch.cuda.synchronize()
    s = p.prey_speed * p.dt
    np.testing.assert_allclose(host(b.goal_x), 5 * s, rtol=0, atol=1e-15)
    np.testing.assert_allclose(host(b.goal_y), 0.0, rtol=0, atol=1e-15)


def test_pp_mixed_batch_env_run(orc):
    """Mixed-size batch: env_reset_mixed puts the prey at the first goal draw
    of every env; then one env_run step at a time is compared with the oracle
    (teacher-forced, bands as above)."""
    import torch

    R, ctx = ctx_and_lib()
    counts = synth.uneven_sizes(7, 120)
    E = len(counts)
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    kw = dict(scenario=1, controller=2, max_steps=100, seed=8)
    p = R.params(**kw)
    po = orc.Params(**kw)
    plan = R.Plan(ctx, counts, None)
    b = R.Batch.empty(E, 0, total_robots=plan.total_robots)
    b.robots = 0
    banner("pp mixed env_run")
    R.env_reset_mixed(ctx, p, plan, b)
    torch.cuda.synchronize()
    gx0 = host(b.goal_x)
    for e, n in enumerate(counts):
        ogx = orc.reset_env(po, e, 0, int(n))[3]
        np.testing.assert_array_equal(gx0[off[e]:off[e + 1]], ogx.astype(np.float32))
    b.step.copy_(torch.from_numpy(np.random.default_rng(3).integers(90, 100, E).astype(np.int32)).cuda())
    rew = torch.zeros(E, device="cuda")
    done = torch.zeros(E, dtype=torch.uint8, device="cuda")
    stats = {"tags": 0, "resets": 0, "band": 0}
    for t in range(12):
        before = {k: host(getattr(b, a)).astype(np.float64) for k, a in
                  (("x", "x"), ("y", "y"), ("th", "theta"), ("gx", "goal_x"), ("gy", "goal_y"))}
        st0, ep0 = host(b.step).copy(), host(b.episode).copy()
        R.env_run(ctx, p, plan, b, 1, t_global0=40 + t, reward_out=rew, done_out=done)
        torch.cuda.synchronize()
        ax, ay, ath, agx = host(b.x), host(b.y), host(b.theta), host(b.goal_x)
        grw, gdn = host(rew), host(done)
        for e, n in enumerate(counts):
            n = int(n)
            sl = slice(off[e], off[e + 1])
            one = {k: v[sl].copy() for k, v in before.items()}
            one["step"], one["episode"] = int(st0[e]), int(ep0[e])
            out = orc.env_step(po, one, e, 40 + t)
            assert out["status"] != 2
            assert out["done"] == gdn[e]
            stats["resets"] += out["done"]
            assert np.abs(one["x"] - ax[sl]).max() <= 1e-5
            assert np.abs(one["y"] - ay[sl]).max() <= 1e-5
            assert angle_diff(one["th"], ath[sl]).max() <= 6.6e-5
            if abs(one["gx"][0] - agx[off[e]]) > 1e-5:
                assert prey_band(orc, po, before["x"][sl], before["y"][sl], before["gx"][sl][0],
                                 before["gy"][sl][0], agx[off[e]], host(b.goal_y)[off[e]])
                stats["band"] += 1
                continue
            if out["reward"] != grw[e]:
                assert tag_band(po, one["x"], one["y"], one["gx"][0], one["gy"][0])
                stats["band"] += 1
            stats["tags"] += int(out["reward"] > 0)
    print(stats)
    assert stats["resets"] >= E // 2 and stats["tags"] > 0 and stats["band"] <= 3
