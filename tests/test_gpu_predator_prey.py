"""GPU parity of the Predator-Prey scenario (env_reset, env_step, rollout)
against the FP64 oracle, teacher-forced: every step starts both sides from the
GPU's state.

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


def test_pp_is_rejected_where_unsupported():
    R, ctx = ctx_and_lib()
    p = R.params(scenario=R.RS_SCN_PREDATOR_PREY)
    plan = R.Plan(ctx, np.array([3, 4], np.int32))
    b = R.Batch.empty(2, 0, total_robots=plan.total_robots)
    b.robots = 0
    with pytest.raises(R.RobostepError):
        R.env_run(ctx, p, plan, b, 1)
