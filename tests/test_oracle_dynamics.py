"""Oracle pins: projection-point map, wheel saturation, Euler step, reward,
termination, reset sampler and observation layout, on hand-built states whose
outcome has a closed form."""
import math

import numpy as np
import pytest


def _state(x, y, th, gx, gy, step=0, episode=0):
    return {"x": np.array(x, float), "y": np.array(y, float), "th": np.array(th, float),
            "gx": np.array(gx, float), "gy": np.array(gy, float), "step": step,
            "episode": episode}


def test_si_to_uni_special_headings(orc):
    p = orc.Params(wheel_radius=0.0)
    v, w = orc.si_to_uni(p, 0.0, 0.13, -0.07)
    assert v == pytest.approx(0.13, abs=1e-15) and w == pytest.approx(-0.07 / 0.05, abs=1e-13)
    v, w = orc.si_to_uni(p, math.pi / 2, 0.13, -0.07)
    assert v == pytest.approx(-0.07, abs=1e-15) and w == pytest.approx(-0.13 / 0.05, abs=1e-13)


def test_uni_si_round_trip(orc):
    p = orc.Params(wheel_radius=0.0)
    rng = np.random.default_rng(0)
    for _ in range(200):
        th, v, w = rng.uniform(-math.pi, math.pi), rng.uniform(-0.2, 0.2), rng.uniform(-3, 3)
        # velocity of the point l ahead of the axle for a unicycle (v, w)
        ux = v * math.cos(th) - p.proj_dist * w * math.sin(th)
        uy = v * math.sin(th) + p.proj_dist * w * math.cos(th)
        v2, w2 = orc.si_to_uni(p, th, ux, uy)
        assert v2 == pytest.approx(v, abs=1e-14) and w2 == pytest.approx(w, abs=1e-12)


def test_wheel_saturation(orc):
    p = orc.Params()
    # pure turn: v=0, w=0.2/0.05=4 rad/s -> wheel speeds +-(L/2)w/R exceed 0.2/R
    v, w = orc.si_to_uni(p, 0.0, 0.0, 0.2)
    assert v == 0.0
    assert w == pytest.approx(2 * 0.2 / 0.105, rel=1e-14)
    # forward 0.2 fits exactly
    v, w = orc.si_to_uni(p, 0.0, 0.2, 0.0)
    assert v == pytest.approx(0.2, abs=1e-15) and w == 0.0
    # mixed: right wheel saturates, left does not
    v, w = orc.si_to_uni(p, 0.0, 0.1, 0.1)
    R, L = 0.016, 0.105
    phr, phl = min((0.1 + L / 2 * 2.0) / R, 0.2 / R), (0.1 - L / 2 * 2.0) / R
    assert v == pytest.approx(R * (phr + phl) / 2, rel=1e-13)
    assert w == pytest.approx(R * (phr - phl) / L, rel=1e-13)


def test_euler_straight_line_and_turn(orc):
    p = orc.Params(max_steps=0, goal_radius=0.0)
    st = _state([0.0, 1.0], [0.0, 0.5], [0.0, 0.3], [1.0, 1.0], [0.0, 0.0])
    out = orc.env_step(p, st, env_id=0, t_global=0, actions=np.array([1, 0], np.uint8))
    assert st["x"][0] == pytest.approx(p.dt * 0.2, abs=1e-15)
    assert st["y"][0] == 0.0 and st["th"][0] == 0.0
    assert st["x"][1] == 1.0 and st["y"][1] == 0.5 and st["th"][1] == pytest.approx(0.3, abs=0)
    # +y from heading 0: no forward motion, saturated turn rate 2 v_max / L
    st = _state([0.0, 1.0], [0.0, 0.5], [0.0, 0.0], [1.0, 1.0], [0.0, 0.0])
    orc.env_step(p, st, env_id=0, t_global=0, actions=np.array([3, 0], np.uint8))
    assert st["x"][0] == 0.0 and st["y"][0] == 0.0
    assert st["th"][0] == pytest.approx(p.dt * 2 * 0.2 / 0.105, rel=1e-14)
    assert out["infeasible"] == 0


def test_heading_wraps_to_pi_interval(orc):
    p = orc.Params(max_steps=0, goal_radius=0.0)
    st = _state([0.0, 1.0], [0.0, 0.5], [math.pi - 0.01, 0.0], [1.0, 1.0], [0.0, 0.0])
    # heading ~pi, command -y turns left (w > 0) past pi
    orc.env_step(p, st, env_id=0, t_global=0, actions=np.array([4, 0], np.uint8))
    expect = math.pi - 0.01 + p.dt * 2 * 0.2 / 0.105 - 2 * math.pi
    assert st["th"][0] == pytest.approx(expect, abs=1e-13)
    assert -math.pi <= st["th"][0] <= math.pi


def test_reward_and_goal_termination(orc):
    p = orc.Params(goal_radius=0.05, max_steps=500)
    st = _state([0.0, 1.0], [0.0, 0.5], [0.0, 0.0], [0.03, 1.01], [0.0, 0.5], step=10)
    out = orc.env_step(p, st, env_id=5, t_global=10, actions=np.array([0, 0], np.uint8))
    assert out["reward"] == pytest.approx(-(0.03 + 0.01), abs=1e-15)
    assert out["done"] == 1
    # reset to episode 1 of env 5, step counter cleared
    assert st["step"] == 0 and st["episode"] == 1
    x, y, th, gx, gy = orc.reset_env(p, 5, 1, 2)
    np.testing.assert_array_equal(st["x"], x)
    np.testing.assert_array_equal(st["gy"], gy)
    # observation is of the reset state
    np.testing.assert_array_equal(out["obs"], orc.observe(x, y, th, gx, gy))


def test_time_limit_termination(orc):
    p = orc.Params(goal_radius=0.05, max_steps=500)
    st = _state([0.0, 1.0], [0.0, 0.5], [0.0, 0.0], [0.5, 0.0], [0.5, 0.0], step=498)
    out = orc.env_step(p, st, env_id=0, t_global=0, actions=np.array([0, 0], np.uint8))
    assert out["done"] == 0 and st["step"] == 499
    out = orc.env_step(p, st, env_id=0, t_global=1, actions=np.array([0, 0], np.uint8))
    assert out["done"] == 1 and st["step"] == 0 and st["episode"] == 1
    # one robot at the goal is not enough
    st = _state([0.0, 1.0], [0.0, 0.5], [0.0, 0.0], [0.0, 0.5], [0.0, 0.0], step=3)
    out = orc.env_step(p, st, env_id=0, t_global=0, actions=np.array([0, 0], np.uint8))
    assert out["done"] == 0


def test_observation_layout(orc):
    x, y = np.array([0.1, -0.4, 0.7]), np.array([0.2, 0.3, -0.5])
    th, gx, gy = np.array([0.5, -2.0, 3.0]), np.array([1.0, 0.0, -1.0]), np.array([0.0, 0.5, 0.5])
    obs = orc.observe(x, y, th, gx, gy)
    assert obs.shape == (3, 10)
    row = obs[1]
    np.testing.assert_allclose(row[:4], [x[1], y[1], math.cos(th[1]), math.sin(th[1])], atol=0)
    np.testing.assert_allclose(row[4:8], [x[0] - x[1], y[0] - y[1], x[2] - x[1], y[2] - y[1]],
                               atol=0)
    np.testing.assert_allclose(row[8:], [gx[1] - x[1], gy[1] - y[1]], atol=0)


@pytest.mark.parametrize("n", [2, 4, 8, 12, 16])
def test_reset_invariants(orc, n):
    p = orc.Params(seed=42)
    s2 = 3000 ** 2
    for env_id in range(40):
        X, Y, GX, GY, hb = orc.reset_lattice(p, env_id, env_id % 3, n)
        for A, B in ((X, Y), (GX, GY)):
            assert (A >= -14000).all() and (A <= 14000).all()
            assert (B >= -8000).all() and (B <= 8000).all()
            d2 = (A[:, None] - A[None, :]) ** 2 + (B[:, None] - B[None, :]) ** 2
            d2[np.arange(n), np.arange(n)] = s2
            assert (d2 >= s2).all()
        x, y, th, gx, gy = orc.reset_env(p, env_id, env_id % 3, n)
        np.testing.assert_array_equal(x, X * 1e-4)
        assert (th >= -math.pi).all() and (th < math.pi).all()


def test_reset_first_draw_is_uniform_lattice_index(orc):
    # robot 0 always accepts its first draw: X = X_lo + floor(W r0 / 2^32)
    p = orc.Params(seed=9)
    for env_id, ep in [(0, 0), (17, 3), (4095, 1)]:
        X, Y, *_ = orc.reset_lattice(p, env_id, ep, 4)
        blk = orc.philox4x32_10([env_id, ep, (2 << 24) | 0, 0], [9, 0])
        assert X[0] == -14000 + ((int(blk[0]) * 28001) >> 32)
        assert Y[0] == -8000 + ((int(blk[1]) * 16001) >> 32)


def test_reset_uniformity(orc):
    p = orc.Params(seed=1)
    xs = np.concatenate([orc.reset_lattice(p, e, 0, 1)[0] for e in range(4000)])
    hist, _ = np.histogram(xs, bins=10, range=(-14000, 14001))
    chi2 = ((hist - 400) ** 2 / 400).sum()
    assert chi2 < 35  # 9 dof


def test_reset_determinism_and_episode_keying(orc):
    p = orc.Params(seed=5)
    a = orc.reset_env(p, 10, 2, 8)
    b = orc.reset_env(p, 10, 2, 8)
    c = orc.reset_env(p, 10, 3, 8)
    for u, v in zip(a, b):
        np.testing.assert_array_equal(u, v)
    assert not np.array_equal(a[0], c[0])
