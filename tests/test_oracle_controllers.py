"""Oracle pins of the waypoint controller and the action noise: special
bearings of the unicycle position controller with closed-form outputs, the
projection-point map checked against its inverse, the nominal command of each
move action, convergence of the heading toward a held direction, and the
distribution, scaling and counter layout of the noise draws."""
import math

import numpy as np
import pytest


def _state(x, y, th, gx=None, gy=None, step=0, episode=0):
    n = len(x)
    return {"x": np.array(x, float), "y": np.array(y, float), "th": np.array(th, float),
            "gx": np.zeros(n) if gx is None else np.array(gx, float),
            "gy": np.zeros(n) if gy is None else np.array(gy, float), "step": step,
            "episode": episode}


@pytest.mark.parametrize("th", [0.0, 0.7, -2.9, math.pi / 2])
def test_position_controller_special_bearings(orc, th):
    p = orc.Params(controller=2)
    kv, kw, rho = p.pos_gain, p.ang_gain, 0.3
    x0, y0 = 0.25, -0.4

    def at(bearing):
        a = th + bearing
        return orc.unicycle_position(p, x0, y0, th, x0 + rho * math.cos(a), y0 + rho * math.sin(a))

    v, w = at(0.0)  # straight ahead: full speed, no turn
    assert v == pytest.approx(kv * rho, abs=1e-15) and abs(w) < 1e-14
    v, w = at(math.pi)  # behind: reverse, no turn
    assert v == pytest.approx(-kv * rho, abs=1e-15) and abs(w) < 1e-14
    v, w = at(math.pi / 2)  # to the left: turn counter-clockwise on the spot
    assert abs(v) < 1e-15 and w == pytest.approx(kw, abs=1e-14)
    v, w = at(-math.pi / 2)  # to the right: clockwise
    assert abs(v) < 1e-15 and w == pytest.approx(-kw, abs=1e-14)
    v, w = at(math.pi / 4)
    assert v == pytest.approx(kv * rho / math.sqrt(2), abs=1e-15)
    assert w == pytest.approx(kw / math.sqrt(2), abs=1e-14)
    assert orc.unicycle_position(p, x0, y0, th, x0, y0) == (0.0, 0.0)  # idle at the waypoint


def test_uni_to_si_is_the_inverse_of_si_to_uni(orc):
    p = orc.Params(wheel_radius=0.0)
    rng = np.random.default_rng(4)
    for _ in range(300):
        th, v, w = rng.uniform(-math.pi, math.pi), rng.uniform(-0.2, 0.2), rng.uniform(-4, 4)
        ux, uy = orc.uni_to_si(p, th, v, w)
        # along the heading the projection point moves with the centre
        assert ux * math.cos(th) + uy * math.sin(th) == pytest.approx(v, abs=1e-15)
        v2, w2 = orc.si_to_uni(p, th, ux, uy)
        assert v2 == pytest.approx(v, abs=1e-15) and w2 == pytest.approx(w, abs=1e-13)


def test_waypoint_nominal_command_per_action(orc):
    p = orc.Params(controller=2)
    s, kv, kw, l = p.waypoint_step, p.pos_gain, p.ang_gain, p.proj_dist
    # five robots, all heading +x, one per action
    st = _state([-1.0, -0.5, 0.0, 0.5, 1.0], [0.0] * 5, [0.0] * 5)
    unx, uny, used = orc.nominal_command(p, st, 0, 0, np.arange(5, dtype=np.uint8))
    expect = [(0.0, 0.0),            # stay: idle
              (kv * s, 0.0),         # +x: ahead
              (-kv * s, 0.0),        # -x: behind, reverse
              (0.0, l * kw),         # +y: left, pure turn; the projection point moves +y
              (0.0, -l * kw)]        # -y: right
    for i, (ex, ey) in enumerate(expect):
        assert unx[i] == pytest.approx(ex, abs=1e-15) and uny[i] == pytest.approx(ey, abs=1e-15)
    assert unx[0] == 0.0 and uny[0] == 0.0
    # heading +y: action +y is straight ahead
    st = _state([0.0, 0.5], [0.0, 0.0], [math.pi / 2, math.pi / 2])
    unx, uny, _ = orc.nominal_command(p, st, 0, 0, np.array([3, 1], np.uint8))
    assert unx[0] == pytest.approx(0.0, abs=1e-15) and uny[0] == pytest.approx(kv * s, abs=1e-15)
    # +x from heading +y is to the right: clockwise turn, projection point moves +x
    assert unx[1] == pytest.approx(l * kw, abs=1e-15) and uny[1] == pytest.approx(0, abs=1e-15)


def test_waypoint_heading_converges_to_held_direction(orc):
    p = orc.Params(controller=2, max_steps=0, goal_radius=0.0)
    st = _state([-1.0, 1.0], [-0.5, 0.5], [math.pi / 2, -2.5])  # never within reach
    x_start = st["x"].copy()
    for t in range(150):
        orc.env_step(p, st, 0, t, actions=np.array([1, 2], np.uint8))
    assert abs(st["th"][0]) < 0.02                               # now heading +x
    assert abs(abs(st["th"][1]) - math.pi) < 0.02                # now heading -x
    assert st["x"][0] - x_start[0] > 0.5 and x_start[1] - st["x"][1] > 0.5


def test_action_noise_distribution_and_layout(orc):
    sigma = 0.05
    p = orc.Params(action_noise=sigma, seed=12345)
    draws = np.array([orc.action_noise(p, e, t, i) for e in range(40) for t in range(50)
                      for i in range(10)])
    assert draws.shape == (20000, 2)
    assert (draws >= -sigma).all() and (draws < sigma).all()
    se = sigma / math.sqrt(3 * draws.shape[0])
    assert np.abs(draws.mean(axis=0)).max() < 5 * se
    assert draws.var(axis=0) == pytest.approx([sigma ** 2 / 3] * 2, rel=0.04)
    assert abs(np.corrcoef(draws[:, 0], draws[:, 1])[0, 1]) < 0.04
    # linear in sigma on the same draws; off at sigma 0
    p2 = orc.Params(action_noise=2 * sigma, seed=12345)
    assert orc.action_noise(p2, 3, 7, 2) == tuple(2 * v for v in orc.action_noise(p, 3, 7, 2))
    assert orc.action_noise(orc.Params(seed=12345), 3, 7, 2) == (0.0, 0.0)
    # counter layout (env_id, t, 6 << 24 | i, 0), words 0 and 1, 24-bit uniforms
    blk = orc.philox4x32_10([3, 7, (6 << 24) | 2, 0], [12345, 0])
    u = [(int(r) >> 8) * 2.0 ** -24 for r in blk[:2]]
    assert orc.action_noise(p, 3, 7, 2) == (sigma * (2 * u[0] - 1), sigma * (2 * u[1] - 1))


@pytest.mark.parametrize("controller", [0, 2])
def test_noise_enters_ahead_of_preclip_and_certificate(orc, controller):
    """A noisy step equals the noise-free pipeline fed with the noisy nominal
    command: noise, then magnitude pre-clip and certificate, then dynamics."""
    p = orc.Params(controller=controller, action_noise=0.15, max_steps=0, goal_radius=0.0, seed=3)
    st = _state([-0.3, -0.1, 0.12, 0.5], [0.0, 0.05, -0.06, 0.4], [0.3, 2.0, -1.0, 3.0])
    acts = np.array([1, 4, 2, 3], np.uint8)
    unx, uny, _ = orc.nominal_command(p, st, 9, 21, acts)
    free = orc.Params(**{**p.__dict__, "action_noise": 0.0})
    unx0, uny0, _ = orc.nominal_command(free, st, 9, 21, acts)
    for i in range(4):
        nx, ny = orc.action_noise(p, 9, 21, i)
        assert unx[i] == unx0[i] + nx and uny[i] == uny0[i] + ny
    px = st["x"] + p.proj_dist * np.cos(st["th"])
    py = st["y"] + p.proj_dist * np.sin(st["th"])
    ux, uy, _, status, _, _ = orc.barrier_certificate(p, px, py, unx, uny)
    assert status == 0
    ref = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in st.items()}
    orc.env_step(p, ref, 9, 21, actions=acts)
    for i in range(4):
        v, w = orc.si_to_uni(p, st["th"][i], ux[i], uy[i])
        c, s = math.cos(st["th"][i]), math.sin(st["th"][i])
        assert ref["x"][i] == pytest.approx(st["x"][i] + p.dt * v * c, abs=1e-15)
        assert ref["y"][i] == pytest.approx(st["y"][i] + p.dt * v * s, abs=1e-15)
        assert ref["th"][i] == pytest.approx(st["th"][i] + p.dt * w, abs=1e-14) or \
            abs(abs(ref["th"][i] - st["th"][i] - p.dt * w) - 2 * math.pi) < 1e-12


# ---- go-to-goal controller (single-integrator controller of Sec. 4.1,
# proportional law on the projection point) ---------------------------------

@pytest.mark.parametrize("kp", [1.0, 2.5])
def test_goto_goal_command_at_special_headings(orc, kp):
    """u_nom = kp (g - p) with p the projection point, not the centre: at
    heading 0 the point sits l ahead in x, at heading pi/2 l ahead in y."""
    p = orc.Params(controller=1, kp=kp)
    l = p.proj_dist
    x0, y0, gx, gy = 0.3, -0.2, 0.37, -0.11
    st = _state([x0, -1.0], [y0, 0.5], [0.0, math.pi / 2], [gx, -0.9], [gy, 0.62])
    unx, uny, _ = orc.nominal_command(p, st, 0, 0)
    assert unx[0] == pytest.approx(kp * (gx - (x0 + l)), abs=1e-15)
    assert uny[0] == pytest.approx(kp * (gy - y0), abs=1e-15)
    # heading pi/2: the projection point is (x, y + l)
    assert unx[1] == pytest.approx(kp * (-0.9 - (-1.0)), abs=1e-14)
    assert uny[1] == pytest.approx(kp * (0.62 - (0.5 + l)), abs=1e-14)
    # using the centre instead would differ by kp * l in the heading direction
    assert abs(unx[0] - kp * (gx - x0)) > 0.5 * kp * l
    assert abs(uny[1] - kp * (0.62 - 0.5)) > 0.5 * kp * l


def test_goto_goal_command_is_zero_at_the_goal(orc):
    p = orc.Params(controller=1)
    th = np.array([0.3, -2.0, 2.9])
    x, y = np.array([0.1, -0.5, 0.8]), np.array([0.2, 0.4, -0.3])
    gx = x + p.proj_dist * np.cos(th)  # the goal is the projection point itself
    gy = y + p.proj_dist * np.sin(th)
    unx, uny, _ = orc.nominal_command(p, _state(x, y, th, gx, gy), 0, 0)
    assert (unx == 0.0).all() and (uny == 0.0).all()


def test_goto_goal_large_error_is_preclipped_to_vmax(orc):
    """A far goal gives |kp (g - p)| > v_max: the executed command is the
    pre-clipped one, v_max along g - p (no barrier row or wall binds for two
    robots far apart in the middle of the arena). Without wheel saturation the
    unicycle step shows it: v = u.(c, s), w = u.(-s, c) / l."""
    p = orc.Params(controller=1, wheel_radius=0.0, max_steps=0, goal_radius=0.0)
    l, dt, vmax = p.proj_dist, p.dt, p.v_max
    st = _state([-0.6, 0.6], [0.0, 0.0], [0.0, math.pi / 2], [0.9, 0.2], [0.7, -0.8])
    start = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in st.items()}
    out = orc.env_step(p, st, 0, 0)
    assert out["status"] == 0 and out["infeasible"] == 0
    for i in range(2):
        th = start["th"][i]
        c, s = math.cos(th), math.sin(th)
        px, py = start["x"][i] + l * c, start["y"][i] + l * s
        ex, ey = start["gx"][i] - px, start["gy"][i] - py
        assert math.hypot(ex, ey) > 2 * vmax       # far outside the clip radius
        ux, uy = vmax * ex / math.hypot(ex, ey), vmax * ey / math.hypot(ex, ey)
        v, w = ux * c + uy * s, (-s * ux + c * uy) / l
        assert st["x"][i] == pytest.approx(start["x"][i] + dt * v * c, abs=1e-15)
        assert st["y"][i] == pytest.approx(start["y"][i] + dt * v * s, abs=1e-15)
        assert st["th"][i] == pytest.approx(th + dt * w, abs=1e-14)
