"""CPU pins of the oracle's unicycle pose controller (f4; JaxRobotarium Sec. 4.1:
unicycle controllers drive robots to desired positions/poses, and Table 1
times a pose controller beside the position one). The reading is the law of
Aicardi et al. (1995): v = k_rho rho cos(alpha), w = k_alpha alpha + k_rho
(sin(alpha) cos(alpha) / alpha)(alpha + k_beta beta) on the distance rho,
the bearing alpha of the goal from the heading and the bearing beta of the
line of sight from the goal heading.

The pins do not retype the law: they check values it must take at special
poses, its symmetries, its Lyapunov function (which a sign error in any term
breaks), convergence to the goal pose, and the waypoint-pose wiring of the
action space."""
import math

import numpy as np
import pytest


def _wrap(a):
    return math.atan2(math.sin(a), math.cos(a))


def test_idle_at_the_goal_pose(orc):
    p = orc.Params()
    for x, y, th in [(0.0, 0.0, 0.0), (0.3, -0.2, 2.0), (-1.0, 0.5, -3.0)]:
        v, w = orc.unicycle_pose(p, x, y, th, x, y, th)
        assert v == 0.0 and w == 0.0


@pytest.mark.parametrize("th", [0.0, 1.0, -2.5])
def test_pure_rotation_at_the_goal_position(orc, th):
    """rho = 0: no linear speed; the turn rate has the sign of the heading
    error, slope k_alpha + k_rho at zero error, and k_alpha * pi/2 at a right
    angle (where sin(alpha) cos(alpha) vanishes)."""
    p = orc.Params()
    for d in (0.3, -0.7, 1.2):
        v, w = orc.unicycle_pose(p, 0.1, 0.2, th, 0.1, 0.2, th + d)
        assert v == 0.0
        assert np.sign(w) == np.sign(d)
    eps = 1e-5
    _, w = orc.unicycle_pose(p, 0.0, 0.0, th, 0.0, 0.0, th + eps)
    assert abs(w / eps - (p.pose_gain_alpha + p.pose_gain_rho)) < 1e-6
    _, w = orc.unicycle_pose(p, 0.0, 0.0, th, 0.0, 0.0, th + math.pi / 2)
    assert abs(w - p.pose_gain_alpha * math.pi / 2) < 1e-12


def test_turn_rate_at_a_45_degree_error_and_at_an_offset_goal_heading(orc):
    """At the goal position with a 45-degree heading error sin(alpha)
    cos(alpha) = 1/2, so w = k_alpha pi/4 + k_rho/2. Facing the goal position
    (alpha = 0) whose heading is off by b: v = k_rho rho and the robot swings
    away from the goal heading first, w = -k_rho k_beta b."""
    p = orc.Params()
    _, w = orc.unicycle_pose(p, 0.0, 0.0, 0.3, 0.0, 0.0, 0.3 + math.pi / 4)
    assert abs(w - (p.pose_gain_alpha * math.pi / 4 + 0.5 * p.pose_gain_rho)) < 1e-12
    for b in (0.6, -0.9):
        v, w = orc.unicycle_pose(p, 0.0, 0.0, 0.0, 0.5, 0.0, b)
        assert abs(v - 0.5 * p.pose_gain_rho) < 1e-12
        assert abs(w + p.pose_gain_rho * p.pose_gain_beta * b) < 1e-12


@pytest.mark.parametrize("th", [0.0, math.pi / 2, -2.0])
def test_straight_ahead_and_straight_behind(orc, th):
    p = orc.Params()
    d = 0.37
    # goal on the heading line, same heading: full speed ahead, no turn
    v, w = orc.unicycle_pose(p, 0.0, 0.0, th, d * math.cos(th), d * math.sin(th), th)
    assert abs(v - p.pose_gain_rho * d) < 1e-12 and abs(w) < 1e-12
    # goal straight behind, same heading: the speed reverses (cos alpha = -1)
    v, _ = orc.unicycle_pose(p, 0.0, 0.0, th, -d * math.cos(th), -d * math.sin(th), th)
    assert abs(v + p.pose_gain_rho * d) < 1e-12


def test_mirror_and_rigid_motion_symmetry(orc):
    """Reflecting the configuration across the x axis keeps v and negates w;
    a rigid motion of the whole configuration changes neither."""
    p = orc.Params()
    rng = np.random.default_rng(0)
    for _ in range(50):
        x, y, th, wx, wy, wth = rng.uniform(-1, 1, 6) * [1, 1, 3, 1, 1, 3]
        v, w = orc.unicycle_pose(p, x, y, th, wx, wy, wth)
        vm, wm = orc.unicycle_pose(p, x, -y, -th, wx, -wy, -wth)
        assert abs(v - vm) < 1e-12 and abs(w + wm) < 1e-12
        a, tx, ty = rng.uniform(-3, 3), rng.uniform(-1, 1), rng.uniform(-1, 1)
        ca, sa = math.cos(a), math.sin(a)
        rot = lambda px, py: (ca * px - sa * py + tx, sa * px + ca * py + ty)
        xr, yr = rot(x, y)
        wxr, wyr = rot(wx, wy)
        vr, wr = orc.unicycle_pose(p, xr, yr, th + a, wxr, wyr, wth + a)
        assert abs(v - vr) < 1e-9 and abs(w - wr) < 1e-9


def _polar(x, y, th, wx, wy, wth):
    rho = math.hypot(wx - x, wy - y)
    phi = math.atan2(wy - y, wx - x)
    return rho, _wrap(phi - th), _wrap(phi - wth)


def test_lyapunov_function_decreases_and_the_pose_converges(orc):
    """V = (rho^2 + alpha^2 + k_beta beta^2) / 2 has derivative
    -k_rho cos^2(alpha) rho^2 - k_alpha alpha^2 <= 0 along the closed loop of
    the unicycle: along Euler-integrated trajectories it never rises by more
    than the O(dt^2) of one step, and the robot reaches the goal pose."""
    p = orc.Params()
    rng = np.random.default_rng(1)
    dt = 1e-3
    for _ in range(12):
        x, y, th = rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(-3, 3)
        wx, wy, wth = rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(-3, 3)
        rho, al, be = _polar(x, y, th, wx, wy, wth)
        if abs(al) > 3.0 or abs(be) > 3.0:
            continue  # keep away from the +-pi cut of the wrapped angles
        V0 = V = 0.5 * (rho ** 2 + al ** 2 + p.pose_gain_beta * be ** 2)
        for k in range(int(12.0 / dt)):
            v, w = orc.unicycle_pose(p, x, y, th, wx, wy, wth)
            x += dt * v * math.cos(th)
            y += dt * v * math.sin(th)
            th += dt * w
            rho, al, be = _polar(x, y, th, wx, wy, wth)
            if rho < 1e-6:
                break
            Vn = 0.5 * (rho ** 2 + al ** 2 + p.pose_gain_beta * be ** 2)
            assert Vn <= V + 5e-6, f"V rose from {V} to {Vn} at step {k}"
            V = Vn
        assert V < 0.05 * V0 + 1e-6
    # one long run to the goal pose
    x, y, th, wx, wy, wth = 0.0, 0.0, 0.0, 0.0, 1.0, 0.0
    for _ in range(int(25.0 / dt)):
        v, w = orc.unicycle_pose(p, x, y, th, wx, wy, wth)
        x += dt * v * math.cos(th)
        y += dt * v * math.sin(th)
        th += dt * w
    assert math.hypot(wx - x, wy - y) < 1e-6
    assert abs(_wrap(wth - th)) < 0.05


def test_pose_waypoint_nominal_command_per_action(orc):
    """Controller 3: a move sets the pose waypoint_step ahead along the move,
    heading along the move. Facing the move: full speed along it, no turn;
    facing across it: a turn on the spot at k_alpha pi/2, which moves the
    projection point by l w perpendicular to the heading; staying: zero."""
    p = orc.Params(controller=3)
    l, s = p.proj_dist, p.waypoint_step
    dirs = {1: (1, 0), 2: (-1, 0), 3: (0, 1), 4: (0, -1)}
    for a, (dx, dy) in dirs.items():
        th = math.atan2(dy, dx)
        st = {"x": np.array([0.1]), "y": np.array([-0.2]), "th": np.array([th]),
              "gx": np.array([0.0]), "gy": np.array([0.0])}
        ux, uy, _ = orc.nominal_command(p, st, 0, 0, actions=np.array([a], np.uint8))
        assert abs(ux[0] - p.pose_gain_rho * s * dx) < 1e-12
        assert abs(uy[0] - p.pose_gain_rho * s * dy) < 1e-12
        th2 = th - math.pi / 2  # the move is 90 degrees to the left
        st["th"] = np.array([th2])
        ux, uy, _ = orc.nominal_command(p, st, 0, 0, actions=np.array([a], np.uint8))
        w = p.pose_gain_alpha * math.pi / 2
        assert abs(ux[0] + l * w * math.sin(th2)) < 1e-12
        assert abs(uy[0] - l * w * math.cos(th2)) < 1e-12
    st = {"x": np.array([0.1]), "y": np.array([-0.2]), "th": np.array([0.4]),
          "gx": np.array([0.0]), "gy": np.array([0.0])}
    ux, uy, _ = orc.nominal_command(p, st, 0, 0, actions=np.array([0], np.uint8))
    assert ux[0] == 0.0 and uy[0] == 0.0
