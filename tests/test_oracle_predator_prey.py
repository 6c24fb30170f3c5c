"""Oracle pins of the Predator-Prey scenario: the prey's flight from a single
tagger in closed form (open field, against a wall with a tie), the arg-max
property of its choice over all 17 candidates on random states, the tag
radius, the tag reward, termination on the step limit only, and the reset of
the shared prey slot."""
import math

import numpy as np
import pytest


def _pp(**kw):
    import oracle

    return oracle.Params(scenario=1, **kw)


def test_prey_flees_a_single_tagger_in_the_open(orc):
    p = _pp()
    s = p.prey_speed * p.dt
    q = (0.1, -0.2)
    # tagger due west: the prey steps due east (direction index 1, angle 0)
    nx, ny, k, _ = orc.prey_move(p, [q[0] - 0.6], [q[1]], *q)
    assert k == 1 and nx == q[0] + s and ny == q[1]
    # tagger to the north-east at 45 degrees: the prey steps to 225 degrees
    nx, ny, k, _ = orc.prey_move(p, [q[0] + 0.4], [q[1] + 0.4], *q)
    assert k == 1 + 10
    assert nx == pytest.approx(q[0] - s / math.sqrt(2), abs=1e-15)
    assert ny == pytest.approx(q[1] - s / math.sqrt(2), abs=1e-15)
    # no tagger can make staying put the unique best: a tagger on the prey
    # makes every move better than staying
    nx, ny, k, sc = orc.prey_move(p, [q[0]], [q[1]], *q)
    assert sc[0] == 0.0 and k != 0


def test_prey_against_a_wall_breaks_ties_on_the_first_index(orc):
    p = _pp()
    s = p.prey_speed * p.dt
    wall = p.x_max - 0.5 * p.safety_radius
    q = (wall, 0.0)
    nx, ny, k, sc = orc.prey_move(p, [wall - 0.5], [0.0], *q)
    # every eastward candidate is clamped onto the wall; straight up (index 5,
    # 90 degrees) and straight down (index 13) tie at 0.25 + s^2
    assert sc[5] == sc[13] == pytest.approx(0.25 + s * s, abs=1e-15)
    assert k == 5 and nx == pytest.approx(wall, abs=1e-15) and ny == pytest.approx(s, abs=1e-15)
    assert sc[1] == sc[0] == pytest.approx(0.25, abs=1e-15)  # east clamps to staying put


def test_prey_choice_is_the_arg_max_over_candidates(orc):
    """Brute force over the 17 candidates on random states (the candidate set
    is built here from its description, independently of the oracle)."""
    p = _pp()
    s = p.prey_speed * p.dt
    lox, hix = p.x_min + p.safety_radius / 2, p.x_max - p.safety_radius / 2
    loy, hiy = p.y_min + p.safety_radius / 2, p.y_max - p.safety_radius / 2
    rng = np.random.default_rng(7)
    for trial in range(300):
        n = int(rng.integers(1, 9))
        x, y = rng.uniform(-1.6, 1.6, n), rng.uniform(-1, 1, n)
        qx, qy = rng.uniform(lox, hix), rng.uniform(loy, hiy)
        if trial % 5 == 0:  # pressed into a corner
            qx, qy = hix, loy
        ang = np.array([2 * math.pi * k / 16 for k in range(16)])
        cx = np.concatenate([[qx], np.clip(qx + s * np.cos(ang), lox, hix)])
        cy = np.concatenate([[qy], np.clip(qy + s * np.sin(ang), loy, hiy)])
        score = ((cx[:, None] - x[None]) ** 2 + (cy[:, None] - y[None]) ** 2).min(axis=1)
        nx, ny, k, sc = orc.prey_move(p, x, y, qx, qy)
        np.testing.assert_allclose(sc, score, rtol=0, atol=1e-15)
        assert sc[k] == sc.max() and (sc[:k] < sc[k]).all()
        assert (nx, ny) == (cx[k], cy[k])
        assert lox <= nx <= hix and loy <= ny <= hiy
        assert math.hypot(nx - qx, ny - qy) <= s + 1e-15


def test_tag_radius(orc):
    p = _pp()
    assert orc.tagged(p, [0.0, 1.0], [0.0, 0.0], 0.249999, 0.0)
    assert not orc.tagged(p, [0.0, 1.0], [0.0, 0.0], 0.250001, 0.0)
    assert orc.tagged(p, [0.0, 1.0], [0.0, 0.0], 0.76, 0.0)  # the second robot


def _state(x, y, th, q, step=0):
    n = len(x)
    return {"x": np.array(x, float), "y": np.array(y, float), "th": np.array(th, float),
            "gx": np.full(n, q[0]), "gy": np.full(n, q[1]), "step": step, "episode": 0}


def test_step_moves_prey_rewards_tags_and_ends_on_the_limit(orc):
    p = _pp(max_steps=100, goal_radius=0.05)
    # robots stay (action 0): only the prey moves; it starts 0.2 m east of robot 0
    st = _state([0.0, -1.0], [0.0, 0.5], [0.0, 0.0], (0.2, 0.0), step=10)
    nqx, nqy, _, _ = orc.prey_move(p, st["x"], st["y"], 0.2, 0.0)
    out = orc.env_step(p, st, 0, 0, actions=np.array([0, 0], np.uint8))
    assert (st["gx"] == nqx).all() and (st["gy"] == nqy).all()  # shared prey slot
    assert nqx == pytest.approx(0.2 + p.prey_speed * p.dt, abs=1e-15)
    assert out["reward"] == p.tag_reward  # 0.21 m < 0.25 m
    assert out["done"] == 0 and st["step"] == 11
    # the observation's last pair is the vector to the prey
    assert out["obs"][0, -2] == pytest.approx(nqx - st["x"][0], abs=1e-15)
    # far away: no tag, no reward; robots at the prey do not end the episode
    st = _state([0.0, -1.0], [0.0, 0.5], [0.0, 0.0], (1.0, 0.5), step=10)
    out = orc.env_step(p, st, 0, 0, actions=np.array([0, 0], np.uint8))
    assert out["reward"] == 0.0 and out["done"] == 0
    # the step limit ends it
    st = _state([0.0, -1.0], [0.0, 0.5], [0.0, 0.0], (1.0, 0.5), step=99)
    out = orc.env_step(p, st, 3, 0, actions=np.array([0, 0], np.uint8))
    assert out["done"] == 1 and st["step"] == 0 and st["episode"] == 1


def test_reset_places_the_prey_at_the_first_goal_draw(orc):
    p = _pp(seed=9)
    for n in (3, 8):
        x, y, th, gx, gy = orc.reset_env(p, 17, 2, n)
        X, Y, GX, GY, _ = orc.reset_lattice(p, 17, 2, n)
        assert (gx == GX[0] * p.grid).all() and (gy == GY[0] * p.grid).all()
        assert (x == X * p.grid).all()
        # the navigation reset of the same key keeps every robot's own goal
        gxn = orc.reset_env(orc.Params(seed=9), 17, 2, n)[3]
        assert (gxn == GX * p.grid).all() and gxn[0] == gx[0]
