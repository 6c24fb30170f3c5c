"""Oracle pins for the barrier-certificate projection.

Pins (none re-use the oracle's solver):
* the closed-form projection onto one half-space (two robots, no bound active);
* brute-force enumeration of all active sets (tests/qp_bruteforce.py) for
  N = 2, 3, 4 on random and stressed states;
* the KKT certificate (stationarity, feasibility, complementarity, lambda >= 0);
* u* = u_nom whenever the pre-clipped nominal command is already feasible;
* the safety invariant: a single-integrator step of length dt from a safe
  state keeps every projection-point pair at least r_s apart;
* empty constraint sets are flagged (coincident robots, crossed wall bounds).
"""
import math

import numpy as np
import pytest

from paper_2505_06771_amd import synth
from tests import qp_bruteforce as bf


def proj_points(st, e, l=0.05):
    return (st["x"][e] + l * np.cos(st["th"][e]), st["y"][e] + l * np.sin(st["th"][e]))


def test_single_halfspace_closed_form(orc):
    p = orc.Params()
    rng = np.random.default_rng(1)
    checked = 0
    while checked < 200:
        c = np.array([rng.uniform(-1.0, 1.0), rng.uniform(-0.5, 0.5)])
        d = rng.uniform(0.18, 0.3)
        a = rng.uniform(-math.pi, math.pi)
        px = np.array([c[0], c[0] + d * math.cos(a)])
        py = np.array([c[1], c[1] + d * math.sin(a)])
        uxn = rng.uniform(-0.12, 0.12, 2)
        uyn = rng.uniform(-0.12, 0.12, 2)
        dx, dy = px[0] - px[1], py[0] - py[1]
        h = dx * dx + dy * dy - p.safety_radius ** 2
        arow = np.array([-2 * dx, -2 * dy, 2 * dx, 2 * dy])
        bval = p.barrier_gain * h ** 3
        uh = np.array([uxn[0], uyn[0], uxn[1], uyn[1]])
        viol = arow @ uh - bval
        ustar = uh - max(0.0, viol) / (arow @ arow) * arow
        _, _, lo, hi = bf.constraint_data(p, px, py)
        if (ustar >= hi - 1e-6).any() or (ustar <= lo + 1e-6).any():
            continue  # a bound would be active: not the single-row case
        ux, uy, lam, st, kkt, mv = orc.barrier_certificate(p, px, py, uxn, uyn)
        assert st == 0
        got = np.array([ux[0], uy[0], ux[1], uy[1]])
        np.testing.assert_allclose(got, ustar, atol=1e-14, rtol=0)
        # multiplier of |u-uhat|^2: 2 max(0, viol)/|a|^2
        assert abs(lam[0] - 2 * max(0.0, viol) / (arow @ arow)) < 1e-12
        checked += 1


@pytest.mark.parametrize("n,count", [(2, 40), (3, 25), (4, 6)])
def test_bruteforce_enumeration(orc, n, count):
    p = orc.Params()
    nbinding = 0
    for seed in range(count):
        kind = ["cluster", "wall", "tangent", "collinear", "corner"][seed % 5]
        st = synth.stressed_states(100 * n + seed, 1, n, kind)
        px, py = proj_points(st, 0)
        if seed % 2:
            uxn, uyn = synth.inward_commands(px[None], py[None])
            uxn, uyn = uxn[0], uyn[0]
        else:
            uxn, uyn = synth.nominal_commands(seed, n)
        A, b, lo, hi = bf.constraint_data(p, px, py)
        uh = bf.preclip(p, uxn, uyn)
        pts = bf.enumerate_kkt_points(A, b, lo, hi, uh)
        ux, uy, lam, status, kkt, mv = orc.barrier_certificate(p, px, py, uxn, uyn)
        if not pts:
            assert status == 1
            continue
        assert status == 0
        for q in pts[1:]:
            np.testing.assert_allclose(q, pts[0], atol=1e-8)  # uniqueness
        got = np.stack([ux, uy], 1).ravel()
        np.testing.assert_allclose(got, pts[0], atol=1e-10, rtol=0)
        nbinding += int(np.abs(got - uh).max() > 1e-9)
    assert nbinding >= count // 3  # the instances actually exercise the QP


@pytest.mark.parametrize("n", [2, 4, 8, 12, 16])
def test_kkt_certificate_stressed(orc, n):
    p = orc.Params()
    for seed in range(12):
        st = synth.stressed_states(7 * n + seed, 1, n, "mixed")
        px, py = proj_points(st, 0)
        uxn, uyn = synth.inward_commands(px[None], py[None], speed=0.25)
        ux, uy, lam, status, kkt, mv = orc.barrier_certificate(p, px, py, uxn[0], uyn[0])
        if status == 1:
            continue
        assert status == 0
        assert kkt[0] < 1e-12 and kkt[1] < 1e-11 and kkt[2] <= 0 and kkt[3] < 1e-11
        assert mv < 1e-11
        assert (lam >= 0).all()


def test_feasible_nominal_is_returned(orc):
    p = orc.Params()
    for seed in range(30):
        st = synth.random_states(seed, 1, 6, min_sep=0.8 if seed % 2 else 0.3)
        px, py = proj_points(st, 0)
        uxn, uyn = synth.nominal_commands(seed, 6, speed=0.05)
        A, b, lo, hi = bf.constraint_data(p, px, py)
        uh = bf.preclip(p, uxn, uyn)
        feasible = (A @ uh <= b).all() and (uh <= hi).all() and (uh >= lo).all()
        ux, uy, *_ = orc.barrier_certificate(p, px, py, uxn, uyn)
        if feasible:
            np.testing.assert_array_equal(np.stack([ux, uy], 1).ravel(), uh)


def test_preclip_magnitude(orc):
    p = orc.Params()
    px, py = np.array([-0.5, 0.5]), np.array([0.0, 0.0])
    ux, uy, *_ = orc.barrier_certificate(p, px, py, np.array([0.3, 0.0]), np.array([0.4, 0.1]))
    assert abs(math.hypot(ux[0], uy[0]) - 0.2) < 1e-15
    assert abs(ux[0] / uy[0] - 0.75) < 1e-12


@pytest.mark.parametrize("n", [3, 6, 8])
def test_safety_invariant_single_integrator(orc, n):
    p = orc.Params()
    worst = 1e9
    for seed in range(20):
        st = synth.stressed_states(500 + seed, 1, n, "mixed")
        px, py = proj_points(st, 0)
        dmin = min(math.hypot(px[i] - px[j], py[i] - py[j]) for i in range(n)
                   for j in range(i + 1, n))
        if dmin < p.safety_radius:
            continue  # start must be safe
        uxn, uyn = synth.inward_commands(px[None], py[None])
        ux, uy, lam, status, kkt, mv = orc.barrier_certificate(p, px, py, uxn[0], uyn[0])
        assert status == 0
        qx, qy = px + p.dt * ux, py + p.dt * uy
        for i in range(n):
            for j in range(i + 1, n):
                worst = min(worst, math.hypot(qx[i] - qx[j], qy[i] - qy[j]))
    assert worst >= p.safety_radius - 1e-12


def test_infeasible_sets_are_flagged(orc):
    p = orc.Params()
    # coincident projection points: the pair row reads 0 <= gamma (-r_s^2)^3 < 0
    px, py = np.array([0.0, 0.0, 0.6]), np.array([0.1, 0.1, 0.0])
    ux, uy, lam, status, kkt, mv = orc.barrier_certificate(p, px, py, np.zeros(3), np.zeros(3))
    assert status == 1
    # crossed wall bounds: far outside the right wall, hi_x < -v_max = lo_x
    px, py = np.array([1.9, 0.0]), np.array([0.0, 0.0])
    ux, uy, lam, status, kkt, mv = orc.barrier_certificate(p, px, py, np.zeros(2), np.zeros(2))
    assert status == 1
    lo_x, hi_x, lo_y, hi_y = orc.bounds(p, px, py)
    assert hi_x[0] < lo_x[0]
    assert ux[0] == pytest.approx(0.5 * (lo_x[0] + hi_x[0]), abs=1e-15)
    # overlapping but separable robots are feasible
    px, py = np.array([0.0, 0.15]), np.array([0.0, 0.0])
    ux, uy, lam, status, kkt, mv = orc.barrier_certificate(p, px, py, np.zeros(2), np.zeros(2))
    assert status == 0 and ux[0] < 0 < ux[1]


def test_wall_bounds_closed_form(orc):
    p = orc.Params()
    px, py = np.array([1.40, -1.45, 0.0]), np.array([0.0, 0.80, -0.86])
    lo_x, hi_x, lo_y, hi_y = orc.bounds(p, px, py)
    kb = 0.4 * 100.0
    assert hi_x[0] == pytest.approx(kb * (1.6 - 0.085 - 1.40) ** 3, rel=1e-14)
    assert lo_x[1] == pytest.approx(-kb * (-1.45 + 1.6 - 0.085) ** 3, rel=1e-14)
    assert hi_y[1] == pytest.approx(min(0.2, kb * (1.0 - 0.085 - 0.80) ** 3), rel=1e-14)
    assert lo_y[2] == pytest.approx(-kb * (-0.86 + 1.0 - 0.085) ** 3, rel=1e-14)
    assert hi_x[2] == 0.2 and lo_x[2] == -0.2


# ---- the violation metric (largest normalised row excess) -----------------

def _wall_hi(p, c, wall):
    """Upper bound of one coordinate from its closed form: the speed limit or
    the cubic wall certificate of the wall pulled in by r_s / 2."""
    m = wall - p.safety_radius / 2 - c
    return min(p.v_max, p.boundary_gain_factor * p.barrier_gain * m ** 3)


def test_max_violation_of_a_pair_row_is_normalised_by_its_norm(orc):
    """Pair row -2 D.u_i + 2 D.u_j <= gamma h^3 has norm 2 sqrt(2) |D|; the
    metric is the row excess divided by it (m/s)."""
    p = orc.Params()
    px, py = np.array([0.0, 0.2]), np.array([0.0, 0.0])
    dx, dy = px[0] - px[1], py[0] - py[1]
    b = p.barrier_gain * (dx * dx + dy * dy - p.safety_radius ** 2) ** 3
    ux, uy = np.array([0.1, -0.1]), np.array([0.0, 0.0])  # head-on, inside the box
    excess = (-2 * dx * ux[0] - 2 * dy * uy[0]) + (2 * dx * ux[1] + 2 * dy * uy[1]) - b
    assert excess > 0.05
    want = excess / (2 * math.sqrt(2) * math.hypot(dx, dy))
    got = orc.max_violation(p, px, py, ux, uy)
    assert got == pytest.approx(want, rel=1e-14)
    assert abs(got - excess) > 0.01  # an unnormalised excess would fail
    # moving apart satisfies the row: nothing is violated
    assert orc.max_violation(p, px, py, -ux, uy) == 0.0


def test_max_violation_of_bounds_and_the_max_over_rows(orc):
    p = orc.Params()
    # robot 0 near the right wall: its x bound is the wall certificate
    px, py = np.array([1.5, -1.0]), np.array([0.0, 0.5])
    hi0 = _wall_hi(p, px[0], p.x_max)
    assert hi0 < 1e-3
    ux, uy = np.array([0.05, 0.0]), np.array([0.0, 0.0])
    assert orc.max_violation(p, px, py, ux, uy) == pytest.approx(0.05 - hi0, rel=1e-14)
    # a speed-box excess of robot 1 in y (lower bound -v_max)
    uy2 = np.array([0.0, -0.32])
    assert orc.max_violation(p, px, py, np.zeros(2), uy2) == pytest.approx(0.12, rel=1e-14)
    # both at once: the metric is the larger of the two
    got = orc.max_violation(p, px, py, ux, uy2)
    assert got == pytest.approx(max(0.05 - hi0, 0.12), rel=1e-14)
    # three robots: a violated pair row next to a smaller bound excess
    px3, py3 = np.array([0.0, 0.19, -1.0]), np.array([0.0, 0.0, 0.5])
    ux3, uy3 = np.array([0.2, -0.2, 0.0]), np.array([0.0, 0.0, 0.21])
    dx = px3[0] - px3[1]
    b = p.barrier_gain * (dx * dx - p.safety_radius ** 2) ** 3
    pair = (-2 * dx * ux3[0] + 2 * dx * ux3[1] - b) / (2 * math.sqrt(2) * abs(dx))
    assert pair > 0.01
    assert orc.max_violation(p, px3, py3, ux3, uy3) == pytest.approx(max(pair, 0.01), rel=1e-13)
