"""GPU tests of the certificate's observability.

* Every stage of the solver (box clip, one-row closed form, two rows on four
  robots, two rows through a shared robot, register active set, general LDS
  solver) runs on the stressed inputs, is counted per env by the qp_stats
  outputs, and each env's command matches the FP64 oracle's exact minimiser
  (1e-4 m/s in FP32, 1e-9 in FP64) whatever stage produced it.
* A solve stopped by the iteration cap is never silent: with a cap set on the
  host (qp_max_iters = 1, so every kernel still ends normally) the status
  output carries 2, qp_stats counts it and the context's failure counters add
  it, in barrier_certificate, env_step, rollout and env_run alike.
"""
import numpy as np
import pytest

from paper_2505_06771_amd import synth
from tests.gpu_util import banner, batch_from_states, ctx_and_lib, dev, host

pytestmark = pytest.mark.gpu

STAGES = ("box", "one_row", "two_rows", "shared_robot", "active_set", "general")


def _stage_inputs(seed, E, n):
    """Six blocks of envs aimed at the six stages: random states and commands
    (the box clip), one tight pair pushed together (one row), two such pairs
    (two rows on four robots), three robots in a row with the outer two
    pushed at the middle one (two rows through a shared robot), stressed
    states with random commands (short active sets) and tight clusters
    commanded toward their centroid (long active sets, the general solver).
    Robots not in a pair or row keep random commands of 5 cm/s."""
    rng = np.random.default_rng(seed)
    k = E // 6
    base = synth.random_states(seed, E, n, min_sep=0.45 if n <= 12 else 0.35)
    px, py = base["x"].copy(), base["y"].copy()
    ux, uy = synth.nominal_commands(seed + 3, (E, n), speed=0.3)
    for e in range(k, 4 * k):
        block = e // k  # 1 pair, 2 two pairs, 3 row of three
        ux[e] *= 0.05 / 0.3
        uy[e] *= 0.05 / 0.3
        a = rng.uniform(-np.pi, np.pi)
        dx, dy = np.cos(a), np.sin(a)
        v = rng.uniform(0.1, 0.15)
        if block in (1, 2):
            for q in range(block):
                cx, cy = (-0.7 + 1.4 * q, rng.uniform(-0.4, 0.4))
                d = rng.uniform(0.19, 0.22)
                i0, i1 = 2 * q, 2 * q + 1
                px[e, i0], py[e, i0] = cx - 0.5 * d * dx, cy - 0.5 * d * dy
                px[e, i1], py[e, i1] = cx + 0.5 * d * dx, cy + 0.5 * d * dy
                ux[e, i0], uy[e, i0] = v * dx, v * dy
                ux[e, i1], uy[e, i1] = -v * dx, -v * dy
        else:
            cx, cy = rng.uniform(-0.3, 0.3), rng.uniform(-0.2, 0.2)
            d = rng.uniform(0.2, 0.22)
            for q, off in enumerate((-1.0, 0.0, 1.0)):
                px[e, q], py[e, q] = cx + off * d * dx, cy + off * d * dy
            ux[e, 0], uy[e, 0] = v * dx, v * dy
            ux[e, 1], uy[e, 1] = 0.0, 0.0
            ux[e, 2], uy[e, 2] = -v * dx, -v * dy
        # the other robots stay clear of the pairs and the row
        for i in range(2 * block if block < 3 else 3, n):
            for _ in range(200):
                if min(np.hypot(px[e, i] - px[e, j], py[e, i] - py[e, j])
                       for j in range(n) if j != i) > 0.4:
                    break
                px[e, i] = rng.uniform(-1.35, 1.35)
                py[e, i] = rng.uniform(-0.75, 0.75)
    st = synth.stressed_states(seed + 1, k, n, "mixed")
    px[4 * k:5 * k], py[4 * k:5 * k] = st["x"], st["y"]
    cl = synth.stressed_states(seed + 2, E - 5 * k, n, "cluster")
    px[5 * k:], py[5 * k:] = cl["x"], cl["y"]
    ix, iy = synth.inward_commands(px[5 * k:], py[5 * k:], speed=0.25)
    ux[5 * k:], uy[5 * k:] = ix, iy
    return px, py, ux, uy


def _certificate(R, ctx, p, tdt, px, py, uxn, uyn):
    import torch

    E, n = px.shape
    d = [dev(a.ravel(), tdt) for a in (px, py, uxn, uyn)]
    ux = torch.zeros(E * n, dtype=tdt, device="cuda")
    uy = torch.zeros_like(ux)
    inf = torch.full((E,), 255, dtype=torch.uint8, device="cuda")
    qs = torch.zeros((E, R.QPS_COUNT), dtype=torch.int32, device="cuda")
    R.barrier_certificate(ctx, p, E, n, *d, ux, uy, infeasible=inf, qp_stats=qs)
    torch.cuda.synchronize()
    return (host(ux).reshape(E, n).astype(np.float64), host(uy).reshape(E, n).astype(np.float64),
            host(inf), host(qs))


@pytest.mark.parametrize("kind", ["f32", "f64"])
@pytest.mark.parametrize("n", [8, 12, 16])
def test_every_solver_stage_runs_and_matches_oracle(orc, n, kind):
    import torch

    R, ctx = ctx_and_lib()
    tdt, ndt = (torch.float32, np.float32) if kind == "f32" else (torch.float64, np.float64)
    E = 600
    px, py, uxn, uyn = (a.astype(ndt) for a in _stage_inputs(100 + n, E, n))
    p = R.params(dtype=R.RS_F64 if kind == "f64" else R.RS_F32)
    banner(f"solver stages n={n} {kind}")
    ctx.qp_failures(reset=True)
    gux, guy, ginf, qs = _certificate(R, ctx, p, tdt, px, py, uxn, uyn)
    # one solve per env: exactly one of the outcome slots is 1
    np.testing.assert_array_equal(qs[:, :R.QPS_ITERATIONS].sum(axis=1), 1)
    stage = np.argmax(qs[:, :R.QPS_ITERATIONS], axis=1)
    assert (qs[:, R.QPS_CAPPED] == 0).all()
    np.testing.assert_array_equal(ginf == 1, stage == R.QPS_INFEASIBLE)
    assert (ginf != 2).all()
    po = orc.Params()
    tol = 1e-4 if kind == "f32" else 1e-9
    worst = np.zeros(len(STAGES))
    for e in range(E):
        oux, ouy, _, status, _, _ = orc.barrier_certificate(
            po, px[e].astype(np.float64), py[e].astype(np.float64), uxn[e].astype(np.float64),
            uyn[e].astype(np.float64))
        assert status in (0, 1)
        assert int(ginf[e]) == status, f"env {e}: status {ginf[e]} vs oracle {status}"
        if status == 1:
            continue
        d = max(np.abs(gux[e] - oux).max(), np.abs(guy[e] - ouy).max())
        s = int(stage[e])
        worst[s] = max(worst[s], d)
        assert d <= tol, f"env {e} (stage {STAGES[s]}): |u_gpu - u_oracle| = {d}"
    counts = {STAGES[s]: int((stage == s).sum()) for s in range(len(STAGES))}
    its = qs[:, R.QPS_ITERATIONS][stage >= R.QPS_ACTIVE_SET]
    print(f"n={n} {kind}: stage counts {counts}, infeasible {int((ginf == 1).sum())}, "
          f"worst |du| per stage {dict(zip(STAGES, worst.round(12)))}, "
          f"active-set iterations mean {its.mean() if its.size else 0:.2f} max "
          f"{its.max() if its.size else 0}")
    for s, name in enumerate(STAGES):
        assert counts[name] >= 3, f"stage {name} ran for {counts[name]} envs only"
    inf_n, cap_n = ctx.qp_failures()
    assert cap_n == 0 and inf_n == int((ginf == 1).sum())


def test_iteration_cap_is_reported_by_barrier_and_env_step(orc):
    import torch

    R, ctx = ctx_and_lib()
    n, E = 12, 600
    px, py, uxn, uyn = (a.astype(np.float32) for a in _stage_inputs(7, E, n))
    banner("iteration cap: barrier_certificate")
    full = _certificate(R, ctx, R.params(), torch.float32, px, py, uxn, uyn)
    ctx.qp_failures(reset=True)
    capped = _certificate(R, ctx, R.params(qp_max_iters=1), torch.float32, px, py, uxn, uyn)
    stage_full = np.argmax(full[3][:, :R.QPS_ITERATIONS], axis=1)
    looped = stage_full >= R.QPS_ACTIVE_SET
    hit = capped[3][:, R.QPS_CAPPED] == 1
    assert looped.sum() >= 5 and hit.sum() >= 5
    # status 2 exactly where the counters say the cap stopped the solve, only
    # for envs that needed the active-set loop
    np.testing.assert_array_equal(capped[2] == 2, hit)
    assert not (hit & ~looped).any()
    # the closed-form stages do not iterate: their commands are unchanged
    same = ~looped & (full[2] == 0)
    np.testing.assert_array_equal(capped[0][same], full[0][same])
    np.testing.assert_array_equal(capped[1][same], full[1][same])
    inf_n, cap_n = ctx.qp_failures(reset=True)
    assert cap_n == int(hit.sum())

    banner("iteration cap: env_step")
    st = synth.stressed_states(8, 300, n, "cluster")
    b = batch_from_states(R, st, n, torch.float32)
    status = torch.full((300,), 255, dtype=torch.uint8, device="cuda")
    qs = torch.zeros((300, R.QPS_COUNT), dtype=torch.int32, device="cuda")
    for t in range(5):
        R.env_step(ctx, R.params(qp_max_iters=1), b, t_global=t, infeasible=status, qp_stats=qs)
    torch.cuda.synchronize()
    q = host(qs)
    np.testing.assert_array_equal(q[:, :R.QPS_ITERATIONS].sum(axis=1), 5)
    _, cap_n = ctx.qp_failures(reset=True)
    assert q[:, R.QPS_CAPPED].sum() == cap_n > 0
    # the last step's status output agrees with its counters' last increment
    assert set(np.unique(host(status))) <= {0, 1, 2}


def test_iteration_cap_is_reported_by_rollout_and_env_run(orc):
    import torch

    R, ctx = ctx_and_lib()
    n, E, H = 8, 256, 8
    st = synth.stressed_states(9, E, n, "cluster")
    w = synth.policy_weights(9, 2 * n + 4)
    bf = lambda a: torch.from_numpy(a).to(torch.bfloat16).cuda().contiguous()
    fl = lambda a: torch.from_numpy(a).float().cuda().contiguous()
    pol = R.Policy(bf(w["w1"]), fl(w["b1"]), bf(w["w2"]), fl(w["b2"]), bf(w["w3"]), fl(w["b3"]))
    dim = 2 * n + 4
    bufs = lambda: (torch.zeros(H * E * n * dim, device="cuda"),
                    torch.zeros(H * E * n, dtype=torch.uint8, device="cuda"),
                    torch.zeros(H * E, device="cuda"),
                    torch.zeros(H * E, dtype=torch.uint8, device="cuda"))
    banner("iteration cap: rollout")
    out = {}
    for cap in (0, 1):
        b = batch_from_states(R, st, n, torch.float32)
        qs = torch.zeros((E, R.QPS_COUNT), dtype=torch.int32, device="cuda")
        ctx.qp_failures(reset=True)
        R.rollout(ctx, R.params(qp_max_iters=cap, seed=9), b, pol, H, 0, *bufs(), qp_stats=qs)
        out[cap] = (host(qs).copy(), ctx.qp_failures(reset=True))
    q0, (_, c0) = out[0]
    q1, (_, c1) = out[1]
    np.testing.assert_array_equal(q0[:, :R.QPS_ITERATIONS].sum(axis=1), H)
    np.testing.assert_array_equal(q1[:, :R.QPS_ITERATIONS].sum(axis=1), H)
    assert c0 == 0 and q0[:, R.QPS_CAPPED].sum() == 0
    assert q0[:, R.QPS_ACTIVE_SET:R.QPS_GENERAL + 1].sum() > 0
    assert c1 == q1[:, R.QPS_CAPPED].sum() > 0
    # the statistics kernel steps exactly like the plain one
    b1 = batch_from_states(R, st, n, torch.float32)
    b2 = batch_from_states(R, st, n, torch.float32)
    R.rollout(ctx, R.params(seed=9), b1, pol, H, 0, *bufs())
    R.rollout(ctx, R.params(seed=9), b2, pol, H, 0, *bufs(),
              qp_stats=torch.zeros((E, R.QPS_COUNT), dtype=torch.int32, device="cuda"))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host(b1.x), host(b2.x))

    banner("iteration cap: env_run")
    counts = np.full(E, n, np.int32)
    plan = R.Plan(ctx, counts)
    for cap in (0, 1):
        b = batch_from_states(R, st, n, torch.float32)
        b.robots = 0
        qs = torch.zeros((E, R.QPS_COUNT), dtype=torch.int32, device="cuda")
        ctx.qp_failures(reset=True)
        R.env_run(ctx, R.params(qp_max_iters=cap), plan, b, H, qp_stats=qs)
        q = host(qs)
        _, c = ctx.qp_failures(reset=True)
        np.testing.assert_array_equal(q[:, :R.QPS_ITERATIONS].sum(axis=1), H)
        assert c == q[:, R.QPS_CAPPED].sum()
        assert (c > 0) == (cap == 1)


def test_qp_failures_counts_infeasible_envs(orc):
    """Overlapping robots (an unsafe state) make the constraint set empty: the
    status output, the counters and the oracle agree."""
    import torch

    R, ctx = ctx_and_lib()
    n, E = 4, 64
    px, py, uxn, uyn = (a.astype(np.float32) for a in _stage_inputs(5, E, n))
    px[::4, 1] = px[::4, 0]  # robots 0 and 1 of every 4th env coincide
    py[::4, 1] = py[::4, 0]
    ctx.qp_failures(reset=True)
    _, _, ginf, qs = _certificate(R, ctx, R.params(), torch.float32, px, py, uxn, uyn)
    inf_n, cap_n = ctx.qp_failures(reset=True)
    po = orc.Params()
    ostat = np.array([orc.barrier_certificate(po, px[e].astype(np.float64),
                                              py[e].astype(np.float64),
                                              uxn[e].astype(np.float64),
                                              uyn[e].astype(np.float64))[3] for e in range(E)])
    np.testing.assert_array_equal(ginf, ostat)
    assert inf_n == int((ostat == 1).sum()) >= E // 4
    assert cap_n == 0
    np.testing.assert_array_equal(qs[:, R.QPS_INFEASIBLE], (ostat == 1).astype(np.int32))
