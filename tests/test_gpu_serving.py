"""GPU tests of the continuous-batching server: every request's result is the
same alone and in the mix (bit for bit), equals a plain env_run of the same
environments and the FP64 oracle's free run of them, and the HBM budget
bounds what is admitted."""
import numpy as np
import pytest

from tests.gpu_util import banner, ctx_and_lib, host

pytestmark = pytest.mark.gpu

REQS = [  # id, envs, robots, horizon
    (1, 70, 3, 50), (2, 200, 8, 37), (3, 33, 16, 61), (4, 128, 5, 20), (5, 90, 12, 45),
    (6, 64, 4, 100), (7, 17, 9, 13),
]


def _serve(R, ctx, reqs, budget, tick, **kw):
    srv = R.Server(ctx, R.params(seed=3, **kw), budget, tick)
    for rid, e, n, h in reqs:
        srv.submit(rid, e, n, h)
    out = {}
    guard = 0
    while True:
        busy = srv.tick()
        while True:
            res = srv.poll_results(256, 16)
            if res is None:
                break
            info, xy, rs = res
            out[info.id] = (xy.copy(), rs.copy(), info.submit_time, info.admit_time,
                            info.finish_time)
        if not busy:
            break
        guard += 1
        assert guard < 10000
    stats = srv.stats()
    srv.close()
    return out, stats


def test_results_alone_equal_results_in_mix():
    R, ctx = ctx_and_lib()
    total = sum(R.Server.request_bytes(e, n) for _, e, n, _ in REQS)
    budget = total // 2  # forces queueing
    banner("serving mix")
    mix, stats = _serve(R, ctx, REQS, budget, tick=16)
    assert sorted(mix) == [r[0] for r in REQS]
    assert stats.peak_bytes <= budget
    assert stats.finished == len(REQS)
    assert stats.robot_steps == sum(e * n * h for _, e, n, h in REQS)
    waited = [rid for rid, v in mix.items() if v[3] > v[2] + 1e-4]
    assert waited, "the budget should have queued some requests"
    for req in REQS:
        banner(f"serving alone {req[0]}")
        # same tick length: the per-tick partial reward sums group the same steps
        alone, _ = _serve(R, ctx, [req], R.Server.request_bytes(req[1], req[2]) + 4096, tick=16)
        np.testing.assert_array_equal(alone[req[0]][0], mix[req[0]][0])
        np.testing.assert_array_equal(alone[req[0]][1], mix[req[0]][1])


def test_server_matches_plain_env_run():
    import torch

    R, ctx = ctx_and_lib()
    rid, e, n, h = 9, 150, 6, 40
    banner("serving vs env_run")
    got, _ = _serve(R, ctx, [(rid, e, n, h)], 1 << 24, tick=11)
    plan = R.Plan(ctx, np.full(e, n, np.int32))
    b = R.Batch.empty(e, n, env_id_base=rid << 20)
    p = R.params(seed=3)
    R.env_reset_mixed(ctx, p, plan, b)
    rsum = torch.zeros(e, device="cuda")
    R.env_run(ctx, p, plan, b, h, t_global0=0, reward_sum=rsum)
    torch.cuda.synchronize()
    xy = np.stack([host(b.x), host(b.y)], 1).reshape(e, n, 2)
    np.testing.assert_array_equal(got[rid][0], xy)
    # reward sums are accumulated per tick on the server, per launch here
    np.testing.assert_allclose(got[rid][1], host(rsum), rtol=1e-5, atol=1e-4)


def test_served_requests_match_the_oracle(orc):
    """Requests served together, each env stepped by the oracle on its own
    (reset from the sampler with env id (id << 20 | e), episode 0; drawn
    actions at stream time = the env's step count; FP64 free run): final
    positions within horizon x 1e-5 m, reward sums within N x horizon x 1e-5."""
    R, ctx = ctx_and_lib()
    reqs = [(3, 6, 3, 17), (4, 5, 6, 20), (5, 4, 10, 12), (6, 3, 16, 9)]
    banner("serving vs oracle")
    got, stats = _serve(R, ctx, reqs, 1 << 20, tick=4)
    assert stats.finished == len(reqs)
    po = orc.Params(seed=3)
    worst = 0.0
    for rid, envs, n, h in reqs:
        xy, rsum = got[rid][0], got[rid][1]
        for e in range(envs):
            env_id = (rid << 20) | e
            x, y, th, gx, gy = orc.reset_env(po, env_id, 0, n)
            st = {"x": x, "y": y, "th": th, "gx": gx, "gy": gy, "step": 0, "episode": 0}
            total = 0.0
            for t in range(h):
                out = orc.env_step(po, st, env_id, t)
                assert out["status"] != 2
                total += out["reward"]
            d = max(np.abs(xy[e, :, 0] - st["x"]).max(), np.abs(xy[e, :, 1] - st["y"]).max())
            worst = max(worst, d)
            assert d <= h * 1e-5, f"request {rid} env {e}: final position gap {d}"
            assert abs(rsum[e] - total) <= n * h * 1e-5, f"request {rid} env {e}: reward sum"
            assert st["step"] == h and st["episode"] == 0
    print(f"served vs oracle: worst final position gap {worst:.3g}")


def test_server_uses_the_parameters_iteration_cap():
    """A server created with qp_max_iters > 0 solves with that cap, as env_run
    does for the same parameters (cap 1 stops every active-set solve)."""
    import torch

    R, ctx = ctx_and_lib()
    rid, e, n, h = 12, 120, 12, 60
    banner("serving iteration cap")
    ctx.qp_failures(reset=True)
    got, _ = _serve(R, ctx, [(rid, e, n, h)], 1 << 24, tick=16, qp_max_iters=1)
    _, served_capped = ctx.qp_failures(reset=True)
    plan = R.Plan(ctx, np.full(e, n, np.int32))
    b = R.Batch.empty(e, n, env_id_base=rid << 20)
    p = R.params(seed=3, qp_max_iters=1)
    R.env_reset_mixed(ctx, p, plan, b)
    R.env_run(ctx, p, plan, b, h, t_global0=0)
    torch.cuda.synchronize()
    _, run_capped = ctx.qp_failures(reset=True)
    assert served_capped == run_capped > 0
    xy = np.stack([host(b.x), host(b.y)], 1).reshape(e, n, 2)
    np.testing.assert_array_equal(got[rid][0], xy)


def test_over_budget_request_is_refused():
    R, ctx = ctx_and_lib()
    srv = R.Server(ctx, R.params(), 1 << 16, 8)
    with pytest.raises(R.RobostepError) as ei:
        srv.submit(1, 4000, 16, 10)
    assert ei.value.status == 5
    with pytest.raises(R.RobostepError):
        srv.submit(2, 10, 17, 10)
    srv.close()
