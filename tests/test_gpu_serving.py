"""GPU tests of the continuous-batching server: every request's result is the
same alone and in the mix (bit for bit), equals a plain env_run of the same
environments, and the HBM budget bounds what is admitted."""
import numpy as np
import pytest

from tests.gpu_util import banner, ctx_and_lib, host

pytestmark = pytest.mark.gpu

REQS = [  # id, envs, robots, horizon
    (1, 70, 3, 50), (2, 200, 8, 37), (3, 33, 16, 61), (4, 128, 5, 20), (5, 90, 12, 45),
    (6, 64, 4, 100), (7, 17, 9, 13),
]


def _serve(R, ctx, reqs, budget, tick):
    srv = R.Server(ctx, R.params(seed=3), budget, tick)
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


def test_over_budget_request_is_refused():
    R, ctx = ctx_and_lib()
    srv = R.Server(ctx, R.params(), 1 << 16, 8)
    with pytest.raises(R.RobostepError) as ei:
        srv.submit(1, 4000, 16, 10)
    assert ei.value.status == 5
    with pytest.raises(R.RobostepError):
        srv.submit(2, 10, 17, 10)
    srv.close()
