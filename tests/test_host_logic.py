"""CPU tests of host-side logic: seeded workload generators and the
benchmark's algorithmic byte count."""
import math

import numpy as np

from paper_2505_06771_amd import synth


def test_uneven_sizes_exact_counts():
    arr = synth.uneven_sizes(0, 8192)
    counts = {n: int((arr == n).sum()) for n in (2, 4, 6, 8, 12)}
    # largest remainder of 0.1/0.3/0.3/0.2/0.1 of 8192
    assert counts == {2: 819, 4: 2458, 6: 2458, 8: 1638, 12: 819}
    assert arr.sum() == 49150
    # seeded shuffle: deterministic, and not sorted
    assert np.array_equal(arr, synth.uneven_sizes(0, 8192))
    assert not np.array_equal(arr, np.sort(arr))


def test_request_stream_ranges():
    reqs = synth.request_stream(3, 2000, 50.0)
    env = np.array([r["envs"] for r in reqs])
    rob = np.array([r["robots"] for r in reqs])
    hor = np.array([r["horizon"] for r in reqs])
    arr = np.array([r["arrival"] for r in reqs])
    assert env.min() >= 64 and env.max() <= 4096
    assert rob.min() >= 3 and rob.max() <= 16 and set(rob) == set(range(3, 17))
    assert hor.min() >= 50 and hor.max() <= 500
    assert (np.diff(arr) > 0).all()
    # Poisson process: mean gap 1/rate; log-uniform envs: mean of log
    assert abs(np.diff(arr).mean() - 1 / 50.0) < 0.003
    assert abs(np.log(env).mean() - 0.5 * (math.log(64) + math.log(4096))) < 0.1


def test_random_states_respect_separation():
    st = synth.random_states(1, 50, 8)
    for e in range(50):
        d = np.hypot(st["x"][e][:, None] - st["x"][e][None], st["y"][e][:, None] - st["y"][e][None])
        d[np.arange(8), np.arange(8)] = 1e9
        assert d.min() >= 0.3
        assert np.abs(st["x"][e]).max() <= 1.4 and np.abs(st["y"][e]).max() <= 0.8


def test_policy_weights_are_bf16_valued():
    import torch

    w = synth.policy_weights(0, 20)
    for k in ("w1", "w2", "w3"):
        t = torch.from_numpy(w[k])
        assert torch.equal(t.to(torch.bfloat16).to(torch.float32), t)
    assert w["w1"].shape == (20, 64) and w["w3"].shape == (64, 5)
    assert np.abs(w["w1"]).max() <= 1 / math.sqrt(20) + 1e-3


def test_rollout_algorithmic_bytes():
    import bench

    E, N, H = 16384, 8, 128
    b = bench.rollout_algorithmic_bytes(E, N, H)
    per_robot_step = 4 * 20 + 1 + 5 / 8  # obs, action, reward+done per env
    assert abs(b / (E * N * H) - per_robot_step) < 0.5  # state and weights amortised
    assert b > E * N * H * per_robot_step


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys

    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], capture_output=True, text=True)
    assert r.returncode == 2 and "one GPU" in r.stderr
