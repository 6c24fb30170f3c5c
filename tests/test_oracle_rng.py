"""Oracle pins: counter-based stream, discrete draws, bfloat16 rounding.

Philox4x32-10 is pinned to the published known-answer vectors of Salmon et al.
(SC'11), stored in tests/golden/philox4x32_10_kat.txt. bfloat16 rounding is
pinned to torch's float32 -> bfloat16 conversion (a library routine).
"""
import os

import numpy as np
import pytest

pytestmark = []
GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat_rows():
    rows = []
    with open(GOLD) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(t, 16) for t in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat_rows())
def test_philox_known_answers(orc, ctr, key, expect):
    out = orc.philox4x32_10(ctr, key)
    assert [int(x) for x in out] == expect


def test_philox_counter_sensitivity(orc):
    base = orc.philox4x32_10([1, 2, 3, 4], [5, 6])
    for w in range(4):
        c = [1, 2, 3, 4]
        c[w] ^= 1
        assert not np.array_equal(orc.philox4x32_10(c, [5, 6]), base)


def test_random_action_distribution(orc):
    p = orc.Params(seed=12345)
    draws = np.array([orc.random_action(p, e, t, i) for e in range(40) for t in range(50)
                      for i in range(5)])
    assert draws.min() == 0 and draws.max() == 4
    counts = np.bincount(draws, minlength=5)
    expected = draws.size / 5
    chi2 = ((counts - expected) ** 2 / expected).sum()
    assert chi2 < 20.0  # 4 dof, p ~ 5e-4


def test_random_action_is_floor_5r(orc):
    # a = floor(5 r / 2^32) with r the word (i & 3) of block (env, t, 0<<24 | i>>2, 0)
    p = orc.Params(seed=(7 << 32) | 99)
    for env_id, t, i in [(0, 0, 0), (3, 17, 5), (1000, 499, 7), (2 ** 31, 3, 2)]:
        blk = orc.philox4x32_10([env_id & 0xFFFFFFFF, t, i >> 2, 0], [99, 7])
        r = int(blk[i & 3])
        assert orc.random_action(p, env_id, t, i) == (r * 5) >> 32


def test_policy_bits_purpose(orc):
    p = orc.Params(seed=3)
    blk = orc.philox4x32_10([11, 22, (1 << 24) | 1, 0], [3, 0])
    assert orc.policy_bits(p, 11, 22, 6) == int(blk[2])


def test_bf16_round_matches_torch(orc):
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    vals = np.concatenate([
        rng.standard_normal(4000).astype(np.float32),
        (rng.standard_normal(2000) * 1e-3).astype(np.float32),
        (rng.standard_normal(2000) * 1e3).astype(np.float32),
        np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -(1.0 + 2 ** -8), 2 ** -130, 0.0],
                 dtype=np.float32),
    ])
    ref = torch.from_numpy(vals).to(torch.bfloat16).to(torch.float64).numpy()
    mine = np.array([orc.bf16_round(float(v)) for v in vals])
    assert np.array_equal(mine, ref)


def test_bf16_ties_to_even(orc):
    # 1 + 2^-8 lies halfway between 1 and 1 + 2^-7: even mantissa is 1.0
    assert orc.bf16_round(1.0 + 2 ** -8) == 1.0
    # 1 + 3*2^-8 lies halfway between 1 + 2^-7 and 1 + 2^-6: even is 1 + 2^-6
    assert orc.bf16_round(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6
    assert orc.bf16_round(1.0 + 2 ** -8 + 2 ** -30) == 1.0 + 2 ** -7
