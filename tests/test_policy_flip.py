"""CPU pins of the helper that explains sampled-action mismatches between the
GPU rollout and the oracle (tests/policy_flip.py): its bf16 rounding equals
torch's and the oracle's, and it explains exactly the mismatches it should."""
import numpy as np
import pytest

from tests.policy_flip import bf16, explain


def test_bf16_rounding_matches_torch_and_oracle(orc):
    import torch

    rng = np.random.default_rng(0)
    a = np.concatenate([rng.standard_normal(2000) * 10.0 ** rng.integers(-6, 4, 2000),
                        [0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8]])
    a32 = a.astype(np.float32)
    ref = torch.from_numpy(a32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(bf16(a32.astype(np.float64)), ref)
    for v in a32[:200]:
        assert bf16(float(v)) == orc.bf16_round(float(v))


def _net(rng, d=20):
    w = {"w1": bf16(rng.uniform(-0.2, 0.2, (d, 64))), "b1": np.zeros(64),
         "w2": bf16(rng.uniform(-0.125, 0.125, (64, 64))), "b2": np.zeros(64),
         "w3": bf16(rng.uniform(-0.125, 0.125, (64, 5))), "b3": np.zeros(5)}
    return w


def _cdf(w, x):
    h1 = bf16(np.maximum(w["b1"] + bf16(x) @ w["w1"], 0))
    h2 = bf16(np.maximum(w["b2"] + h1 @ w["w2"], 0))
    lg = w["b3"] + h2 @ w["w3"]
    p = np.exp(lg - lg.max())
    return np.cumsum(p / p.sum())


def test_explains_a_draw_at_a_cdf_boundary():
    rng = np.random.default_rng(1)
    w = _net(rng)
    x = rng.uniform(-1, 1, 20)
    c = _cdf(w, x)
    # u just below C_1 draws action 1; the neighbour 2 is explained by the band
    assert explain(w, x, c[1] - 3e-6, 2) == "cdf"
    assert explain(w, x, c[1] - 3e-6, 1) == "agree"


def test_rejects_a_mismatch_far_from_every_boundary():
    rng = np.random.default_rng(2)
    w = _net(rng)
    x = rng.uniform(-1, 1, 20)
    c = _cdf(w, x)
    u = 0.5 * (c[1] + c[2])  # action 2, far from both of its boundaries
    assert explain(w, x, u, 2) == "agree"
    assert explain(w, x, u, 0) is None
    assert explain(w, x, u, 4) is None


def test_explains_a_hidden_unit_at_a_rounding_midpoint():
    """A layer-1 unit whose exact pre-activation sits at a bf16 midpoint (within
    FP32 summation error) may round either way; when the other rounding moves
    the drawn action, the mismatch is explained by that unit."""
    rng = np.random.default_rng(3)
    found = False
    for trial in range(200):
        w = _net(rng)
        x = rng.uniform(-1, 1, 20)
        xb = bf16(x)
        s1 = xb @ w["w1"]
        k = int(np.argmax(s1))
        # move the bias so unit k's exact sum lands on the midpoint above its
        # value, rounding to even (down) there
        v = bf16(s1[k])
        m, e = np.frexp(v)
        ulp = np.ldexp(1.0 / 256.0, e)
        mid = v + ulp / 2 if (np.rint(m * 256) % 2 == 0) else v - ulp / 2
        w["b1"][k] = mid - s1[k]
        s1k = w["b1"][k] + s1[k]
        c_lo = _cdf(w, x)
        h_alt = bf16(np.maximum(w["b1"] + xb @ w["w1"], 0))
        alt = {float(bf16(s1k - 1e-6)), float(bf16(s1k + 1e-6))} - {float(h_alt[k])}
        if not alt:
            continue
        w2 = {kk: vv.copy() for kk, vv in w.items()}
        # the action under the other rounding of unit k
        h1 = h_alt.copy()
        h1[k] = alt.pop()
        h2 = bf16(np.maximum(h1 @ w["w2"], 0))
        lg = h2 @ w["w3"]
        p = np.exp(lg - lg.max())
        c_hi = np.cumsum(p / p.sum())
        # a uniform between the two cumulative sums of some boundary, away
        # from both by more than the 1e-5 band
        for b in range(4):
            lo, hi = sorted((c_lo[b], c_hi[b]))
            if hi - lo > 1e-4:
                u = 0.5 * (lo + hi)
                a_nom = int(np.searchsorted(c_lo[:4], u, side="right"))
                a_alt = int(np.searchsorted(c_hi[:4], u, side="right"))
                if a_nom != a_alt:
                    why = explain(w2, x, u, a_alt)
                    assert why == f"layer1:{k}", why
                    found = True
                    break
        if found:
            break
    assert found
