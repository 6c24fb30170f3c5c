"""Oracle pins for the policy MLP and the categorical draw.

The MLP reduces to three GEMMs with bf16 rounding between layers; it is pinned
to torch float64 matmuls on the same bf16-rounded tensors (rounding by torch).
The inverse-CDF draw is pinned to numpy's searchsorted over the softmax CDF and
to closed forms (uniform logits, one dominant logit)."""
import numpy as np
import pytest

from paper_2505_06771_amd import synth


def test_mlp_matches_textbook_gemm(orc):
    torch = pytest.importorskip("torch")
    w = synth.policy_weights(3, 20, bias_scale=0.1)
    rng = np.random.default_rng(4)
    obs = rng.uniform(-2, 2, (3000, 20)).astype(np.float32).astype(np.float64)

    def bf(t):
        return t.to(torch.float32).to(torch.bfloat16).to(torch.float64)

    W = {k: torch.from_numpy(v.astype(np.float64)) for k, v in w.items()}
    X = bf(torch.from_numpy(obs))
    h1 = bf(torch.relu(X @ W["w1"] + W["b1"]))
    h2 = bf(torch.relu(h1 @ W["w2"] + W["b2"]))
    ref = (h2 @ W["w3"] + W["b3"]).numpy()
    got = np.stack([orc.policy_logits(w, o) for o in obs])
    close = np.abs(got - ref).max(axis=1) < 1e-12
    # torch rounds the FP64 sums through FP32 before bf16; the two can differ
    # only for sums within 2^-24 of a bf16 midpoint
    assert close.mean() > 0.995
    assert np.abs(got - ref).max() < 0.05


def test_sample_inverse_cdf(orc):
    rng = np.random.default_rng(0)
    for _ in range(2000):
        logits = rng.standard_normal(5) * 2
        r = int(rng.integers(0, 2 ** 32))
        u = (r >> 8) * 2.0 ** -24
        pr = np.exp(logits - logits.max())
        pr /= pr.sum()
        k = int(np.searchsorted(np.cumsum(pr), u, side="right"))
        assert orc.sample_action(logits, r) == min(k, 4)


def test_sample_closed_forms(orc):
    for r in [0, 1 << 8, 2 ** 32 - 1, 0x33333333, 0x66666666, 0x99999999, 0xCCCCCCCC]:
        u = (r >> 8) * 2.0 ** -24
        assert orc.sample_action(np.zeros(5), r) == min(int(u * 5), 4)
        # exp(-1000) underflows to 0: all mass on action 2
        assert orc.sample_action(np.array([-1000.0, -1000.0, 0.0, -1000.0, -1000.0]), r) == 2
