"""Explains a sampled action on which the GPU rollout and the FP64 oracle
disagree, or reports that nothing does.

Both sides evaluate the policy on the same (GPU) observation, rounded to
bfloat16; the oracle sums in FP64, the GPU's MFMA in FP32. Products of two
bf16 values are exact in FP32, so the only difference is the FP32 summation:
at most about k * 2^-24 * (|b| + sum_k |x_k w_k|) for a sum of k products.
A hidden unit whose exact pre-activation lies that close to a bf16 rounding
midpoint may round to the neighbouring bf16 on the GPU. A disagreement is
explained when one such flip (of one unit of either hidden layer), propagated
through the rest of the network in FP64, makes the oracle draw the GPU's
action from the same uniform, or when the uniform lies within 1e-5 of the
cumulative-probability boundary between the two actions (FP32 softmax
rounding). Anything else is a defect.
"""
import numpy as np

EPS24 = 2.0 ** -24
CDF_BAND = 1e-5


def bf16(a):
    """Round to the nearest bfloat16, ties to even (float64 in and out)."""
    a = np.asarray(a, np.float64)
    m, e = np.frexp(a)
    return np.ldexp(np.rint(m * 256.0) / 256.0, e)


def _sample(logits, u):
    pr = np.exp(logits - logits.max())
    cdf = np.cumsum(pr / pr.sum())
    k = int(np.searchsorted(cdf[:4], u, side="right"))
    return min(k, 4), cdf


def _alternatives(s, err):
    """bf16 values other than the nominal one that relu(s') may round to for
    s' within err of s (unit by unit); nominal = bf16(relu(s))."""
    nom = bf16(np.maximum(s, 0.0))
    lo = bf16(np.maximum(s - err, 0.0))
    hi = bf16(np.maximum(s + err, 0.0))
    out = []
    for k in np.nonzero((lo != nom) | (hi != nom))[0]:
        for v in {float(lo[k]), float(hi[k])} - {float(nom[k])}:
            out.append((int(k), v))
    return nom, out


def explain(w, obs_row, u, gpu_action):
    """w: bf16-valued float64 weights (w1 [D,64], b1, w2 [64,64], b2, w3 [64,5],
    b3); obs_row: the GPU's observation; u: the 24-bit uniform. Returns
    'cdf', 'layer1:<unit>', 'layer2:<unit>' or None."""
    x = bf16(obs_row)
    d = x.size
    s1 = w["b1"] + x @ w["w1"]
    e1 = 2 * (d + 1) * EPS24 * (np.abs(w["b1"]) + np.abs(x) @ np.abs(w["w1"]))
    h1, alt1 = _alternatives(s1, e1)

    def rest_from_h1(h):
        s2 = w["b2"] + h @ w["w2"]
        return s2, bf16(np.maximum(s2, 0.0))

    s2, h2 = rest_from_h1(h1)
    e2 = 2 * 65 * EPS24 * (np.abs(w["b2"]) + np.abs(h1) @ np.abs(w["w2"]))
    _, alt2 = _alternatives(s2, e2)
    a0, cdf = _sample(w["b3"] + h2 @ w["w3"], u)
    if a0 == gpu_action:
        return "agree"
    lo, hi = min(a0, gpu_action), max(a0, gpu_action)
    if np.abs(cdf[lo:hi] - u).min() < CDF_BAND:
        return "cdf"
    for k, v in alt1:
        h = h1.copy()
        h[k] = v
        _, hh2 = rest_from_h1(h)
        if _sample(w["b3"] + hh2 @ w["w3"], u)[0] == gpu_action:
            return f"layer1:{k}"
    for k, v in alt2:
        h = h2.copy()
        h[k] = v
        if _sample(w["b3"] + h @ w["w3"], u)[0] == gpu_action:
            return f"layer2:{k}"
    return None
