"""Seeded synthetic inputs for the batched Robotarium step.

This module only draws inputs: robot states, nominal commands, policy weights,
mixed-size batches and request streams. It holds none of the simulator's
arithmetic (no controller, certificate, dynamics or observation), so the HIP
path and the FP64 oracle can both be fed from it without sharing any of the
method.

The workloads mirror the navigation setting of JaxRobotarium (arXiv 2505.06771,
Sec. 4.2 and the Navigation scenario of the appendix): robots in a
3.2 m x 2 m arena, start poses with a 0.3 m minimum separation, goals uniform in
the arena, headings uniform. The stressed generators add the configurations
that make the certificate hard: tight clusters, robots at the walls, pairs at
the safety radius, collinear triples and overlapping (unsafe) robots.
"""
from __future__ import annotations

import math

import numpy as np

ARENA = (-1.6, 1.6, -1.0, 1.0)
SAFETY_RADIUS = 0.17


def _uniform_separated(rng, n, box, min_sep, max_tries=10000):
    """n points uniform in box with pairwise distance >= min_sep (rejection)."""
    xs, ys = [], []
    tries = 0
    while len(xs) < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place points")
        x = rng.uniform(box[0], box[1])
        y = rng.uniform(box[2], box[3])
        if all((x - a) ** 2 + (y - b) ** 2 >= min_sep ** 2 for a, b in zip(xs, ys)):
            xs.append(x)
            ys.append(y)
    return np.array(xs), np.array(ys)


def random_states(seed: int, num_envs: int, n: int, margin: float = 0.2, min_sep: float = 0.3):
    """Navigation start states: dict of float64 arrays [E, n] (x, y, th, gx, gy)."""
    rng = np.random.default_rng(seed)
    box = (ARENA[0] + margin, ARENA[1] - margin, ARENA[2] + margin, ARENA[3] - margin)
    out = {k: np.zeros((num_envs, n)) for k in ("x", "y", "th", "gx", "gy")}
    for e in range(num_envs):
        out["x"][e], out["y"][e] = _uniform_separated(rng, n, box, min_sep)
        out["gx"][e], out["gy"][e] = _uniform_separated(rng, n, box, min_sep)
        out["th"][e] = rng.uniform(-math.pi, math.pi, n)
    return out


def stressed_states(seed: int, num_envs: int, n: int, kind: str):
    """States where the certificate binds. kind in
    {'cluster', 'wall', 'tangent', 'collinear', 'corner', 'mixed'}."""
    rng = np.random.default_rng(seed)
    out = random_states(seed + 7919, num_envs, n)
    kinds = ["cluster", "wall", "tangent", "collinear", "corner"]
    for e in range(num_envs):
        k = kinds[rng.integers(len(kinds))] if kind == "mixed" else kind
        if k == "cluster":
            cx, cy = rng.uniform(-1.0, 1.0), rng.uniform(-0.5, 0.5)
            # hexagonal-ish packing just above the safety radius (projection
            # points are 5 cm ahead of the centres, so some pairs start tight)
            pitch = rng.uniform(0.2, 0.26)
            pts = []
            ring = 0
            while len(pts) < n:
                if ring == 0:
                    pts.append((0.0, 0.0))
                else:
                    for s in range(6 * ring):
                        a = 2 * math.pi * s / (6 * ring) + rng.uniform(-0.05, 0.05)
                        pts.append((ring * pitch * math.cos(a), ring * pitch * math.sin(a)))
                ring += 1
            pts = np.array(pts[:n])
            out["x"][e] = np.clip(cx + pts[:, 0], -1.45, 1.45)
            out["y"][e] = np.clip(cy + pts[:, 1], -0.85, 0.85)
        elif k == "wall":
            side = rng.integers(4)
            t = np.sort(rng.uniform(-0.8, 0.8, n)) * (1.8 if side < 2 else 1.0)
            t = t + 0.3 * np.arange(n) - 0.15 * (n - 1)
            if side < 2:
                out["y"][e] = np.clip(t, -0.9, 0.9)
                out["x"][e] = (1.0 if side == 0 else -1.0) * rng.uniform(1.38, 1.5, n)
            else:
                out["x"][e] = np.clip(t, -1.5, 1.5)
                out["y"][e] = (1.0 if side == 2 else -1.0) * rng.uniform(0.78, 0.9, n)
        elif k == "tangent":
            xs, ys = _uniform_separated(rng, (n + 1) // 2, (-1.3, 1.3, -0.7, 0.7), 0.6)
            d = rng.uniform(0.17, 0.23, xs.size)
            a = rng.uniform(-math.pi, math.pi, xs.size)
            px = np.concatenate([xs, xs + d * np.cos(a)])[:n]
            py = np.concatenate([ys, ys + d * np.sin(a)])[:n]
            out["x"][e], out["y"][e] = px, py
        elif k == "collinear":
            a = rng.uniform(-math.pi, math.pi)
            pitch = rng.uniform(0.2, 0.24)
            off = (np.arange(n) - (n - 1) / 2) * pitch
            cx, cy = rng.uniform(-0.3, 0.3), rng.uniform(-0.2, 0.2)
            out["x"][e] = np.clip(cx + off * math.cos(a), -1.5, 1.5)
            out["y"][e] = np.clip(cy + off * math.sin(a), -0.9, 0.9)
        elif k == "corner":
            sx, sy = rng.choice([-1.0, 1.0]), rng.choice([-1.0, 1.0])
            g = int(math.ceil(math.sqrt(n)))
            ii = np.arange(n)
            out["x"][e] = sx * (1.45 - 0.22 * (ii % g))
            out["y"][e] = sy * (0.85 - 0.22 * (ii // g))
        else:
            raise ValueError(kind)
    return out


def nominal_commands(seed: int, shape, speed: float = 0.3):
    """Random single-integrator commands, some above the 0.2 m/s limit so the
    magnitude pre-clip is exercised."""
    rng = np.random.default_rng(seed)
    r = speed * np.sqrt(rng.uniform(0.0, 1.0, shape))
    a = rng.uniform(-math.pi, math.pi, shape)
    return r * np.cos(a), r * np.sin(a)


def inward_commands(px, py, speed: float = 0.2):
    """Commands that push every robot toward the centroid of its environment
    (makes pairwise rows bind)."""
    cx = px.mean(axis=-1, keepdims=True)
    cy = py.mean(axis=-1, keepdims=True)
    dx, dy = cx - px, cy - py
    nrm = np.maximum(np.hypot(dx, dy), 1e-9)
    return speed * dx / nrm, speed * dy / nrm


def random_actions(seed: int, shape):
    return np.random.default_rng(seed).integers(0, 5, shape).astype(np.uint8)


def policy_weights(seed: int, in_dim: int, hidden: int = 64, n_actions: int = 5,
                   bias_scale: float = 0.0):
    """Seeded MLP weights U(+-1/sqrt(fan_in)), rounded to bfloat16 by torch.
    Returns float32 arrays holding bf16 values: w1 [in,h], w2 [h,h], w3 [h,5]
    (row-major [in][out]) and float32 biases."""
    import torch

    rng = np.random.default_rng(seed)

    def mat(fan_in, fan_out):
        b = 1.0 / math.sqrt(fan_in)
        w = torch.from_numpy(rng.uniform(-b, b, (fan_in, fan_out)).astype(np.float32))
        return w.to(torch.bfloat16).to(torch.float32).numpy()

    w1, w2, w3 = mat(in_dim, hidden), mat(hidden, hidden), mat(hidden, n_actions)
    b1 = (bias_scale * rng.standard_normal(hidden)).astype(np.float32)
    b2 = (bias_scale * rng.standard_normal(hidden)).astype(np.float32)
    b3 = (bias_scale * rng.standard_normal(n_actions)).astype(np.float32)
    return {"w1": w1, "b1": b1, "w2": w2, "b2": b2, "w3": w3, "b3": b3}


def uneven_sizes(seed: int, num_envs: int, sizes=(2, 4, 6, 8, 12),
                 proportions=(0.1, 0.3, 0.3, 0.2, 0.1)):
    """Robot counts per env: exact largest-remainder counts, seeded shuffle."""
    quotas = [num_envs * p for p in proportions]
    counts = [int(math.floor(q)) for q in quotas]
    rem = num_envs - sum(counts)
    order = sorted(range(len(sizes)), key=lambda k: -(quotas[k] - counts[k]))
    for k in order[:rem]:
        counts[k] += 1
    arr = np.concatenate([np.full(c, s, np.int32) for s, c in zip(sizes, counts)])
    np.random.default_rng(seed).shuffle(arr)
    return arr


def request_stream(seed: int, count: int, rate_hz: float, e_range=(64, 4096), n_range=(3, 16),
                   h_range=(50, 500)):
    """Poisson arrivals of rollout requests: list of dicts with arrival time
    (s), envs (log-uniform), robots (uniform), horizon (uniform)."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate_hz, count))
    envs = np.exp(rng.uniform(math.log(e_range[0]), math.log(e_range[1]), count))
    envs = np.clip(np.round(envs).astype(np.int64), e_range[0], e_range[1])
    robots = rng.integers(n_range[0], n_range[1] + 1, count)
    horizon = rng.integers(h_range[0], h_range[1] + 1, count)
    return [{"id": k, "arrival": float(t[k]), "envs": int(envs[k]), "robots": int(robots[k]),
             "horizon": int(horizon[k])} for k in range(count)]
