"""Helpers of the GPU parity tests: device transfers and oracle state views."""
import math
import sys

import numpy as np


def banner(msg: str):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def ctx_and_lib():
    import torch

    from paper_2505_06771_amd import robostep as R

    assert torch.cuda.is_available(), "GPU test needs a GPU"
    R.lib()  # raises if the HIP library is missing
    return R, R.Context(0)


def dev(a, dtype):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype).contiguous()


def host(t):
    return t.detach().cpu().numpy()


def batch_from_states(R, st, n, dtype, env_id_base=0, step=None, episode=None):
    import torch

    E = st["x"].shape[0]
    b = R.Batch(dev(st["x"].ravel(), dtype), dev(st["y"].ravel(), dtype),
                dev(st["th"].ravel(), dtype), dev(st["gx"].ravel(), dtype),
                dev(st["gy"].ravel(), dtype),
                dev(np.zeros(E, np.int32) if step is None else step, torch.int32),
                dev(np.zeros(E, np.int32) if episode is None else episode, torch.int32),
                n, env_id_base)
    return b


def oracle_state(b):
    """Float64 copies of a device batch for the oracle's batched calls."""
    return {"x": host(b.x).astype(np.float64), "y": host(b.y).astype(np.float64),
            "th": host(b.theta).astype(np.float64), "gx": host(b.goal_x).astype(np.float64),
            "gy": host(b.goal_y).astype(np.float64),
            "step": host(b.step).astype(np.int32).copy(),
            "episode": host(b.episode).astype(np.int32).copy()}


def angle_diff(a, b):
    d = np.asarray(a, np.float64) - np.asarray(b, np.float64)
    return np.abs((d + math.pi) % (2 * math.pi) - math.pi)


def prey_candidates(po, qx, qy):
    """The prey's 17 candidate positions (stay, then 16 directions), rebuilt
    from their definition for the band checks of the Predator-Prey tests."""
    s = po.prey_speed * po.dt
    lox, hix = po.x_min + po.safety_radius / 2, po.x_max - po.safety_radius / 2
    loy, hiy = po.y_min + po.safety_radius / 2, po.y_max - po.safety_radius / 2
    ang = 2 * math.pi * np.arange(16) / 16
    cx = np.concatenate([[qx], np.clip(qx + s * np.cos(ang), lox, hix)])
    cy = np.concatenate([[qy], np.clip(qy + s * np.sin(ang), loy, hiy)])
    return cx, cy


def prey_band(orc, po, x, y, qx, qy, gpu_qx, gpu_qy, tol=1e-5):
    """True when the GPU's prey position is a candidate whose oracle score is
    within `tol` (m^2) of the best one: a near-tie that FP32 rounding may
    resolve either way."""
    _, _, k, sc = orc.prey_move(po, x, y, qx, qy)
    cx, cy = prey_candidates(po, qx, qy)
    d = np.hypot(cx - gpu_qx, cy - gpu_qy)
    j = int(np.argmin(d))
    return d[j] <= 1e-5 and sc[k] - sc[j] <= tol


def tag_band(po, x, y, qx, qy, tol=1e-5):
    """True when some robot centre is within `tol` of the tag radius."""
    d = np.hypot(np.asarray(x) - qx, np.asarray(y) - qy)
    return bool((np.abs(d - po.tag_radius) < tol).any())


def pose_band(po, th, actions, tol=1e-4):
    """Robots whose pose-controller bearing (controller 3) lies within `tol` of
    +-pi: the goal straight behind, where the law turns one way or the other
    and FP32 rounding may pick either. th, actions: arrays of one shape."""
    if getattr(po, "controller", 0) != 3:
        return np.zeros(np.shape(th), bool)
    a = np.asarray(actions)
    dx = (a == 1).astype(np.float64) - (a == 2)
    dy = (a == 3).astype(np.float64) - (a == 4)
    c, s = np.cos(th), np.sin(th)
    ca, sa = c * dx + s * dy, c * dy - s * dx
    return (a != 0) & (ca < 0) & (np.abs(sa) < tol)
