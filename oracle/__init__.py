"""FP64 CPU oracle of the batched Robotarium environment step (ctypes wrapper).

TEST INFRASTRUCTURE ONLY. Only the test-suite, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package. It shares no code
with the HIP library (``paper_2505_06771_amd``) and must never stand in for it.

The C source (``robostep_oracle.c``) follows JaxRobotarium (arXiv 2505.06771)
Sec. 4.1 (unicycle model, single-integrator controllers, barrier-certificate
QP) and the Navigation scenario of the appendix (observation, reward); the
readings of what the paper leaves unstated are documented in the C source.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, fields

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "robostep_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liborc.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no FP contraction so sums are plain)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared",
               "-D_GNU_SOURCE", _SRC, "-o", _LIB_PATH, "-lm", "-lpthread"]
        subprocess.run(cmd, check=True)
    return _LIB_PATH


class OrcParams(ctypes.Structure):
    _fields_ = [
        ("x_min", ctypes.c_double), ("x_max", ctypes.c_double),
        ("y_min", ctypes.c_double), ("y_max", ctypes.c_double),
        ("dt", ctypes.c_double), ("proj_dist", ctypes.c_double),
        ("barrier_gain", ctypes.c_double), ("safety_radius", ctypes.c_double),
        ("boundary_gain_factor", ctypes.c_double), ("v_max", ctypes.c_double),
        ("action_speed", ctypes.c_double), ("kp", ctypes.c_double),
        ("wheel_radius", ctypes.c_double), ("base_length", ctypes.c_double),
        ("goal_radius", ctypes.c_double), ("reset_margin", ctypes.c_double),
        ("min_sep", ctypes.c_double), ("grid", ctypes.c_double),
        ("max_steps", ctypes.c_int32), ("controller", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("waypoint_step", ctypes.c_double), ("pos_gain", ctypes.c_double),
        ("ang_gain", ctypes.c_double), ("action_noise", ctypes.c_double),
        ("prey_speed", ctypes.c_double), ("tag_radius", ctypes.c_double),
        ("tag_reward", ctypes.c_double), ("scenario", ctypes.c_int32),
        ("pose_gain_rho", ctypes.c_double), ("pose_gain_alpha", ctypes.c_double),
        ("pose_gain_beta", ctypes.c_double),
    ]


@dataclass
class Params:
    """Simulation constants (arena, dt, projection distance, gain, safety radius
    and speed limit of the single-env navigation configuration)."""
    x_min: float = -1.6
    x_max: float = 1.6
    y_min: float = -1.0
    y_max: float = 1.0
    dt: float = 0.033
    proj_dist: float = 0.05
    barrier_gain: float = 100.0
    safety_radius: float = 0.17
    boundary_gain_factor: float = 0.4
    v_max: float = 0.2
    action_speed: float = 0.2
    kp: float = 1.0
    wheel_radius: float = 0.016
    base_length: float = 0.105
    goal_radius: float = 0.05
    reset_margin: float = 0.2
    min_sep: float = 0.3
    grid: float = 1e-4
    max_steps: int = 500
    controller: int = 0
    seed: int = 0
    waypoint_step: float = 0.2
    pos_gain: float = 0.8
    ang_gain: float = math.pi / 2
    action_noise: float = 0.0
    prey_speed: float = 0.3
    tag_radius: float = 0.25
    tag_reward: float = 10.0
    scenario: int = 0
    pose_gain_rho: float = 0.8
    pose_gain_alpha: float = 2.0
    pose_gain_beta: float = 0.5

    def c(self) -> OrcParams:
        return OrcParams(**{f.name: getattr(self, f.name) for f in fields(self)})


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_I32 = ctypes.POINTER(ctypes.c_int32)
_I64 = ctypes.POINTER(ctypes.c_int64)
_U32 = ctypes.POINTER(ctypes.c_uint32)
_U8 = ctypes.POINTER(ctypes.c_uint8)
_P = ctypes.POINTER(OrcParams)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        L.orc_philox4x32_10.argtypes = [_U32, _U32, _U32]
        L.orc_bf16_round.argtypes = [ctypes.c_double]
        L.orc_bf16_round.restype = ctypes.c_double
        L.orc_reset_lattice.argtypes = [_P, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32,
                                        _I64, _I64, _I64, _I64, _U32]
        L.orc_reset_env.argtypes = [_P, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32,
                                    _D, _D, _D, _D, _D]
        L.orc_random_action.argtypes = [_P, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32]
        L.orc_random_action.restype = ctypes.c_int32
        L.orc_bounds.argtypes = [_P, ctypes.c_int32, _D, _D, _D, _D, _D, _D]
        L.orc_barrier_certificate.argtypes = [_P, ctypes.c_int32, _D, _D, _D, _D, _D, _D,
                                              _D, _D, _D]
        L.orc_barrier_certificate.restype = ctypes.c_int32
        L.orc_max_violation.argtypes = [_P, ctypes.c_int32, _D, _D, _D, _D]
        L.orc_max_violation.restype = ctypes.c_double
        L.orc_si_to_uni.argtypes = [_P, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                    _D, _D]
        L.orc_unicycle_position.argtypes = [_P] + [ctypes.c_double] * 5 + [_D, _D]
        L.orc_unicycle_pose.argtypes = [_P] + [ctypes.c_double] * 6 + [_D, _D]
        L.orc_uni_to_si.argtypes = [_P, ctypes.c_double, ctypes.c_double, ctypes.c_double, _D,
                                    _D]
        L.orc_action_noise.argtypes = [_P, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32, _D,
                                       _D]
        L.orc_nominal_command.argtypes = [_P, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int64,
                                          _D, _D, _D, _D, _D, _U8, _U8, _D, _D]
        L.orc_prey_move.argtypes = [_P, ctypes.c_int32, _D, _D, ctypes.c_double,
                                    ctypes.c_double, _D, _D, _D]
        L.orc_prey_move.restype = ctypes.c_int32
        L.orc_tagged.argtypes = [_P, ctypes.c_int32, _D, _D, ctypes.c_double, ctypes.c_double]
        L.orc_tagged.restype = ctypes.c_int32
        L.orc_observe.argtypes = [ctypes.c_int32, _D, _D, _D, _D, _D, _D]
        L.orc_env_step.argtypes = [_P, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int64,
                                   _D, _D, _D, _D, _D, _I32, _I32, _U8, _U8, _D, _D, _U8,
                                   _U8, _D]
        L.orc_env_step.restype = ctypes.c_int32
        L.orc_policy_logits.argtypes = [ctypes.c_int32, _D, _D, _D, _D, _D, _D, _D, _D]
        L.orc_sample_action.argtypes = [_D, ctypes.c_uint32]
        L.orc_sample_action.restype = ctypes.c_int32
        L.orc_policy_bits.argtypes = [_P, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32]
        L.orc_policy_bits.restype = ctypes.c_uint32
        L.orc_env_step_batch.argtypes = [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                         ctypes.c_int64, _D, _D, _D, _D, _D, _I32, _I32, _U8,
                                         _D, _D, _U8, _U8, ctypes.c_int32]
        L.orc_env_step_batch.restype = ctypes.c_int32
        L.orc_rollout.argtypes = [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                  ctypes.c_int64, _D, _D, _D, _D, _D, _D, ctypes.c_int32,
                                  _D, _D, _D, _D, _D, _I32, _I32, _D, _U8, _D, _U8,
                                  ctypes.c_int32]
        L.orc_rollout.restype = ctypes.c_int32
        _lib = L
    return _lib


def _ptr(a, typ):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(typ)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------------------
# Thin wrappers (numpy in, numpy out)
# ---------------------------------------------------------------------------

def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_ptr(c, _U32), _ptr(k, _U32), _ptr(out, _U32))
    return out


def bf16_round(x: float) -> float:
    return lib().orc_bf16_round(float(x))


def reset_lattice(p: Params, env_id: int, episode: int, n: int):
    X, Y, GX, GY = (np.zeros(n, np.int64) for _ in range(4))
    hb = np.zeros(n, np.uint32)
    cp = p.c()
    lib().orc_reset_lattice(ctypes.byref(cp), env_id, episode, n, _ptr(X, _I64), _ptr(Y, _I64),
                            _ptr(GX, _I64), _ptr(GY, _I64), _ptr(hb, _U32))
    return X, Y, GX, GY, hb


def reset_env(p: Params, env_id: int, episode: int, n: int):
    arrs = [np.zeros(n) for _ in range(5)]
    cp = p.c()
    lib().orc_reset_env(ctypes.byref(cp), env_id, episode, n, *[_ptr(a, _D) for a in arrs])
    return arrs  # x, y, th, gx, gy


def random_action(p: Params, env_id: int, t_global: int, i: int) -> int:
    cp = p.c()
    return lib().orc_random_action(ctypes.byref(cp), env_id, t_global, i)


def bounds(p: Params, px, py):
    px, py = _f64(px), _f64(py)
    n = px.size
    out = [np.zeros(n) for _ in range(4)]
    cp = p.c()
    lib().orc_bounds(ctypes.byref(cp), n, _ptr(px, _D), _ptr(py, _D), *[_ptr(a, _D) for a in out])
    return out  # lo_x, hi_x, lo_y, hi_y


def barrier_certificate(p: Params, px, py, ux_nom, uy_nom):
    """Returns (ux, uy, lambda_pairs, status, kkt[4], max_violation)."""
    px, py, uxn, uyn = _f64(px), _f64(py), _f64(ux_nom), _f64(uy_nom)
    n = px.size
    ux, uy = np.zeros(n), np.zeros(n)
    lam = np.zeros(max(n * (n - 1) // 2, 1))
    kkt = np.zeros(4)
    mv = ctypes.c_double(0.0)
    cp = p.c()
    st = lib().orc_barrier_certificate(ctypes.byref(cp), n, _ptr(px, _D), _ptr(py, _D),
                                       _ptr(uxn, _D), _ptr(uyn, _D), _ptr(ux, _D), _ptr(uy, _D),
                                       _ptr(lam, _D), _ptr(kkt, _D), ctypes.byref(mv))
    return ux, uy, lam[: n * (n - 1) // 2], st, kkt, mv.value


def max_violation(p: Params, px, py, ux, uy) -> float:
    px, py, ux, uy = _f64(px), _f64(py), _f64(ux), _f64(uy)
    cp = p.c()
    return lib().orc_max_violation(ctypes.byref(cp), px.size, _ptr(px, _D), _ptr(py, _D),
                                   _ptr(ux, _D), _ptr(uy, _D))


def si_to_uni(p: Params, theta: float, ux: float, uy: float):
    v, w = ctypes.c_double(), ctypes.c_double()
    cp = p.c()
    lib().orc_si_to_uni(ctypes.byref(cp), theta, ux, uy, ctypes.byref(v), ctypes.byref(w))
    return v.value, w.value


def unicycle_position(p: Params, x: float, y: float, theta: float, wx: float, wy: float):
    v, w = ctypes.c_double(), ctypes.c_double()
    cp = p.c()
    lib().orc_unicycle_position(ctypes.byref(cp), x, y, theta, wx, wy, ctypes.byref(v),
                                ctypes.byref(w))
    return v.value, w.value


def unicycle_pose(p: Params, x: float, y: float, theta: float, wx: float, wy: float,
                  wth: float):
    v, w = ctypes.c_double(), ctypes.c_double()
    cp = p.c()
    lib().orc_unicycle_pose(ctypes.byref(cp), x, y, theta, wx, wy, wth, ctypes.byref(v),
                            ctypes.byref(w))
    return v.value, w.value


def uni_to_si(p: Params, theta: float, v: float, w: float):
    ux, uy = ctypes.c_double(), ctypes.c_double()
    cp = p.c()
    lib().orc_uni_to_si(ctypes.byref(cp), theta, v, w, ctypes.byref(ux), ctypes.byref(uy))
    return ux.value, uy.value


def action_noise(p: Params, env_id: int, t_global: int, i: int):
    nx, ny = ctypes.c_double(), ctypes.c_double()
    cp = p.c()
    lib().orc_action_noise(ctypes.byref(cp), env_id, t_global, i, ctypes.byref(nx),
                           ctypes.byref(ny))
    return nx.value, ny.value


def nominal_command(p: Params, state: dict, env_id: int, t_global: int, actions=None):
    """Nominal command (before the magnitude pre-clip) of every robot of one
    env; returns (unx, uny, actions used)."""
    n = state["x"].size
    act = None if actions is None else np.ascontiguousarray(actions, dtype=np.uint8)
    used = np.zeros(n, np.uint8)
    unx, uny = np.zeros(n), np.zeros(n)
    cp = p.c()
    lib().orc_nominal_command(ctypes.byref(cp), n, env_id, t_global,
                              *[_ptr(_f64(state[k]), _D) for k in ("x", "y", "th", "gx", "gy")],
                              _ptr(act, _U8), _ptr(used, _U8), _ptr(unx, _D), _ptr(uny, _D))
    return unx, uny, (used if act is None else act)


def prey_move(p: Params, x, y, qx: float, qy: float):
    """Predator-Prey prey move: returns (new qx, new qy, chosen index, scores[17])."""
    x, y = _f64(x), _f64(y)
    nqx, nqy = ctypes.c_double(), ctypes.c_double()
    scores = np.zeros(17)
    cp = p.c()
    k = lib().orc_prey_move(ctypes.byref(cp), x.size, _ptr(x, _D), _ptr(y, _D), qx, qy,
                            ctypes.byref(nqx), ctypes.byref(nqy), _ptr(scores, _D))
    return nqx.value, nqy.value, k, scores


def tagged(p: Params, x, y, qx: float, qy: float) -> bool:
    x, y = _f64(x), _f64(y)
    cp = p.c()
    return bool(lib().orc_tagged(ctypes.byref(cp), x.size, _ptr(x, _D), _ptr(y, _D), qx, qy))


def observe(x, y, th, gx, gy):
    x, y, th, gx, gy = (_f64(a) for a in (x, y, th, gx, gy))
    n = x.size
    obs = np.zeros((n, 2 * n + 4))
    lib().orc_observe(n, *[_ptr(a, _D) for a in (x, y, th, gx, gy)], _ptr(obs, _D))
    return obs


def env_step(p: Params, state: dict, env_id: int, t_global: int, actions=None):
    """One step of one env. ``state`` holds x,y,th,gx,gy (float64 [n]) and
    step, episode (ints); it is updated in place. Returns a dict of outputs."""
    n = state["x"].size
    step = ctypes.c_int32(int(state["step"]))
    ep = ctypes.c_int32(int(state["episode"]))
    act = None if actions is None else np.ascontiguousarray(actions, dtype=np.uint8)
    used = np.zeros(n, np.uint8)
    obs = np.zeros((n, 2 * n + 4))
    rew = ctypes.c_double()
    done, infe = ctypes.c_uint8(), ctypes.c_uint8()
    mv = ctypes.c_double()
    cp = p.c()
    st = lib().orc_env_step(ctypes.byref(cp), n, env_id, t_global,
                            *[_ptr(state[k], _D) for k in ("x", "y", "th", "gx", "gy")],
                            ctypes.byref(step), ctypes.byref(ep), _ptr(act, _U8), _ptr(used, _U8),
                            _ptr(obs, _D), ctypes.byref(rew), ctypes.byref(done),
                            ctypes.byref(infe), ctypes.byref(mv))
    state["step"] = step.value
    state["episode"] = ep.value
    return {"status": st, "actions": used if act is None else act, "obs": obs,
            "reward": rew.value, "done": done.value, "infeasible": infe.value,
            "max_violation": mv.value}


def policy_logits(weights: dict, obs_row):
    """weights: w1 [in,64], b1 [64], w2 [64,64], b2, w3 [64,5], b3 (bf16-valued float64)."""
    o = _f64(obs_row)
    w = {k: _f64(v) for k, v in weights.items()}
    logits = np.zeros(5)
    lib().orc_policy_logits(o.size, _ptr(w["w1"], _D), _ptr(w["b1"], _D), _ptr(w["w2"], _D),
                            _ptr(w["b2"], _D), _ptr(w["w3"], _D), _ptr(w["b3"], _D), _ptr(o, _D),
                            _ptr(logits, _D))
    return logits


def sample_action(logits, r: int) -> int:
    lg = _f64(logits)
    return lib().orc_sample_action(_ptr(lg, _D), int(r))


def policy_bits(p: Params, env_id: int, t_global: int, i: int) -> int:
    cp = p.c()
    return lib().orc_policy_bits(ctypes.byref(cp), env_id, t_global, i)


def env_step_batch(p: Params, n: int, st: dict, env_id_base: int, t_global: int, actions=None,
                   want_obs=True, nthreads=1):
    """Batched step; st holds x,y,th,gx,gy float64 [E*n], step, episode int32 [E]."""
    E = st["step"].size
    obs = np.zeros((E, n, 2 * n + 4)) if want_obs else None
    rew = np.zeros(E)
    done = np.zeros(E, np.uint8)
    infe = np.zeros(E, np.uint8)
    act = None if actions is None else np.ascontiguousarray(actions, dtype=np.uint8)
    cp = p.c()
    status = lib().orc_env_step_batch(ctypes.byref(cp), n, E, env_id_base, t_global,
                                      *[_ptr(st[k], _D) for k in ("x", "y", "th", "gx", "gy")],
                                      _ptr(st["step"], _I32), _ptr(st["episode"], _I32),
                                      _ptr(act, _U8), _ptr(obs, _D), _ptr(rew, _D),
                                      _ptr(done, _U8), _ptr(infe, _U8), nthreads)
    return {"status": status, "obs": obs, "reward": rew, "done": done, "infeasible": infe}


def rollout(p: Params, n: int, st: dict, env_id_base: int, t_global0: int, weights: dict,
            horizon: int, want_obs=True, nthreads=1):
    E = st["step"].size
    dim = 2 * n + 4
    obs = np.zeros((horizon, E, n, dim)) if want_obs else None
    act = np.zeros((horizon, E, n), np.uint8)
    rew = np.zeros((horizon, E))
    done = np.zeros((horizon, E), np.uint8)
    w = {k: _f64(v) for k, v in weights.items()}
    cp = p.c()
    status = lib().orc_rollout(ctypes.byref(cp), n, E, env_id_base, t_global0,
                               *[_ptr(w[k], _D) for k in ("w1", "b1", "w2", "b2", "w3", "b3")],
                               horizon, *[_ptr(st[k], _D) for k in ("x", "y", "th", "gx", "gy")],
                               _ptr(st["step"], _I32), _ptr(st["episode"], _I32), _ptr(obs, _D),
                               _ptr(act, _U8), _ptr(rew, _D), _ptr(done, _U8), nthreads)
    return {"status": status, "obs": obs, "actions": act, "reward": rew, "done": done}


__all__ = [n for n in dir() if not n.startswith("_")]
