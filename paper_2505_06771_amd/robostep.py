"""Python binding of librobostep.so (ctypes; argument marshalling only).

Every step of the simulation runs in the HIP kernels behind the C ABI declared
in include/robostep.h; this module only turns torch tensors (device memory) and
torch streams into pointers and raises on error. There is no CPU fallback: if
the library is not built, importing the binding's calls raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "librobostep.so")

RS_F32, RS_F64 = 0, 1
RS_CTRL_DISCRETE, RS_CTRL_GOTO, RS_CTRL_WAYPOINT, RS_CTRL_POSE = 0, 1, 2, 3
RS_SCN_NAVIGATION, RS_SCN_PREDATOR_PREY = 0, 1
# certificate statistics (qp_stats slots)
QPS_BOX, QPS_ONE_ROW, QPS_TWO_ROWS, QPS_SHARED_ROBOT, QPS_ACTIVE_SET, QPS_GENERAL = range(6)
QPS_INFEASIBLE, QPS_CAPPED, QPS_ITERATIONS, QPS_COUNT = 6, 7, 8, 9
STATUS = {0: "ok", 1: "invalid argument", 2: "unsupported", 3: "out of memory",
          4: "device error", 5: "over budget", 6: "not found"}


class RobostepError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class RsParams(ctypes.Structure):
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
        ("dtype", ctypes.c_int32), ("qp_max_iters", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("waypoint_step", ctypes.c_double), ("pos_gain", ctypes.c_double),
        ("ang_gain", ctypes.c_double), ("action_noise", ctypes.c_double),
        ("prey_speed", ctypes.c_double), ("tag_radius", ctypes.c_double),
        ("tag_reward", ctypes.c_double), ("scenario", ctypes.c_int32),
        ("pose_gain_rho", ctypes.c_double), ("pose_gain_alpha", ctypes.c_double),
        ("pose_gain_beta", ctypes.c_double),
    ]


class RsBatch(ctypes.Structure):
    _fields_ = [
        ("num_envs", ctypes.c_int32), ("robots", ctypes.c_int32),
        ("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("theta", ctypes.c_void_p),
        ("goal_x", ctypes.c_void_p), ("goal_y", ctypes.c_void_p),
        ("step", ctypes.c_void_p), ("episode", ctypes.c_void_p),
        ("env_id_base", ctypes.c_uint64),
    ]


class RsPolicy(ctypes.Structure):
    _fields_ = [
        ("w1", ctypes.c_void_p), ("w2", ctypes.c_void_p), ("w3", ctypes.c_void_p),
        ("b1", ctypes.c_void_p), ("b2", ctypes.c_void_p), ("b3", ctypes.c_void_p),
        ("in_dim", ctypes.c_int32),
    ]


class RsSchedule(ctypes.Structure):
    _fields_ = [("block_threads", ctypes.c_int32), ("lanes_per_env", ctypes.c_int32 * 17),
                ("qp_iters", ctypes.c_int32 * 17), ("envs_per_wave", ctypes.c_int32 * 17)]


class RsRequestInfo(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("envs", ctypes.c_int32), ("robots", ctypes.c_int32),
                ("horizon", ctypes.c_int32), ("submit_time", ctypes.c_double),
                ("admit_time", ctypes.c_double), ("finish_time", ctypes.c_double)]


class RsServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("admitted", ctypes.c_int64),
                ("finished", ctypes.c_int64), ("ticks", ctypes.c_int64),
                ("robot_steps", ctypes.c_int64), ("bytes_in_use", ctypes.c_int64),
                ("peak_bytes", ctypes.c_int64), ("queued", ctypes.c_int32),
                ("running", ctypes.c_int32)]


_lib = None
_VP = ctypes.c_void_p


def use_library(path: str):
    """Load the library from `path` (e.g. the phase-timer build) instead of
    librobostep.so; only before the first call into the library."""
    global LIB_PATH
    if _lib is not None and os.path.abspath(path) != os.path.abspath(LIB_PATH):
        raise RuntimeError("the library is already loaded")
    LIB_PATH = path


def lib():
    """Load the HIP library; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_2505_06771_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    i32, i64, u64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "rs_params_default": (None, [P(RsParams)]),
        "rs_params_check": (i32, [P(RsParams)]),
        "rs_status_string": (ctypes.c_char_p, [i32]),
        "rs_last_error": (ctypes.c_char_p, []),
        "rs_create": (i32, [ctypes.c_int, P(_VP)]),
        "rs_destroy": (i32, [_VP]),
        "env_reset": (i32, [_VP, P(RsParams), P(RsBatch), _VP, _VP, _VP]),
        "rs_qp_failures": (i32, [_VP, P(i64), P(i64), i32]),
        "rs_phase_cycles": (i32, [_VP, _VP, i32]),
        "env_step": (i32, [_VP, P(RsParams), P(RsBatch), _VP, i64, _VP, _VP, _VP, _VP, _VP, _VP,
                           _VP]),
        "env_steps": (i32, [_VP, P(RsParams), P(RsBatch), i32, i64, _VP, _VP, _VP, _VP, _VP]),
        "barrier_certificate": (i32, [_VP, P(RsParams), i32, i32, _VP, _VP, _VP, _VP, _VP, _VP,
                                      _VP, _VP, _VP, _VP, _VP]),
        "rollout": (i32, [_VP, P(RsParams), P(RsBatch), P(RsPolicy), i32, i64, _VP, _VP, _VP,
                          _VP, _VP, _VP]),
        "rs_plan_create": (i32, [_VP, i32, _VP, P(RsSchedule), P(_VP)]),
        "rs_plan_destroy": (i32, [_VP]),
        "rs_plan_total_robots": (i64, [_VP]),
        "rs_plan_robot_offset": (_VP, [_VP]),
        "rs_plan_obs_offset": (i64, [_VP, i32]),
        "env_reset_mixed": (i32, [_VP, P(RsParams), _VP, P(RsBatch), _VP, _VP]),
        "env_run": (i32, [_VP, P(RsParams), _VP, P(RsBatch), i32, _VP, i64, _VP, _VP, _VP, _VP,
                          _VP, _VP, _VP]),
        "env_run_noalloc": (i32, [_VP, P(RsParams), _VP, P(RsBatch), i32, _VP, i64, _VP, _VP,
                                  _VP, _VP, _VP, _VP, _VP, _VP]),
        "rs_autotune": (i32, [_VP, P(RsParams), _VP, i32, i32, i32, dbl, P(RsSchedule)]),
        "rs_get_schedule": (i32, [_VP, P(RsSchedule)]),
        "rs_set_schedule": (i32, [_VP, P(RsSchedule)]),
        "rs_autotune_batch": (i32, [_VP, P(RsParams), _VP, P(RsBatch), i32, dbl, P(RsSchedule)]),
        "rs_server_create": (i32, [_VP, P(RsParams), i64, i32, P(_VP)]),
        "rs_server_destroy": (i32, [_VP]),
        "rs_request_bytes": (i64, [i32, i32]),
        "rs_server_submit": (i32, [_VP, i64, i32, i32, i32]),
        "rs_server_tick": (i32, [_VP, P(i32)]),
        "rs_server_poll": (i32, [_VP, P(RsRequestInfo), _VP, _VP]),
        "rs_server_stats_get": (i32, [_VP, P(RsServerStats)]),
        "rs_snapshot_bytes": (i64, [i32, i32, i64]),
        "rs_snapshot": (i32, [_VP, i32, P(RsBatch), i64, _VP, i64, _VP]),
        "rs_restore": (i32, [_VP, i32, P(RsBatch), i64, _VP, i64, _VP]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name, None)
        if fn is None:
            continue
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(status):
    if status != 0:
        raise RobostepError(status, lib().rs_last_error().decode())


def _ptr(t) -> Optional[int]:
    """Device pointer of a tensor (None -> NULL)."""
    if t is None:
        return None
    assert t.is_contiguous(), "tensors passed to robostep must be contiguous"
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch

        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def params(**kw) -> RsParams:
    """Default simulation constants (see rs_params_default), overridden by kw."""
    p = RsParams()
    lib().rs_params_default(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


class Context:
    def __init__(self, device: int = 0):
        self.handle = _VP()
        _check(lib().rs_create(device, ctypes.byref(self.handle)))

    def phase_cycles(self, waves: int):
        """[waves, 8] phase cycles of the last rollout launch (diagnostic
        library only, see build.py --phase-timers)."""
        import numpy as np

        out = np.zeros((waves, 8), np.int64)
        _check(lib().rs_phase_cycles(self.handle, out.ctypes.data, waves))
        return out

    def qp_failures(self, reset: bool = False):
        """(infeasible, capped) certificate solves counted on the device by
        every call on this context (waits for the device)."""
        inf, cap = ctypes.c_int64(0), ctypes.c_int64(0)
        _check(lib().rs_qp_failures(self.handle, ctypes.byref(inf), ctypes.byref(cap),
                                    1 if reset else 0))
        return int(inf.value), int(cap.value)

    def close(self):
        if self.handle:
            lib().rs_destroy(self.handle)
            self.handle = _VP()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Batch:
    """Device SoA state of E environments (tensors on the GPU)."""
    x: object
    y: object
    theta: object
    goal_x: object
    goal_y: object
    step: object
    episode: object
    robots: int
    env_id_base: int = 0

    @property
    def num_envs(self) -> int:
        return int(self.step.numel())

    def c(self) -> RsBatch:
        return RsBatch(self.num_envs, self.robots, _ptr(self.x), _ptr(self.y), _ptr(self.theta),
                       _ptr(self.goal_x), _ptr(self.goal_y), _ptr(self.step), _ptr(self.episode),
                       self.env_id_base)

    @staticmethod
    def empty(num_envs: int, robots: int, dtype=None, device="cuda", env_id_base=0,
              total_robots: Optional[int] = None):
        import torch

        dtype = dtype or torch.float32
        n = total_robots if total_robots is not None else num_envs * robots
        f = lambda: torch.zeros(n, dtype=dtype, device=device)
        i = lambda: torch.zeros(num_envs, dtype=torch.int32, device=device)
        return Batch(f(), f(), f(), f(), f(), i(), i(), robots, env_id_base)


def env_reset(ctx: Context, p: RsParams, b: Batch, mask=None, obs=None, stream=None):
    cb = b.c()
    _check(lib().env_reset(ctx.handle, ctypes.byref(p), ctypes.byref(cb), _ptr(mask), _ptr(obs),
                           _stream(stream)))


def env_step(ctx: Context, p: RsParams, b: Batch, actions=None, t_global: int = 0, obs=None,
             reward=None, done=None, max_violation=None, infeasible=None, qp_stats=None,
             stream=None):
    cb = b.c()
    _check(lib().env_step(ctx.handle, ctypes.byref(p), ctypes.byref(cb), _ptr(actions), t_global,
                          _ptr(obs), _ptr(reward), _ptr(done), _ptr(max_violation),
                          _ptr(infeasible), _ptr(qp_stats), _stream(stream)))


def env_steps(ctx: Context, p: RsParams, b: Batch, steps: int, t_global0: int = 0, reward=None,
              done=None, obs_final=None, qp_stats=None, stream=None):
    """`steps` env_step calls (actions drawn) in one launch; reward/done [steps][E]."""
    cb = b.c()
    _check(lib().env_steps(ctx.handle, ctypes.byref(p), ctypes.byref(cb), steps, t_global0,
                           _ptr(reward), _ptr(done), _ptr(obs_final), _ptr(qp_stats),
                           _stream(stream)))


def barrier_certificate(ctx: Context, p: RsParams, num_envs: int, robots: int, px, py, ux_nom,
                        uy_nom, ux, uy, lam=None, max_violation=None, infeasible=None,
                        qp_stats=None, stream=None):
    _check(lib().barrier_certificate(ctx.handle, ctypes.byref(p), num_envs, robots, _ptr(px),
                                     _ptr(py), _ptr(ux_nom), _ptr(uy_nom), _ptr(ux), _ptr(uy),
                                     _ptr(lam), _ptr(max_violation), _ptr(infeasible),
                                     _ptr(qp_stats), _stream(stream)))


@dataclass
class Policy:
    """bf16 weights (torch.bfloat16 [in][out]) and float32 biases on the GPU."""
    w1: object
    b1: object
    w2: object
    b2: object
    w3: object
    b3: object

    def c(self) -> RsPolicy:
        return RsPolicy(_ptr(self.w1), _ptr(self.w2), _ptr(self.w3), _ptr(self.b1), _ptr(self.b2),
                        _ptr(self.b3), int(self.w1.shape[0]))


def rollout(ctx: Context, p: RsParams, b: Batch, policy: Policy, horizon: int, t_global0: int,
            obs, actions, reward, done, qp_stats=None, stream=None):
    cb = b.c()
    cp = policy.c()
    _check(lib().rollout(ctx.handle, ctypes.byref(p), ctypes.byref(cb), ctypes.byref(cp), horizon,
                         t_global0, _ptr(obs), _ptr(actions), _ptr(reward), _ptr(done),
                         _ptr(qp_stats), _stream(stream)))


class Plan:
    """Schedule of a mixed-size batch (robots per env on the host)."""

    def __init__(self, ctx: Context, robots_per_env, schedule: Optional[RsSchedule] = None):
        import numpy as np

        arr = np.ascontiguousarray(robots_per_env, dtype=np.int32)
        self.robots_per_env = arr
        self.handle = _VP()
        _check(lib().rs_plan_create(ctx.handle, arr.size, arr.ctypes.data,
                                    ctypes.byref(schedule) if schedule is not None else None,
                                    ctypes.byref(self.handle)))
        self.num_envs = int(arr.size)
        self.total_robots = int(lib().rs_plan_total_robots(self.handle))

    def obs_offset(self, env: int) -> int:
        return int(lib().rs_plan_obs_offset(self.handle, env))

    def close(self):
        if self.handle:
            lib().rs_plan_destroy(self.handle)
            self.handle = _VP()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _batch_dtype(b: Batch) -> int:
    import torch

    return RS_F64 if b.x.dtype == torch.float64 else RS_F32


def snapshot(ctx: Context, b: Batch, stream=None):
    """Host copy of the batch's state (pose, goal, step, episode) as a numpy
    uint8 buffer in the rs_snapshot layout."""
    import numpy as np

    dtype = _batch_dtype(b)
    robots_total = int(b.x.numel())
    n = lib().rs_snapshot_bytes(dtype, b.num_envs, robots_total)
    buf = np.zeros(n, np.uint8)
    cb = b.c()
    _check(lib().rs_snapshot(ctx.handle, dtype, ctypes.byref(cb), robots_total,
                             buf.ctypes.data, n, _stream(stream)))
    return buf


def restore(ctx: Context, b: Batch, buf, stream=None):
    """Write a snapshot buffer back into the batch (same shape and precision)."""
    import numpy as np

    buf = np.ascontiguousarray(buf, dtype=np.uint8)
    cb = b.c()
    _check(lib().rs_restore(ctx.handle, _batch_dtype(b), ctypes.byref(cb), int(b.x.numel()),
                            buf.ctypes.data, buf.size, _stream(stream)))


def env_reset_mixed(ctx: Context, p: RsParams, plan: Plan, b: Batch, mask=None, stream=None):
    cb = b.c()
    _check(lib().env_reset_mixed(ctx.handle, ctypes.byref(p), plan.handle, ctypes.byref(cb),
                                 _ptr(mask), _stream(stream)))


def env_run(ctx: Context, p: RsParams, plan: Plan, b: Batch, steps: int, t_global0: int = 0,
            t_start=None, steps_per_env=None, reward_out=None, done_out=None, reward_sum=None,
            obs_final=None, qp_stats=None, stream=None):
    cb = b.c()
    _check(lib().env_run(ctx.handle, ctypes.byref(p), plan.handle, ctypes.byref(cb), steps,
                         _ptr(t_start), t_global0, _ptr(steps_per_env), _ptr(reward_out),
                         _ptr(done_out), _ptr(reward_sum), _ptr(obs_final), _ptr(qp_stats),
                         _stream(stream)))


def env_run_noalloc(ctx: Context, p: RsParams, robots_per_env, b: Batch, steps: int,
                    t_global0: int = 0, t_start=None, steps_per_env=None, reward_out=None,
                    done_out=None, reward_sum=None, obs_final=None, qp_stats=None, bad_envs=None,
                    stream=None):
    """env_run without a plan: robots_per_env is a device int32 tensor [E];
    bad_envs (device int32 [1], optional) receives the number of envs whose
    count is outside 2..16 (then nothing runs). Allocates nothing."""
    cb = b.c()
    _check(lib().env_run_noalloc(ctx.handle, ctypes.byref(p), _ptr(robots_per_env),
                                 ctypes.byref(cb), steps, _ptr(t_start), t_global0,
                                 _ptr(steps_per_env), _ptr(reward_out), _ptr(done_out),
                                 _ptr(reward_sum), _ptr(obs_final), _ptr(qp_stats),
                                 _ptr(bad_envs), _stream(stream)))


NOALLOC_MAX_ENVS = 65536


def autotune(ctx: Context, p: RsParams, robots, envs: int = 4096, steps: int = 50,
             tol: float = 1e-4) -> RsSchedule:
    import numpy as np

    arr = np.ascontiguousarray(robots, dtype=np.int32)
    out = RsSchedule()
    _check(lib().rs_autotune(ctx.handle, ctypes.byref(p), arr.ctypes.data, arr.size, envs, steps,
                             tol, ctypes.byref(out)))
    return out


def set_schedule(ctx: Context, schedule: RsSchedule):
    """Set the context's schedule (plans made afterwards, env_run_noalloc, server)."""
    _check(lib().rs_set_schedule(ctx.handle, ctypes.byref(schedule)))


def get_schedule(ctx: Context) -> RsSchedule:
    out = RsSchedule()
    _check(lib().rs_get_schedule(ctx.handle, ctypes.byref(out)))
    return out


def autotune_batch(ctx: Context, p: RsParams, plan: Plan, b: Batch, steps: int = 50,
                   tol: float = 1e-4) -> RsSchedule:
    """Autotune on the caller's own mixed batch (its state is left unchanged)."""
    out = RsSchedule()
    cb = b.c()
    _check(lib().rs_autotune_batch(ctx.handle, ctypes.byref(p), plan.handle, ctypes.byref(cb),
                                   steps, tol, ctypes.byref(out)))
    return out


class Server:
    """Continuous-batching rollout server (see rs_server_* in robostep.h)."""

    def __init__(self, ctx: Context, p: RsParams, hbm_budget_bytes: int, tick_steps: int):
        self.handle = _VP()
        self._p = p
        _check(lib().rs_server_create(ctx.handle, ctypes.byref(p), int(hbm_budget_bytes),
                                      tick_steps, ctypes.byref(self.handle)))

    @staticmethod
    def request_bytes(envs: int, robots: int) -> int:
        return int(lib().rs_request_bytes(envs, robots))

    def submit(self, rid: int, envs: int, robots: int, horizon: int):
        _check(lib().rs_server_submit(self.handle, rid, envs, robots, horizon))

    def tick(self) -> bool:
        busy = ctypes.c_int32(0)
        _check(lib().rs_server_tick(self.handle, ctypes.byref(busy)))
        return bool(busy.value)

    def poll(self, with_results=True):
        import numpy as np

        info = RsRequestInfo()
        # a first call without buffers tells us the sizes; results need them
        st = lib().rs_server_poll(self.handle, ctypes.byref(info), None, None)
        if st == 6:
            return None
        _check(st)
        return info

    def poll_results(self, max_envs: int, max_robots: int):
        """Pop one finished request with its results (numpy arrays)."""
        import numpy as np

        info = RsRequestInfo()
        xy = np.zeros(max_envs * max_robots * 2, np.float32)
        rs_ = np.zeros(max_envs, np.float32)
        st = lib().rs_server_poll(self.handle, ctypes.byref(info), xy.ctypes.data, rs_.ctypes.data)
        if st == 6:
            return None
        _check(st)
        n = info.envs * info.robots
        return info, xy[: 2 * n].reshape(info.envs, info.robots, 2), rs_[: info.envs]

    def stats(self) -> RsServerStats:
        s = RsServerStats()
        _check(lib().rs_server_stats_get(self.handle, ctypes.byref(s)))
        return s

    def close(self):
        if self.handle:
            lib().rs_server_destroy(self.handle)
            self.handle = _VP()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
