"""CPU checks of the C ABI: the HIP library loads, exports every function that
include/robostep.h declares, and its host-only calls behave (defaults, status
strings, request sizing, argument validation before any device work)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "robostep.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s+\**([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "return")))


@pytest.fixture(scope="module")
def R():
    from paper_2505_06771_amd import robostep

    if not os.path.exists(robostep.LIB_PATH):
        from paper_2505_06771_amd import build

        build.build()
    robostep.lib()
    return robostep


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("env_reset", "env_step", "barrier_certificate", "rollout", "env_run",
              "rs_create", "rs_server_submit", "rs_autotune"):
        assert n in names
    assert len(names) >= 25


def test_every_declared_symbol_is_exported(R):
    L = R.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, f"not exported: {missing}"


def test_params_default_match_the_configuration(R):
    p = R.params()
    assert (p.x_min, p.x_max, p.y_min, p.y_max) == (-1.6, 1.6, -1.0, 1.0)
    assert p.dt == 0.033 and p.proj_dist == 0.05 and p.barrier_gain == 100.0
    assert p.safety_radius == 0.17 and p.v_max == 0.2 and p.max_steps == 500
    assert p.goal_radius == 0.05 and p.dtype == R.RS_F32


def test_params_struct_matches_oracle_constants(R):
    import oracle

    o = oracle.Params()
    p = R.params()
    for f in ("x_min", "x_max", "dt", "proj_dist", "barrier_gain", "safety_radius",
              "boundary_gain_factor", "v_max", "action_speed", "kp", "wheel_radius",
              "base_length", "goal_radius", "reset_margin", "min_sep", "grid", "max_steps",
              "waypoint_step", "pos_gain", "ang_gain", "action_noise", "prey_speed",
              "tag_radius", "tag_reward", "scenario", "pose_gain_rho", "pose_gain_alpha",
              "pose_gain_beta"):
        assert getattr(o, f) == getattr(p, f), f


def test_struct_layouts_match_the_header(R, tmp_path):
    """ctypes mirrors of the ABI structs have the C sizes and field offsets."""
    import subprocess

    src = tmp_path / "sizes.c"
    fields = {"rs_params": ["seed", "qp_max_iters", "grid", "waypoint_step", "action_noise",
                            "tag_reward", "scenario", "pose_gain_rho", "pose_gain_beta"],
              "rs_batch": ["env_id_base", "episode"],
              "rs_policy": ["in_dim", "b3"],
              "rs_schedule": ["qp_iters", "lanes_per_env", "envs_per_wave"],
              "rs_request_info": ["finish_time", "horizon"],
              "rs_server_stats": ["running", "peak_bytes"]}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "robostep.h"', "int main(void){"]
    for st, fs in fields.items():
        lines.append(f'printf("{st} %zu\\n", sizeof({st}));')
        for f in fs:
            lines.append(f'printf("{st}.{f} %zu\\n", offsetof({st}, {f}));')
    lines.append("return 0;}")
    src.write_text("\n".join(lines))
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                  check=True).stdout.splitlines())
    mirror = {"rs_params": R.RsParams, "rs_batch": R.RsBatch, "rs_policy": R.RsPolicy,
              "rs_schedule": R.RsSchedule, "rs_request_info": R.RsRequestInfo,
              "rs_server_stats": R.RsServerStats}
    for st, cls in mirror.items():
        assert ctypes.sizeof(cls) == int(out[st]), st
        for f in fields[st]:
            assert getattr(cls, f).offset == int(out[f"{st}.{f}"]), f"{st}.{f}"


def test_status_strings(R):
    L = R.lib()
    assert L.rs_status_string(0) == b"ok"
    assert L.rs_status_string(5) == b"over budget"


def test_request_bytes(R):
    L = R.lib()
    assert L.rs_request_bytes(0, 4) == 0
    b = L.rs_request_bytes(100, 8)
    assert b >= 100 * 8 * 20 and b % 256 == 0


def test_null_arguments_are_rejected_without_device_work(R):
    L = R.lib()
    p = R.params()
    st = L.env_step(None, ctypes.byref(p), None, None, 0, None, None, None, None, None, None,
                    None)
    assert st == 1
    assert b"NULL" in L.rs_last_error()
    st = L.barrier_certificate(None, ctypes.byref(p), 4, 4, None, None, None, None, None, None,
                               None, None, None, None, None)
    assert st == 1
    out = ctypes.c_void_p()
    st = L.rs_plan_create(None, 4, None, None, ctypes.byref(out))
    assert st == 1


def test_gpu_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2505_06771_amd import robostep

    monkeypatch.setattr(robostep, "_lib", None)
    monkeypatch.setattr(robostep, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="missing"):
        robostep.lib()


def test_snapshot_size_and_argument_checks(R):
    """Snapshot layout size, and restore refuses a buffer whose header does not
    match the batch before any device copy."""
    import numpy as np

    L = R.lib()
    assert L.rs_snapshot_bytes(R.RS_F32, 10, 40) == 32 + 5 * 40 * 4 + 2 * 10 * 4
    assert L.rs_snapshot_bytes(R.RS_F64, 10, 40) == 32 + 5 * 40 * 8 + 2 * 10 * 4
    fake = ctypes.c_void_p(0x1000)
    b = R.RsBatch(10, 4, 0x1000, 0x1000, 0x1000, 0x1000, 0x1000, 0x1000, 0x1000, 0)
    n = L.rs_snapshot_bytes(R.RS_F32, 10, 40)
    buf = np.zeros(n, np.uint8)
    # not a snapshot: wrong magic
    assert L.rs_restore(fake, R.RS_F32, ctypes.byref(b), 40, buf.ctypes.data, n, None) == 1
    assert b"not a snapshot" in L.rs_last_error()
    # right magic, wrong shape
    buf[:8] = np.frombuffer(b"RSSNAP1\0", np.uint8)
    buf[8:12] = np.frombuffer(np.int32(0).tobytes(), np.uint8)
    buf[12:16] = np.frombuffer(np.int32(11).tobytes(), np.uint8)
    buf[16:24] = np.frombuffer(np.int64(40).tobytes(), np.uint8)
    assert L.rs_restore(fake, R.RS_F32, ctypes.byref(b), 40, buf.ctypes.data, n, None) == 1
    assert b"does not match" in L.rs_last_error()
    # buffer too small
    assert L.rs_snapshot(fake, R.RS_F32, ctypes.byref(b), 40, buf.ctypes.data, n - 1, None) == 1
    assert L.rs_snapshot(None, R.RS_F32, ctypes.byref(b), 40, buf.ctypes.data, n, None) == 1


def test_params_check_covers_controllers_and_noise(R):
    """Parameter validation runs on the host, before any device work."""
    L = R.lib()
    ok = lambda **kw: L.rs_params_check(ctypes.byref(R.params(**kw)))
    assert ok() == 0
    assert ok(controller=R.RS_CTRL_WAYPOINT, action_noise=0.05) == 0
    assert ok(controller=R.RS_CTRL_GOTO) == 0
    assert ok(controller=R.RS_CTRL_POSE) == 0
    assert ok(controller=4) == 1 and b"controller" in L.rs_last_error()
    assert ok(controller=R.RS_CTRL_POSE, waypoint_step=0.0) == 1
    assert ok(controller=R.RS_CTRL_POSE, pose_gain_alpha=-1.0) == 1
    assert ok(controller=R.RS_CTRL_WAYPOINT, waypoint_step=0.0) == 1
    assert b"waypoint_step" in L.rs_last_error()
    assert ok(action_noise=-0.1) == 1 and b"action_noise" in L.rs_last_error()
    assert ok(scenario=R.RS_SCN_PREDATOR_PREY) == 0
    assert ok(scenario=2) == 1 and b"scenario" in L.rs_last_error()
    assert ok(scenario=R.RS_SCN_PREDATOR_PREY, prey_speed=-0.1) == 1
    assert ok(pos_gain=-1.0) == 1
    assert ok(dt=0.0) == 1
    assert ok() == 0 and L.rs_last_error() == b""


def test_binding_argument_counts_match_the_header(R):
    """Every function the ctypes binding declares takes as many arguments as
    its prototype in include/robostep.h (a missing argument would shift every
    later pointer)."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    protos = {}
    for m in re.finditer(r"([A-Za-z_][A-Za-z0-9_]*)\s*\(([^;{]*?)\)\s*;", text, flags=re.S):
        args = m.group(2).strip()
        protos[m.group(1)] = 0 if args in ("", "void") else args.count(",") + 1
    L = R.lib()
    checked = 0
    for name, n in protos.items():
        fn = getattr(L, name, None)
        if fn is None or fn.argtypes is None:
            continue
        assert len(fn.argtypes) == n, f"{name}: binding {len(fn.argtypes)} args, header {n}"
        checked += 1
    assert checked >= 25


def test_set_schedule_validates_on_the_host(R):
    """rs_set_schedule refuses malformed schedules before touching the
    context (no device work: a NULL context is refused first)."""
    L = R.lib()
    s = R.RsSchedule()
    assert L.rs_set_schedule(None, ctypes.byref(s)) == 1
    assert b"NULL" in L.rs_last_error()
