"""ctypes front end of the FP64 CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It builds ``liboracle.so`` from ``oracle.c`` with gcc
(``-O2 -ffp-contract=off -fopenmp``) and exposes the plain-definition MV/FFC,
forward kinematics and clearance functions documented in that file.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so (always when force, else only when missing or stale)."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


class _Team(C.Structure):
    _fields_ = [("n_robots", C.c_int32),
                ("n_joints", C.c_void_p), ("joint_off", C.c_void_p), ("joint_type", C.c_void_p),
                ("joint_fixed", C.c_void_p), ("sphere_off", C.c_void_p),
                ("sphere_frame", C.c_void_p), ("sphere_xyzr", C.c_void_p),
                ("self_off", C.c_void_p), ("self_pairs", C.c_void_p), ("base", C.c_void_p)]


class _Env(C.Structure):
    _fields_ = [("n_spheres", C.c_int32), ("spheres", C.c_void_p),
                ("n_boxes", C.c_int32), ("boxes", C.c_void_p),
                ("n_cyls", C.c_int32), ("cyls", C.c_void_p),
                ("n_points", C.c_int64), ("points", C.c_void_p),
                ("point_radius", C.c_double),
                ("kd_perm", C.c_void_p), ("kd_split", C.c_void_p), ("kd_axis", C.c_void_p),
                ("kd_nodes", C.c_int64)]


class _Paths(C.Structure):
    _fields_ = [("n_queries", C.c_int32), ("n_robots", C.c_int32), ("dof_stride", C.c_int32),
                ("wp_begin", C.c_void_p), ("wp_t", C.c_void_p), ("wp_q", C.c_void_p)]


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
                build()
            L = C.CDLL(LIB)
            P, D, I32, I64 = C.c_void_p, C.c_double, C.c_int32, C.c_int64
            L.orc_clear_sphere_sphere.argtypes = [P, D, P, D]
            L.orc_clear_sphere_box.argtypes = [P, D, P]
            L.orc_clear_sphere_cylinder.argtypes = [P, D, P]
            L.orc_clear_sphere_point.argtypes = [P, D, P, D]
            for f in ("orc_clear_sphere_sphere", "orc_clear_sphere_box",
                      "orc_clear_sphere_cylinder", "orc_clear_sphere_point"):
                getattr(L, f).restype = D
            L.orc_fk_robot.argtypes = [P, I32, P, P, P]
            L.orc_fk_robot.restype = None
            L.orc_path_state.argtypes = [P, P, I64, I32, I32, I64, P]
            L.orc_path_state.restype = None
            L.orc_query_horizon.argtypes = [P, I64]
            L.orc_query_horizon.restype = I64
            L.orc_mv.argtypes = [P, P, P, I64, I64, I32, I32, C.c_uint32, P, P, I32]
            L.orc_mv.restype = C.c_int
            L.orc_ffc.argtypes = [P, P, I64, I64, P, I32]
            L.orc_ffc.restype = C.c_int
            L.orc_team_spheres.argtypes = [P, P, I64, I64, P]
            L.orc_team_spheres.restype = None
            L.orc_motion_steps.argtypes = [P, I32, D, I32]
            L.orc_motion_steps.restype = I64
            L.orc_env_build.argtypes = [P]
            L.orc_env_build.restype = C.c_int
            L.orc_env_free.argtypes = [P]
            L.orc_env_free.restype = None
            L.orc_points_any_hit.argtypes = [P, P, D]
            L.orc_points_any_hit.restype = C.c_int
            L.orc_points_any_hit_brute.argtypes = [P, P, D]
            L.orc_points_any_hit_brute.restype = C.c_int
            L.orc_threads.argtypes = []
            L.orc_threads.restype = C.c_int
            _lib = L
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


class Team:
    """Flat FP64 team arrays in the oracle's own layout."""

    def __init__(self, robots):
        self.robots = list(robots)
        n = len(self.robots)
        self.n_joints = np.array([r.dof for r in self.robots], np.int32)
        self.joint_off = np.concatenate([[0], np.cumsum(self.n_joints)[:-1]]).astype(np.int32)
        self.joint_type = np.ascontiguousarray(np.concatenate([r.joint_type for r in self.robots]).astype(np.int32))
        self.joint_fixed = np.ascontiguousarray(np.concatenate([r.joint_fixed for r in self.robots]).astype(np.float64))
        ns = [r.n_spheres for r in self.robots]
        self.sphere_off = np.concatenate([[0], np.cumsum(ns)]).astype(np.int32)
        self.sphere_frame = np.ascontiguousarray(np.concatenate([r.sphere_frame for r in self.robots]).astype(np.int32))
        self.sphere_xyzr = np.ascontiguousarray(np.concatenate([r.sphere_xyzr for r in self.robots]).astype(np.float64))
        npairs = [len(r.self_pairs) for r in self.robots]
        self.self_off = np.concatenate([[0], np.cumsum(npairs)]).astype(np.int32)
        sp = [r.self_pairs.reshape(-1, 2) for r in self.robots]
        self.self_pairs = np.ascontiguousarray(np.concatenate(sp).astype(np.int32)) if sp else np.zeros((0, 2), np.int32)
        if self.self_pairs.size == 0:
            self.self_pairs = np.zeros((1, 2), np.int32)
        self.base = np.ascontiguousarray(np.stack([r.base for r in self.robots]).astype(np.float64))
        self.c = _Team(n, _ptr(self.n_joints), _ptr(self.joint_off), _ptr(self.joint_type),
                       _ptr(self.joint_fixed), _ptr(self.sphere_off), _ptr(self.sphere_frame),
                       _ptr(self.sphere_xyzr), _ptr(self.self_off), _ptr(self.self_pairs),
                       _ptr(self.base))

    @property
    def n_robots(self):
        return len(self.robots)

    @property
    def total_spheres(self):
        return int(self.sphere_off[-1])


class Env:
    def __init__(self, env, build_index: bool = True):
        self.spheres = np.ascontiguousarray(np.asarray(env.spheres, np.float64).reshape(-1, 4))
        self.boxes = np.ascontiguousarray(np.asarray(env.boxes, np.float64).reshape(-1, 15))
        self.cyls = np.ascontiguousarray(np.asarray(env.cylinders, np.float64).reshape(-1, 8))
        self.points = np.ascontiguousarray(np.asarray(env.points, np.float64).reshape(-1, 3))
        self.c = _Env(len(self.spheres), _ptr(self.spheres), len(self.boxes), _ptr(self.boxes),
                      len(self.cyls), _ptr(self.cyls), len(self.points), _ptr(self.points),
                      float(env.point_radius), None, None, None, 0)
        self._built = False
        if build_index and len(self.points):
            if lib().orc_env_build(C.byref(self.c)) != 0:
                raise MemoryError("oracle: k-d tree allocation failed")
            self._built = True

    def __del__(self):
        if getattr(self, "_built", False) and _lib is not None:
            _lib.orc_env_free(C.byref(self.c))


class Paths:
    def __init__(self, paths):
        self.py = paths
        self.wp_begin = np.ascontiguousarray(paths.wp_begin.astype(np.int64))
        self.wp_t = np.ascontiguousarray(paths.wp_t.astype(np.int32))
        self.wp_q = np.ascontiguousarray(paths.wp_q.astype(np.float64))
        self.c = _Paths(paths.n_queries, paths.n_robots, paths.dof_stride, _ptr(self.wp_begin),
                        _ptr(self.wp_t), _ptr(self.wp_q))


def mv(team: Team, env: Env | None, paths: Paths, check_env: bool = True, q0: int = 0,
       q1: int | None = None, nthreads: int = 0, first_hit: bool = False, exhaustive: bool = False,
       focus: int = 0):
    """MV (Alg. 1).  focus: bit r puts robot r in focus (prioritised MV, §III-C):
    only robots in focus get obstacle and self tests, and only robot pairs with a
    robot in focus are tested; 0 = every robot."""
    q1 = paths.py.n_queries if q1 is None else q1
    out = np.zeros(q1 - q0, np.uint8)
    fh = np.zeros(q1 - q0, np.int64) if first_hit else None
    rc = lib().orc_mv(C.byref(team.c), C.byref(env.c) if env is not None else None,
                      C.byref(paths.c), q0, q1, int(bool(check_env)), int(bool(exhaustive)), int(focus) & 0xFFFFFFFF,
                      _ptr(out), _ptr(fh) if fh is not None else None, nthreads)
    if rc != 0:
        raise MemoryError("oracle MV failed")
    return (out, fh) if first_hit else out


def ffc(team: Team, paths: Paths, q0: int = 0, q1: int | None = None, nthreads: int = 0):
    q1 = paths.py.n_queries if q1 is None else q1
    out = np.zeros((q1 - q0, 3), np.int32)
    rc = lib().orc_ffc(C.byref(team.c), C.byref(paths.c), q0, q1, _ptr(out), nthreads)
    if rc != 0:
        raise MemoryError("oracle FFC failed")
    return out


def fk_robot(team: Team, r: int, q, frames: bool = False):
    q = np.ascontiguousarray(np.asarray(q, np.float64))
    ns = team.robots[r].n_spheres
    out = np.zeros((ns, 4))
    fr = np.zeros((team.robots[r].dof + 1, 12)) if frames else None
    lib().orc_fk_robot(C.byref(team.c), r, _ptr(q), _ptr(out), _ptr(fr) if frames else None)
    return (out, fr) if frames else out


def team_spheres(team: Team, paths: Paths, qi: int, t: int):
    out = np.zeros((team.total_spheres, 4))
    lib().orc_team_spheres(C.byref(team.c), C.byref(paths.c), qi, t, _ptr(out))
    return out


def path_state(times, configs, dof: int, t: int):
    times = np.ascontiguousarray(np.asarray(times, np.int32))
    configs = np.ascontiguousarray(np.asarray(configs, np.float64).reshape(len(times), -1))
    out = np.zeros(dof)
    lib().orc_path_state(_ptr(times), _ptr(configs), len(times), configs.shape[1], dof, t, _ptr(out))
    return out


def horizon(paths: Paths, qi: int) -> int:
    return int(lib().orc_query_horizon(C.byref(paths.c), qi))


def clear_sphere_sphere(x, r, y, s):
    x = np.ascontiguousarray(x, np.float64); y = np.ascontiguousarray(y, np.float64)
    return lib().orc_clear_sphere_sphere(_ptr(x), r, _ptr(y), s)


def clear_sphere_box(x, r, box):
    x = np.ascontiguousarray(x, np.float64); box = np.ascontiguousarray(box, np.float64)
    return lib().orc_clear_sphere_box(_ptr(x), r, _ptr(box))


def clear_sphere_cylinder(x, r, cyl):
    x = np.ascontiguousarray(x, np.float64); cyl = np.ascontiguousarray(cyl, np.float64)
    return lib().orc_clear_sphere_cylinder(_ptr(x), r, _ptr(cyl))


def clear_sphere_point(x, r, p, rp):
    x = np.ascontiguousarray(x, np.float64); p = np.ascontiguousarray(p, np.float64)
    return lib().orc_clear_sphere_point(_ptr(x), r, _ptr(p), rp)


def points_any_hit(env: Env, x, r, brute: bool = False) -> bool:
    x = np.ascontiguousarray(x, np.float64)
    f = lib().orc_points_any_hit_brute if brute else lib().orc_points_any_hit
    return bool(f(C.byref(env.c), _ptr(x), r))


def motion_steps(dq, step: float, metric: str) -> int:
    dq = np.ascontiguousarray(np.asarray(dq, np.float64))
    return int(lib().orc_motion_steps(_ptr(dq), len(dq), step, 0 if metric == "l2" else 1))


def threads() -> int:
    return int(lib().orc_threads())
