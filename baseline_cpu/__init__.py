"""CPU SIMD baseline in the style of the paper's own implementation (rake
packing of W = 8 timesteps per batch, FP32, early exit; §III-A, §IV-A), for
measurement next to the GPU library on the same host.  ``simd_rake.c`` is built
with gcc (AVX2 via 8-wide vector extensions, OpenMP over queries).

Used only by ``bench.py`` and its tests.  It is neither the FP64 oracle (plain
FP32 without near-contact re-evaluation, so a test within rounding of contact
may answer differently) nor part of the GPU library, which never calls it.
Point-cloud environments are not supported.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "simd_rake.c")
LIB = os.path.join(HERE, "libsimdrake.so")
_lib = None


def build() -> str:
    cmd = ["gcc", "-O3", "-march=x86-64-v3", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-o", LIB + ".tmp", SRC,
           "-lm"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("gcc failed building the SIMD baseline:\n" + res.stderr)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB)
        P, I32, I64 = C.c_void_p, C.c_int32, C.c_int64
        L.simd_mv.argtypes = [I32, P, P, P, P, P, P, P, P, P, I32, P, I32, P, I32, P, I32, I32, I64, I32, P, P, P, P,
                              P, I32]
        L.simd_mv.restype = C.c_int
        _lib = L
    return _lib


def _a(x, dt):
    return np.ascontiguousarray(np.asarray(x, dtype=dt))


def _p(a):
    return a.ctypes.data if a.size else None


def mv(team, env, paths, check_env: bool = True, exhaustive: bool = False, nthreads: int = 0):
    """MV of every query of ``paths`` (workloads.Paths) for ``team`` (list of
    workloads.Robot) and ``env`` (workloads.Env or None).  Returns (valid uint8
    [Q], robot-states evaluated)."""
    if env is not None and len(np.asarray(env.points).reshape(-1, 3)):
        raise ValueError("the SIMD baseline does not handle point clouds")
    n = len(team)
    nj = _a([r.dof for r in team], np.int32)
    jtype = _a(np.concatenate([r.joint_type for r in team]), np.int32)
    jfixed = _a(np.concatenate([np.asarray(r.joint_fixed).reshape(-1, 12) for r in team]), np.float64)
    base = _a(np.stack([np.asarray(r.base).reshape(12) for r in team]), np.float64)
    ns = _a([r.n_spheres for r in team], np.int32)
    sframe = _a(np.concatenate([r.sphere_frame for r in team]), np.int32)
    sxyzr = _a(np.concatenate([np.asarray(r.sphere_xyzr).reshape(-1, 4) for r in team]), np.float64)
    nself = _a([len(np.asarray(r.self_pairs).reshape(-1, 2)) for r in team], np.int32)
    pairs = _a(np.concatenate([np.asarray(r.self_pairs).reshape(-1, 2) for r in team]), np.int32)
    if env is None:
        sph, box, cyl = np.zeros((0, 4)), np.zeros((0, 15)), np.zeros((0, 8))
    else:
        sph = _a(np.asarray(env.spheres).reshape(-1, 4), np.float64)
        box = _a(np.asarray(env.boxes).reshape(-1, 15), np.float64)
        cyl = _a(np.asarray(env.cylinders).reshape(-1, 8), np.float64)
    wb = _a(paths.wp_begin, np.int64)
    wt = _a(paths.wp_t, np.int32)
    wq = _a(paths.wp_q, np.float64)
    out = np.zeros(max(paths.n_queries, 1), np.uint8)
    states = C.c_int64(0)
    rc = lib().simd_mv(n, _p(nj), _p(jtype), _p(jfixed), _p(base), _p(ns), _p(sframe), _p(sxyzr), _p(nself),
                       _p(pairs), len(sph), _p(sph), len(box), _p(box), len(cyl), _p(cyl), int(bool(check_env)),
                       int(bool(exhaustive)), paths.n_queries, paths.dof_stride, _p(wb), _p(wt), _p(wq), _p(out),
                       C.byref(states), int(nthreads))
    if rc != 0:
        raise ValueError("SIMD baseline rejected its arguments")
    return out[:paths.n_queries], states.value
