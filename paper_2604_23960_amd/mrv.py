"""Thin ctypes binding of libmrv (C ABI in include/mrv.h).

Argument marshalling only: every step of MV/FFC runs in the HIP library.  The
library must have been built (``paper_2604_23960_amd.build``); loading fails
loudly otherwise.  PyTorch, when used, only supplies device memory and the
stream (``*_device`` calls take torch CUDA tensors).
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmrv.so")

MRV_OK, MRV_PENDING = 0, 1
MRV_E_INVALID, MRV_E_NOMEM, MRV_E_DEVICE, MRV_E_BUSY = -1, -2, -3, -4
MRV_E_HANDLE, MRV_E_CANCELLED, MRV_E_TIMEOUT = -5, -6, -7
CHECK_ENV, EXHAUSTIVE, HIERARCHICAL = 1, 2, 4
ORDER_BISECT, ORDER_RAKE, ORDER_LINEAR = 0, 8, 16
PAIRS_FIRST, OBSTACLES_FIRST, PAIR_PRIORITY = 32, 64, 128
MAX_T = 1 << 20
NOALLOC_MAX_QUERIES = 1 << 18

EXPORTS = ["mrv_create", "mrv_destroy", "mrv_last_error", "mrv_load_team", "mrv_load_env", "mrv_unload",
           "mrv_mv", "mrv_ffc", "mrv_mv_device", "mrv_ffc_device", "mrv_sync", "mrv_motion_steps",
           "mrv_set_tiling", "mrv_get_tiling", "mrv_last_stats", "mrv_submit", "mrv_poll", "mrv_wait",
           "mrv_cancel", "mrv_autotune", "mrv_graph_create", "mrv_graph_launch", "mrv_graph_destroy",
           "mrv_spheres", "mrv_mv_focus", "mrv_mv_focus_device", "mrv_memory_stats", "mrv_mv_device_noalloc"]


class MrvError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"mrv status {status}: {msg}")
        self.status = status


class CtxOpts(C.Structure):
    _fields_ = [("device", C.c_int32), ("stream", C.c_void_p), ("device_arena", C.c_void_p),
                ("arena_bytes", C.c_size_t), ("near_eps", C.c_double),
                ("max_inflight", C.c_int32), ("serve_bytes", C.c_size_t), ("recheck_records", C.c_int64),
                ("flags", C.c_uint32)]


class RobotDesc(C.Structure):
    _fields_ = [("n_joints", C.c_int32), ("joint_type", C.c_void_p), ("joint_fixed", C.c_void_p),
                ("n_spheres", C.c_int32), ("sphere_frame", C.c_void_p), ("sphere_xyzr", C.c_void_p),
                ("n_self_pairs", C.c_int32), ("self_pairs", C.c_void_p), ("base", C.c_double * 12)]


class EnvDesc(C.Structure):
    _fields_ = [("n_spheres", C.c_int32), ("spheres", C.c_void_p), ("n_boxes", C.c_int32),
                ("boxes", C.c_void_p), ("n_cyls", C.c_int32), ("cylinders", C.c_void_p),
                ("n_points", C.c_int64), ("points", C.c_void_p), ("point_radius", C.c_double),
                ("grid_cell", C.c_double)]


class PathsDesc(C.Structure):
    _fields_ = [("n_queries", C.c_int32), ("dof_stride", C.c_int32), ("wp_begin", C.c_void_p),
                ("wp_t", C.c_void_p), ("wp_q", C.c_void_p), ("n_wp", C.c_int64)]


class Conflict(C.Structure):
    _fields_ = [("t", C.c_int32), ("ri", C.c_int32), ("rj", C.c_int32)]


class Tiling(C.Structure):
    _fields_ = [("chunk", C.c_int32), ("wg_per_cu", C.c_int32), ("interleave", C.c_int32), ("claim", C.c_int32)]

    def as_tuple(self):
        return self.chunk, self.wg_per_cu, self.interleave, self.claim


class Stats(C.Structure):
    _fields_ = [("tiles_run", C.c_uint64), ("tiles_skipped", C.c_uint64),
                ("states_evaluated", C.c_uint64), ("states_covered", C.c_uint64),
                ("rr_tests", C.c_uint64), ("env_tests", C.c_uint64), ("self_tests", C.c_uint64),
                ("near_rechecks", C.c_uint64), ("kernel_ms", C.c_double), ("point_tests", C.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Request(C.Structure):
    _fields_ = [("kind", C.c_int32), ("team", C.c_int32), ("env", C.c_int32), ("flags", C.c_uint32),
                ("paths", PathsDesc), ("focus", C.c_uint32)]


_lib = None
_lock = threading.Lock()


def lib():
    """Load libmrv.so; raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(f"{LIB_PATH} is missing: build it with paper_2604_23960_amd.build")
            L = C.CDLL(LIB_PATH)
            P, I32, U32, I64 = C.c_void_p, C.c_int32, C.c_uint32, C.c_int64
            sig = {
                "mrv_create": [C.POINTER(CtxOpts), C.POINTER(C.c_void_p)],
                "mrv_destroy": [P],
                "mrv_load_team": [P, P, I32, C.POINTER(I32)],
                "mrv_load_env": [P, C.POINTER(EnvDesc), C.POINTER(I32)],
                "mrv_unload": [P, I32],
                "mrv_mv": [P, I32, I32, C.POINTER(PathsDesc), U32, P],
                "mrv_ffc": [P, I32, C.POINTER(PathsDesc), U32, P],
                "mrv_mv_device": [P, I32, I32, C.POINTER(PathsDesc), U32, P],
                "mrv_mv_device_noalloc": [P, I32, I32, C.POINTER(PathsDesc), U32, P],
                "mrv_mv_focus": [P, I32, I32, C.POINTER(PathsDesc), U32, U32, P],
                "mrv_mv_focus_device": [P, I32, I32, C.POINTER(PathsDesc), U32, U32, P],
                "mrv_ffc_device": [P, I32, C.POINTER(PathsDesc), U32, P],
                "mrv_sync": [P],
                "mrv_set_tiling": [P, I32, I32, U32, C.POINTER(Tiling)],
                "mrv_get_tiling": [P, I32, I32, U32, C.POINTER(Tiling)],
                "mrv_last_stats": [P, C.POINTER(Stats)],
                "mrv_submit": [P, C.POINTER(Request), C.POINTER(C.c_uint64)],
                "mrv_poll": [P, C.c_uint64, P],
                "mrv_wait": [P, C.c_uint64, I32, P],
                "mrv_cancel": [P, C.c_uint64],
                "mrv_autotune": [P, I32, I32, I32, C.POINTER(PathsDesc), U32, C.POINTER(Tiling)],
                "mrv_graph_create": [P, I32, I32, I32, C.POINTER(PathsDesc), U32, P, C.POINTER(C.c_void_p)],
                "mrv_graph_launch": [P, P],
                "mrv_graph_destroy": [P, P],
                "mrv_spheres": [P, I32, C.POINTER(PathsDesc), I32, P, P, P],
                "mrv_memory_stats": [P, P, P, P],
            }
            for name, args in sig.items():
                f = getattr(L, name)
                f.argtypes = args
                f.restype = I32
            L.mrv_last_error.argtypes = []
            L.mrv_last_error.restype = C.c_char_p
            L.mrv_motion_steps.argtypes = [P, I32, C.c_double, I32]
            L.mrv_motion_steps.restype = I64
            _lib = L
    return _lib


def last_error() -> str:
    return lib().mrv_last_error().decode()


def check(status: int) -> int:
    if status < 0:
        raise MrvError(status, last_error())
    return status


def _c(a, dtype):
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


def motion_steps(dq, step: float, metric: str) -> int:
    dq = _c(dq, np.float64)
    n = lib().mrv_motion_steps(dq.ctypes.data, len(dq), step, 0 if metric == "l2" else 1)
    if n < 0:
        raise MrvError(MRV_E_INVALID, last_error())
    return int(n)


class HostPaths:
    """Keeps the numpy arrays of a path set alive next to its C descriptor."""

    def __init__(self, paths):
        self.wp_begin = _c(paths.wp_begin, np.int64)
        self.wp_t = _c(paths.wp_t, np.int32)
        self.wp_q = _c(paths.wp_q, np.float64)
        self.n_queries = int(paths.n_queries)
        self.desc = PathsDesc(self.n_queries, int(paths.dof_stride), self.wp_begin.ctypes.data,
                              self.wp_t.ctypes.data, self.wp_q.ctypes.data, int(self.wp_begin[-1]))


class DevicePaths:
    """Path arrays resident in device memory (torch tensors on the context's device)."""

    def __init__(self, paths, device="cuda"):
        import torch
        self.wp_begin = torch.as_tensor(np.asarray(paths.wp_begin, np.int64)).to(device)
        self.wp_t = torch.as_tensor(np.asarray(paths.wp_t, np.int32)).to(device)
        self.wp_q = torch.as_tensor(np.ascontiguousarray(paths.wp_q, np.float64)).to(device)
        self.n_queries = int(paths.n_queries)
        self.desc = PathsDesc(self.n_queries, int(paths.dof_stride), self.wp_begin.data_ptr(),
                              self.wp_t.data_ptr(), self.wp_q.data_ptr(), int(paths.wp_begin[-1]))


class Context:
    """device_arena: a torch uint8 CUDA tensor whose memory the library sub-allocates
    for every device buffer of the context (kept alive by the context)."""

    def __init__(self, device: int = 0, stream=None, near_eps: float = 0.0, max_inflight: int = 0,
                 serve_bytes: int = 0, recheck_records: int = 0, device_arena=None):
        self._keep = []
        arena_ptr, arena_bytes = None, 0
        if device_arena is not None:
            arena_ptr, arena_bytes = device_arena.data_ptr(), device_arena.numel() * device_arena.element_size()
            self._keep.append(device_arena)
        h = C.c_void_p()
        opts = CtxOpts(device, stream, arena_ptr, arena_bytes, near_eps, max_inflight, serve_bytes,
                       recheck_records, 0)
        check(lib().mrv_create(C.byref(opts), C.byref(h)))
        self.h = h

    def memory_stats(self) -> dict:
        """Device bytes now allocated, the most allocated at once, the arena's usable size."""
        v = [C.c_size_t() for _ in range(3)]
        check(lib().mrv_memory_stats(self.h, *[C.byref(x) for x in v]))
        return dict(used=v[0].value, peak=v[1].value, capacity=v[2].value)

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            check(lib().mrv_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- resident data
    def load_team(self, robots) -> int:
        descs = (RobotDesc * len(robots))()
        keep = []
        for i, r in enumerate(robots):
            jt, jf = _c(r.joint_type, np.int32), _c(r.joint_fixed, np.float64)
            sf, sx = _c(r.sphere_frame, np.int32), _c(r.sphere_xyzr, np.float64)
            sp = _c(np.asarray(r.self_pairs).reshape(-1, 2), np.int32)
            keep += [jt, jf, sf, sx, sp]
            d = descs[i]
            d.n_joints = len(jt)
            d.joint_type = jt.ctypes.data
            d.joint_fixed = jf.ctypes.data
            d.n_spheres = len(sf)
            d.sphere_frame = sf.ctypes.data
            d.sphere_xyzr = sx.ctypes.data
            d.n_self_pairs = len(sp)
            d.self_pairs = sp.ctypes.data if len(sp) else None
            for k in range(12):
                d.base[k] = float(r.base[k])
        out = C.c_int32()
        check(lib().mrv_load_team(self.h, descs, len(robots), C.byref(out)))
        return out.value

    def load_env(self, env) -> int:
        sp = _c(np.asarray(env.spheres).reshape(-1, 4), np.float64)
        bx = _c(np.asarray(env.boxes).reshape(-1, 15), np.float64)
        cy = _c(np.asarray(env.cylinders).reshape(-1, 8), np.float64)
        pt = _c(np.asarray(env.points).reshape(-1, 3), np.float64)
        d = EnvDesc(len(sp), sp.ctypes.data if len(sp) else None, len(bx), bx.ctypes.data if len(bx) else None,
                    len(cy), cy.ctypes.data if len(cy) else None, len(pt), pt.ctypes.data if len(pt) else None,
                    float(env.point_radius), float(getattr(env, "grid_cell", 0.0) or 0.0))
        out = C.c_int32()
        check(lib().mrv_load_env(self.h, C.byref(d), C.byref(out)))
        return out.value

    def unload(self, handle: int):
        check(lib().mrv_unload(self.h, handle))

    # -- host-array calls
    def mv(self, team: int, env: int, paths, flags: int = CHECK_ENV, focus: int = 0) -> np.ndarray:
        """focus != 0: prioritised MV over the robots whose bits are set (mrv_mv_focus)."""
        hp = paths if isinstance(paths, HostPaths) else HostPaths(paths)
        out = np.zeros(max(hp.n_queries, 1), np.uint8)
        if focus:
            check(lib().mrv_mv_focus(self.h, team, env, C.byref(hp.desc), flags, focus, out.ctypes.data))
        else:
            check(lib().mrv_mv(self.h, team, env, C.byref(hp.desc), flags, out.ctypes.data))
        return out[:hp.n_queries]

    def ffc(self, team: int, paths, flags: int = 0) -> np.ndarray:
        hp = paths if isinstance(paths, HostPaths) else HostPaths(paths)
        out = np.zeros((max(hp.n_queries, 1), 3), np.int32)
        check(lib().mrv_ffc(self.h, team, C.byref(hp.desc), flags, out.ctypes.data))
        return out[:hp.n_queries]

    # -- device-array calls (async on the context stream)
    def mv_device(self, team: int, env: int, dpaths: DevicePaths, flags: int, out_ptr: int, focus: int = 0):
        if focus:
            check(lib().mrv_mv_focus_device(self.h, team, env, C.byref(dpaths.desc), flags, focus, out_ptr))
        else:
            check(lib().mrv_mv_device(self.h, team, env, C.byref(dpaths.desc), flags, out_ptr))

    def mv_device_noalloc(self, team: int, env: int, dpaths: DevicePaths, flags: int, out_ptr: int):
        """mv_device with the library's fixed per-device scratch: allocates nothing."""
        check(lib().mrv_mv_device_noalloc(self.h, team, env, C.byref(dpaths.desc), flags, out_ptr))

    def ffc_device(self, team: int, dpaths: DevicePaths, flags: int, out_ptr: int):
        check(lib().mrv_ffc_device(self.h, team, C.byref(dpaths.desc), flags, out_ptr))

    def sync(self):
        check(lib().mrv_sync(self.h))

    def spheres(self, team: int, paths, state_query, state_t, total_spheres: int) -> np.ndarray:
        """FP32 world sphere centres/radii [n_states, S, 4] as the kernels compute them."""
        hp = paths if isinstance(paths, HostPaths) else HostPaths(paths)
        sq = _c(state_query, np.int32)
        st = _c(state_t, np.int32)
        out = np.zeros((max(len(sq), 1), total_spheres, 4), np.float32)
        check(lib().mrv_spheres(self.h, team, C.byref(hp.desc), len(sq), sq.ctypes.data, st.ctypes.data,
                                out.ctypes.data))
        return out[:len(sq)]

    # -- tuning / stats
    def set_tiling(self, team: int, kind: int, chunk: int = 0, wg_per_cu: int = 0, flags: int | None = None,
                   interleave: int = 0, claim: int = 0):
        """flags None: both modes (early-terminating and exhaustive)."""
        t = Tiling(chunk, wg_per_cu, interleave, claim)
        for f in ((0, EXHAUSTIVE) if flags is None else (flags,)):
            check(lib().mrv_set_tiling(self.h, team, kind, f, C.byref(t)))

    def get_tiling(self, team: int, kind: int, flags: int = 0):
        """(chunk, wg_per_cu, interleave, claim) in effect."""
        t = Tiling()
        check(lib().mrv_get_tiling(self.h, team, kind, flags, C.byref(t)))
        return t.as_tuple()

    def last_stats(self) -> dict:
        s = Stats()
        check(lib().mrv_last_stats(self.h, C.byref(s)))
        return s.as_dict()

    def autotune(self, team: int, env: int, kind: int, sample_paths, flags: int):
        hp = sample_paths if isinstance(sample_paths, HostPaths) else HostPaths(sample_paths)
        t = Tiling()
        check(lib().mrv_autotune(self.h, team, env, kind, C.byref(hp.desc), flags, C.byref(t)))
        return t.as_tuple()

    # -- captured graphs
    def graph_create(self, team: int, env: int, kind: int, dpaths: DevicePaths, flags: int, out_ptr: int):
        g = C.c_void_p()
        check(lib().mrv_graph_create(self.h, team, env, kind, C.byref(dpaths.desc), flags, out_ptr, C.byref(g)))
        return g

    def graph_launch(self, g):
        check(lib().mrv_graph_launch(self.h, g))

    def graph_destroy(self, g):
        check(lib().mrv_graph_destroy(self.h, g))

    # -- serving
    def submit(self, kind: int, team: int, env: int, paths, flags: int, focus: int = 0) -> int:
        hp = paths if isinstance(paths, HostPaths) else HostPaths(paths)
        req = Request(kind, team, env, flags, hp.desc, focus)
        t = C.c_uint64()
        check(lib().mrv_submit(self.h, C.byref(req), C.byref(t)))
        return t.value

    def poll(self, ticket: int, kind: int, n_queries: int, timeout_ms: int | None = 0):
        """Returns the result array, or None while pending (timeout_ms=0)."""
        out = np.zeros(max(n_queries, 1), np.uint8) if kind == 0 else np.zeros((max(n_queries, 1), 3), np.int32)
        if timeout_ms == 0:
            s = lib().mrv_poll(self.h, ticket, out.ctypes.data)
        else:
            s = lib().mrv_wait(self.h, ticket, -1 if timeout_ms is None else timeout_ms, out.ctypes.data)
        if s == MRV_PENDING:
            return None
        check(s)
        return out[:n_queries]

    def cancel(self, ticket: int):
        check(lib().mrv_cancel(self.h, ticket))
