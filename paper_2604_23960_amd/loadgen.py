"""Simulated planner clients for the serving loop (mrv_submit / mrv_wait) and for
the plain one-call-per-query form.

Every request is one MV or FFC query of one client's resident team.  Arrivals
follow a Poisson process of total rate ``rate`` (requests/s; ``inf`` = all at
once).  Latency = completion time - arrival time, so queueing delay counts.
"""
from __future__ import annotations

import ctypes as C
import math
import threading
import time

import numpy as np

from . import mrv


def arrival_times(n: int, rate: float, seed: int = 0) -> np.ndarray:
    if not math.isfinite(rate):
        return np.zeros(n)
    rng = np.random.default_rng([seed, 7])
    return np.cumsum(rng.exponential(1.0 / rate, n))


def _sleep_until(t_abs: float):
    while True:
        d = t_abs - time.perf_counter()
        if d <= 0:
            return
        # sleep(0) still yields the interpreter lock to the thread collecting results
        time.sleep(d - 1e-3 if d > 2e-3 else 0)


def summarize(lat: np.ndarray, t_first: float, t_last: float, states: float) -> dict:
    """Throughput and latency of one run.  ``sustained``: the queue did not grow over
    the run, i.e. the mean latency of the last quarter of the requests (in arrival
    order) is within twice that of the first quarter plus a millisecond."""
    span = max(t_last - t_first, 1e-9)
    q = max(len(lat) // 4, 1)
    head, tail = float(lat[:q].mean()), float(lat[-q:].mean())
    return dict(queries=int(len(lat)), seconds=span, qps=len(lat) / span, states_per_s=states / span,
                p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(np.percentile(lat, 99) * 1e3),
                mean_ms=float(lat.mean() * 1e3), first_quarter_ms=head * 1e3, last_quarter_ms=tail * 1e3,
                sustained=bool(tail <= 2.0 * head + 1e-3))


def _states(reqs) -> float:
    return float(sum(r.horizon * len(r.paths.wp_begin[:-1]) // max(r.paths.n_queries, 1) for r in reqs))


def prepare(reqs):
    """Host descriptors built once so the timed loops only marshal pointers."""
    return [mrv.HostPaths(r.paths) for r in reqs]


def run_served(ctx: mrv.Context, handles, env: int, reqs, hps, rate: float, seed: int = 0,
               flags_mv: int = mrv.CHECK_ENV, flags_ffc: int = 0):
    """Submit on one thread at the arrival times, collect on another.  The C request
    structs and result buffers are built before the clock starts so the timed
    loops only cross the C ABI."""
    n = len(reqs)
    L = mrv.lib()
    arr = arrival_times(n, rate, seed)
    creq = [mrv.Request(r.kind, handles[r.client], env if r.kind == 0 else -1,
                        flags_mv if r.kind == 0 else flags_ffc, hps[i].desc) for i, r in enumerate(reqs)]
    outs = [np.zeros(1, np.uint8) if r.kind == 0 else np.zeros((1, 3), np.int32) for r in reqs]
    optr = [o.ctypes.data for o in outs]
    tickets = (C.c_uint64 * max(n, 1))()
    tptr = [C.cast(C.addressof(tickets) + 8 * i, C.POINTER(C.c_uint64)) for i in range(n)]
    rptr = [C.pointer(x) for x in creq]
    arrive = np.zeros(n)
    done = np.zeros(n)
    ready = threading.Semaphore(0)
    errors = []
    t0 = time.perf_counter() + 0.01

    def submitter():
        try:
            for i in range(n):
                _sleep_until(t0 + arr[i])
                arrive[i] = t0 + arr[i]
                while True:
                    st = L.mrv_submit(ctx.h, rptr[i], tptr[i])
                    if st == mrv.MRV_OK:
                        break
                    if st != mrv.MRV_E_BUSY:
                        raise mrv.MrvError(st, mrv.last_error())
                    time.sleep(0)
                ready.release()
        except Exception as e:      # surface in the main thread
            errors.append(e)
            ready.release()

    th = threading.Thread(target=submitter)
    th.start()
    for i in range(n):
        ready.acquire()
        if errors:
            break
        st = L.mrv_wait(ctx.h, tickets[i], -1, optr[i])
        if st != mrv.MRV_OK:
            errors.append(mrv.MrvError(st, mrv.last_error()))
            break
        done[i] = time.perf_counter()
    th.join()
    if errors:
        raise errors[0]
    lat = done - arrive
    results = [o[0] if r.kind == 0 else o for o, r in zip(outs, reqs)]
    return summarize(lat, arrive.min(), done.max(), _states(reqs)), [np.atleast_1d(x) for x in results]


def run_plain(ctx: mrv.Context, handles, env: int, reqs, hps, rate: float, seed: int = 0,
              flags_mv: int = mrv.CHECK_ENV, flags_ffc: int = 0):
    n = len(reqs)
    arr = arrival_times(n, rate, seed)
    arrive = np.zeros(n)
    done = np.zeros(n)
    results = [None] * n
    t0 = time.perf_counter() + 0.01
    for i, r in enumerate(reqs):
        _sleep_until(t0 + arr[i])
        arrive[i] = t0 + arr[i]
        if r.kind == 0:
            results[i] = ctx.mv(handles[r.client], env, hps[i], flags_mv)
        else:
            results[i] = ctx.ffc(handles[r.client], hps[i], flags_ffc)
        done[i] = time.perf_counter()
    lat = done - arrive
    return summarize(lat, arrive.min(), done.max(), _states(reqs)), results


def run_plain_streams(ctxs, handles_per_ctx, envs, reqs, hps, rate: float, seed: int = 0,
                      flags_mv: int = mrv.CHECK_ENV, flags_ffc: int = 0):
    """The plain form on several streams: one host thread per context (each with
    its own stream and resident copies of the teams), request i taken by thread
    i mod len(ctxs) at its arrival time, one synchronous call per query."""
    n, k = len(reqs), len(ctxs)
    arr = arrival_times(n, rate, seed)
    arrive = np.zeros(n)
    done = np.zeros(n)
    results = [None] * n
    t0 = time.perf_counter() + 0.01
    errors = []

    def worker(w):
        try:
            ctx, handles, env = ctxs[w], handles_per_ctx[w], envs[w]
            for i in range(w, n, k):
                _sleep_until(t0 + arr[i])
                arrive[i] = max(t0 + arr[i], arrive[i])
                r = reqs[i]
                if r.kind == 0:
                    results[i] = ctx.mv(handles[r.client], env, hps[i], flags_mv)
                else:
                    results[i] = ctx.ffc(handles[r.client], hps[i], flags_ffc)
                done[i] = time.perf_counter()
        except Exception as e:
            errors.append(e)

    ths = [threading.Thread(target=worker, args=(w,)) for w in range(k)]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    if errors:
        raise errors[0]
    arrive[:] = t0 + arr
    lat = done - arrive
    return summarize(lat, arrive.min(), done.max(), _states(reqs)), results


def binding_overhead_us(ctx: mrv.Context, handle: int, dof_stride: int, reps: int = 2000) -> float:
    """Host time of one plain-form call through the Python binding (output array,
    argument marshalling, the C call) on an empty query list, which the library
    answers before any device work: what the plain loop adds per query on top of
    the library itself."""
    from .workloads import paths_from_lists
    hp = mrv.HostPaths(paths_from_lists([], dof_stride))
    ctx.mv(handle, -1, hp, 0)
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.mv(handle, -1, hp, 0)
    return (time.perf_counter() - t0) / reps * 1e6
