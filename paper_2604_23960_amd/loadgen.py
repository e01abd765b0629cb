"""Simulated planner clients for the serving loop (mrv_submit / mrv_wait) and for
the plain one-call-per-query form.

Every request is one MV or FFC query of one client's resident team.  Arrivals
follow a Poisson process of total rate ``rate`` (requests/s; ``inf`` = all at
once).  Latency = completion time - arrival time, so queueing delay counts.
"""
from __future__ import annotations

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
    span = max(t_last - t_first, 1e-9)
    return dict(queries=int(len(lat)), seconds=span, qps=len(lat) / span, states_per_s=states / span,
                p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(np.percentile(lat, 99) * 1e3),
                mean_ms=float(lat.mean() * 1e3))


def prepare(reqs):
    """Host descriptors built once so the timed loops only marshal pointers."""
    return [mrv.HostPaths(r.paths) for r in reqs]


def run_served(ctx: mrv.Context, handles, env: int, reqs, hps, rate: float, seed: int = 0,
               flags_mv: int = mrv.CHECK_ENV, flags_ffc: int = 0):
    n = len(reqs)
    arr = arrival_times(n, rate, seed)
    tickets = [0] * n
    arrive = np.zeros(n)
    done = np.zeros(n)
    results = [None] * n
    ready = threading.Semaphore(0)
    t0 = time.perf_counter() + 0.01

    def submitter():
        for i, r in enumerate(reqs):
            _sleep_until(t0 + arr[i])
            arrive[i] = t0 + arr[i]
            while True:
                try:
                    tickets[i] = ctx.submit(r.kind, handles[r.client], env if r.kind == 0 else -1, hps[i],
                                            flags_mv if r.kind == 0 else flags_ffc)
                    break
                except mrv.MrvError as e:
                    if e.status != mrv.MRV_E_BUSY:
                        raise
                    time.sleep(50e-6)
            ready.release()

    th = threading.Thread(target=submitter)
    th.start()
    for i, r in enumerate(reqs):
        ready.acquire()
        results[i] = ctx.poll(tickets[i], r.kind, 1, timeout_ms=None)
        done[i] = time.perf_counter()
    th.join()
    lat = done - arrive
    states = float(sum(r.horizon * len(r.paths.wp_begin[:-1]) // max(r.paths.n_queries, 1) for r in reqs))
    return summarize(lat, arrive.min(), done.max(), states), results


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
    states = float(sum(r.horizon * len(r.paths.wp_begin[:-1]) // max(r.paths.n_queries, 1) for r in reqs))
    return summarize(lat, arrive.min(), done.max(), states), results
