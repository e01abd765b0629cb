"""GPU tests of the serving loop: results in the mix equal results alone and the
oracle's; error paths (busy, cancel, handle in use) behave."""
import time

import numpy as np
import pytest

import oracle
from paper_2604_23960_amd import loadgen
from paper_2604_23960_amd import mrv
from paper_2604_23960_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def served():
    teams, env, reqs = W.serving_workload(240, n_clients=6, t_hi=384)
    ctx = mrv.Context(0)
    handles = [ctx.load_team(t) for t in teams]
    e = ctx.load_env(env)
    yield ctx, teams, env, reqs, handles, e
    ctx.close()


def flags_of(r):
    return mrv.CHECK_ENV if r.kind == 0 else 0


def test_mix_equals_alone_equals_oracle(served):
    ctx, teams, env, reqs, handles, e = served
    say("serving mix vs alone", len(reqs))
    hps = loadgen.prepare(reqs)
    tickets = [ctx.submit(r.kind, handles[r.client], e if r.kind == 0 else -1, hps[i], flags_of(r))
               for i, r in enumerate(reqs)]
    mixed = [ctx.poll(t, r.kind, 1, timeout_ms=None) for t, r in zip(tickets, reqs)]
    alone = []
    for i, r in enumerate(reqs):
        t = ctx.submit(r.kind, handles[r.client], e if r.kind == 0 else -1, hps[i], flags_of(r))
        alone.append(ctx.poll(t, r.kind, 1, timeout_ms=None))
    for m, a in zip(mixed, alone):
        assert np.array_equal(m, a)
    oe = oracle.Env(env)
    n_checked = 0
    for i, r in enumerate(reqs):
        ot = oracle.Team(teams[r.client])
        op = oracle.Paths(r.paths)
        if r.kind == 0:
            ref = oracle.mv(ot, oe, op)
            assert np.array_equal(mixed[i], ref), i
        else:
            ref = oracle.ffc(ot, op)
            assert np.array_equal(mixed[i], ref), i
        n_checked += 1
    assert n_checked == len(reqs)
    # the plain synchronous form answers the same
    for i, r in enumerate(reqs[:40]):
        got = ctx.mv(handles[r.client], e, hps[i], mrv.CHECK_ENV) if r.kind == 0 else ctx.ffc(handles[r.client], hps[i])
        assert np.array_equal(got, mixed[i])


def test_poisson_load_and_latency_report(served):
    ctx, teams, env, reqs, handles, e = served
    say("poisson load")
    hps = loadgen.prepare(reqs)
    s, res = loadgen.run_served(ctx, handles, e, reqs, hps, rate=2000.0)
    assert s["queries"] == len(reqs) and s["p99_ms"] >= s["p50_ms"] > 0
    p, res2 = loadgen.run_plain(ctx, handles, e, reqs[:60], hps[:60], rate=float("inf"))
    for a, b in zip(res[:60], res2):
        assert np.array_equal(a, b)


def test_busy_cancel_and_handles(served):
    say("busy / cancel / unload")
    w = W.arms_workload(20000)
    big = mrv.HostPaths(w.paths)
    ex_flags = mrv.CHECK_ENV | mrv.EXHAUSTIVE
    # a full queue answers BUSY; a team in use cannot be unloaded
    ctx = mrv.Context(0, max_inflight=2)
    try:
        team = ctx.load_team(w.team)
        env = ctx.load_env(w.env)
        t1 = ctx.submit(0, team, env, big, ex_flags)
        t2 = ctx.submit(0, team, env, big, ex_flags)
        with pytest.raises(mrv.MrvError) as ex:
            ctx.submit(0, team, env, big, mrv.CHECK_ENV)
        assert ex.value.status == mrv.MRV_E_BUSY
        with pytest.raises(mrv.MrvError) as ex:
            ctx.unload(team)
        assert ex.value.status == mrv.MRV_E_BUSY
        r1 = ctx.poll(t1, 0, w.paths.n_queries, timeout_ms=None)
        r2 = ctx.poll(t2, 0, w.paths.n_queries, timeout_ms=None)
        assert np.array_equal(r1, r2)
        with pytest.raises(mrv.MrvError) as ex:
            ctx.poll(t1, 0, 1)
        assert ex.value.status == mrv.MRV_E_HANDLE
        # a short wait on a long request reports the timeout; the request still completes
        t3 = ctx.submit(0, team, env, big, ex_flags)
        with pytest.raises(mrv.MrvError) as ex:
            ctx.poll(t3, 0, w.paths.n_queries, timeout_ms=1)
        assert ex.value.status == mrv.MRV_E_TIMEOUT
        assert np.array_equal(ctx.poll(t3, 0, w.paths.n_queries, timeout_ms=None), r1)
        ctx.unload(team)    # nothing in flight any more
    finally:
        ctx.close()
    # cancelling a request that still waits for a slot: four requests with flags that
    # cannot share a batch occupy the four slots, the fifth waits and is cancelled
    ctx = mrv.Context(0, max_inflight=8)
    try:
        team = ctx.load_team(w.team)
        env = ctx.load_env(w.env)
        flag_sets = [ex_flags, mrv.EXHAUSTIVE, ex_flags | mrv.HIERARCHICAL, ex_flags | mrv.ORDER_RAKE,
                     ex_flags | mrv.ORDER_LINEAR]
        tickets = [ctx.submit(0, team, env, big, f) for f in flag_sets]
        ctx.cancel(tickets[-1])
        outs = [ctx.poll(t, 0, w.paths.n_queries, timeout_ms=None) for t in tickets[:-1]]
        with pytest.raises(mrv.MrvError) as ex:
            ctx.poll(tickets[-1], 0, w.paths.n_queries, timeout_ms=None)
        assert ex.value.status == mrv.MRV_E_CANCELLED
        direct = ctx.mv(team, env, big, ex_flags)
        for f, o in zip(flag_sets, outs):
            exp = direct if f & mrv.CHECK_ENV else ctx.mv(team, env, big, f)
            assert np.array_equal(o, exp), f
        with pytest.raises(mrv.MrvError) as ex:
            ctx.cancel(tickets[-1])
        assert ex.value.status == mrv.MRV_E_HANDLE
    finally:
        ctx.close()
