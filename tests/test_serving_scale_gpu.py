"""GPU parity of the serving loop at the scale of the serving workload: 64
simulated planner clients with resident teams of 2-8 robots (arm models on
distinct corners plus SE(2) rectangles), motion lengths log-uniform over 8-4,096
timesteps, 70 % MV (Alg. 1) and 30 % FFC (Alg. 2), submitted through
mrv_submit and collected through mrv_wait while earlier requests still run, so
batches of many teams and both kinds overlap on the device.  Every answer is
compared element by element with the FP64 oracle, and a sample is served again
alone and must give the same answer."""
import time
from collections import defaultdict

import numpy as np
import pytest

import oracle
from paper_2604_23960_amd import loadgen
from paper_2604_23960_amd import mrv
from paper_2604_23960_amd import workloads as W

pytestmark = pytest.mark.gpu

N_REQUESTS = 4000


def say(*a):
    print("[case]", *a, flush=True)


MV_FLAGS = [mrv.CHECK_ENV, mrv.CHECK_ENV | mrv.EXHAUSTIVE, mrv.CHECK_ENV | mrv.ORDER_RAKE,
            mrv.CHECK_ENV | mrv.HIERARCHICAL, 0]
FFC_FLAGS = [0, mrv.EXHAUSTIVE]


def oracle_answers(teams, env, reqs, flags):
    """The oracle on every request, batched per (client, kind, environment use)."""
    groups = defaultdict(list)
    for i, r in enumerate(reqs):
        groups[(r.client, r.kind, bool(flags[i] & mrv.CHECK_ENV))].append(i)
    oe = oracle.Env(env)
    out = [None] * len(reqs)
    for (client, kind, use_env), idx in groups.items():
        team = teams[client]
        p = W.paths_from_lists([[reqs[i].paths.path(0, r) for r in range(len(team))] for i in idx], 7)
        ot, op = oracle.Team(team), oracle.Paths(p)
        res = oracle.mv(ot, oe, op, check_env=use_env) if kind == 0 else oracle.ffc(ot, op)
        for k, i in enumerate(idx):
            out[i] = res[k:k + 1]
    return out


def test_serving_workload_scale_matches_oracle():
    teams, env, reqs = W.serving_workload(N_REQUESTS)
    assert len(teams) == 64 and max(r.horizon for r in reqs) > 3000
    rng = np.random.default_rng(33)
    flags = [int(MV_FLAGS[rng.integers(len(MV_FLAGS))]) if r.kind == 0 else int(FFC_FLAGS[rng.integers(2)])
             for r in reqs]
    t0 = time.perf_counter()
    ref = oracle_answers(teams, env, reqs, flags)
    say(f"oracle answers for {len(reqs)} requests in {time.perf_counter() - t0:.1f} s")
    ctx = mrv.Context(0, max_inflight=2 * N_REQUESTS)
    try:
        handles = [ctx.load_team(t) for t in teams]
        e = ctx.load_env(env)
        hps = loadgen.prepare(reqs)
        # the whole set in flight at once: submit everything, then collect
        say("serving", len(reqs), "requests of 64 clients, all in flight")
        tickets = [ctx.submit(r.kind, handles[r.client], e if r.kind == 0 else -1, hps[i], flags[i])
                   for i, r in enumerate(reqs)]
        mixed = [ctx.poll(t, r.kind, 1, timeout_ms=None) for t, r in zip(tickets, reqs)]
        bad = [i for i in range(len(reqs)) if not np.array_equal(mixed[i], ref[i])]
        assert not bad, [(i, reqs[i].kind, flags[i], mixed[i], ref[i]) for i in bad[:5]]
        # Poisson arrivals at a rate the loop sustains, collected as they finish
        say("serving with Poisson arrivals")
        sub = list(range(0, len(reqs), 2))
        s, res = loadgen.run_served(ctx, handles, e, [reqs[i] for i in sub], [hps[i] for i in sub], rate=20000.0)
        # run_served sends MV with environment checks and FFC without flags: compare
        # where the oracle answer above was taken with the same checks
        n_cmp = 0
        for k, i in enumerate(sub):
            if reqs[i].kind == 1:
                assert np.array_equal(np.asarray(res[k]).reshape(-1, 3), ref[i]), i
                n_cmp += 1
            elif flags[i] & mrv.CHECK_ENV:
                assert np.array_equal(np.asarray(res[k]).reshape(-1), ref[i]), i
                n_cmp += 1
        assert n_cmp > len(sub) // 2
        assert s["queries"] == len(sub)
        # alone: one request in flight at a time
        say("serving 200 requests alone")
        for i in range(0, len(reqs), len(reqs) // 200):
            r = reqs[i]
            t = ctx.submit(r.kind, handles[r.client], e if r.kind == 0 else -1, hps[i], flags[i])
            assert np.array_equal(ctx.poll(t, r.kind, 1, timeout_ms=None), mixed[i]), i
    finally:
        ctx.close()
