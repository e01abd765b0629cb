"""GPU tests: autotuned tilings and captured call graphs give the same answers
as the eager path and the oracle; graph replays are checked one by one with
eager work between them."""
import numpy as np
import pytest

import oracle
from paper_2604_23960_amd import mrv
from paper_2604_23960_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def test_autotune_keeps_answers():
    say("autotune")
    w = W.arms_workload(512)
    ctx = mrv.Context(0)
    try:
        team, env = ctx.load_team(w.team), ctx.load_env(w.env)
        tuned = ctx.autotune(team, env, 0, w.paths.subset(np.arange(128)), mrv.CHECK_ENV | mrv.EXHAUSTIVE)
        chunk, wg, il, claim = tuned
        assert 1 <= chunk <= 64 and 0 <= wg <= 8 and 0 <= il <= 3 and 0 <= claim <= 16
        got = ctx.get_tiling(team, 0, mrv.EXHAUSTIVE)
        assert got[0] == chunk and got[1] == wg and got[3] == (claim or 4)
        ref = oracle.mv(oracle.Team(w.team), oracle.Env(w.env), oracle.Paths(w.paths))
        assert np.array_equal(ctx.mv(team, env, w.paths, mrv.CHECK_ENV | mrv.EXHAUSTIVE), ref)
        # cached: same answer, no retiming needed
        assert ctx.autotune(team, env, 0, w.paths.subset(np.arange(16)), mrv.CHECK_ENV | mrv.EXHAUSTIVE) == tuned
        # early-terminating MV also searches the interleave
        ctx.autotune(team, env, 0, w.paths.subset(np.arange(128)), mrv.CHECK_ENV)
        assert np.array_equal(ctx.mv(team, env, w.paths, mrv.CHECK_ENV), ref)
        ctx.autotune(team, -1, 1, w.paths.subset(np.arange(64)), 0)
        assert np.array_equal(ctx.ffc(team, w.paths), oracle.ffc(oracle.Team(w.team), oracle.Paths(w.paths)))
    finally:
        ctx.close()


def test_interleaves_and_claim_sizes_keep_answers():
    say("interleaves and claim sizes")
    w = W.arms_workload(384)
    ctx = mrv.Context(0)
    try:
        team, env = ctx.load_team(w.team), ctx.load_env(w.env)
        ot, oe, op = oracle.Team(w.team), oracle.Env(w.env), oracle.Paths(w.paths)
        ref_env, ref_rr = oracle.mv(ot, oe, op), oracle.mv(ot, oe, op, check_env=False)
        ref_ffc = oracle.ffc(ot, op)
        for il in (1, 2, 3):
            for claim in (1, 3, 16):
                for flags in (0, mrv.EXHAUSTIVE):
                    ctx.set_tiling(team, 0, 5, 0, flags, interleave=il, claim=claim)
                    ctx.set_tiling(team, 1, 7, 0, flags, interleave=il, claim=claim)
                    assert ctx.get_tiling(team, 0, flags)[2:] == (il, claim)
                    assert np.array_equal(ctx.mv(team, env, w.paths, mrv.CHECK_ENV | flags), ref_env), (il, claim)
                    assert np.array_equal(ctx.mv(team, env, w.paths, flags), ref_rr), (il, claim)
                    assert np.array_equal(ctx.ffc(team, w.paths, flags), ref_ffc), (il, claim)
        for bad in (dict(interleave=4), dict(claim=17), dict(claim=-1)):
            with pytest.raises(mrv.MrvError):
                ctx.set_tiling(team, 0, 0, 0, 0, **bad)
    finally:
        ctx.close()


def test_graph_replays_match_eager():
    import torch
    say("graph replays")
    w = W.arms_workload(1024)
    ctx = mrv.Context(0)
    try:
        team, env = ctx.load_team(w.team), ctx.load_env(w.env)
        dp = mrv.DevicePaths(w.paths)
        out_g = torch.zeros(w.paths.n_queries, dtype=torch.uint8, device="cuda")
        out_e = torch.zeros(w.paths.n_queries, dtype=torch.uint8, device="cuda")
        g = ctx.graph_create(team, env, 0, dp, mrv.CHECK_ENV, out_g.data_ptr())
        # a graph that was only captured has not run
        assert int(out_g.sum().item()) == 0
        ctx.mv_device(team, env, dp, mrv.CHECK_ENV, out_e.data_ptr())
        ctx.sync()
        eager = out_e.cpu().numpy()
        assert np.array_equal(eager, oracle.mv(oracle.Team(w.team), oracle.Env(w.env), oracle.Paths(w.paths)))
        for rep in range(4):
            out_g.fill_(7)
            torch.cuda.synchronize()
            ctx.graph_launch(g)
            ctx.sync()
            assert np.array_equal(out_g.cpu().numpy(), eager), rep
            # eager work between replays
            ctx.mv_device(team, env, dp, 0, out_e.data_ptr())
            ctx.sync()
        # a graph without environment checks (about a fifth of these motions are
        # valid, so answers differ between path sets): refill its buffers with other
        # queries (same count, no more waypoints than captured) and replay
        dp2 = mrv.DevicePaths(w.paths)
        g2 = ctx.graph_create(team, env, 0, dp2, 0, out_g.data_ptr())
        ctx.graph_launch(g2)
        ctx.sync()
        first = oracle.mv(oracle.Team(w.team), None, oracle.Paths(w.paths), check_env=False)
        assert np.array_equal(out_g.cpu().numpy(), first)
        other = W.arms_workload(1024, seed=9).paths
        assert other.n_queries == w.paths.n_queries
        n_wp = other.wp_t.shape[0]
        assert n_wp <= dp2.wp_t.shape[0]
        dp2.wp_begin.copy_(torch.as_tensor(other.wp_begin))
        dp2.wp_t[:n_wp].copy_(torch.as_tensor(other.wp_t))
        dp2.wp_q[:n_wp].copy_(torch.as_tensor(other.wp_q))
        out_g.fill_(7)
        torch.cuda.synchronize()
        ctx.graph_launch(g2)
        ctx.sync()
        ref = oracle.mv(oracle.Team(w.team), None, oracle.Paths(other), check_env=False)
        assert not np.array_equal(ref, first)        # the refill changes the answers
        assert np.array_equal(out_g.cpu().numpy(), ref)
        ctx.graph_destroy(g2)
        with pytest.raises(mrv.MrvError) as e:
            ctx.unload(team)
        assert e.value.status == mrv.MRV_E_BUSY
        ctx.graph_destroy(g)
        ctx.unload(team)
    finally:
        ctx.close()
