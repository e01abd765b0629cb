"""Parity at the full sizes of the benchmark workloads, in the launch configuration
bench.py times (device-resident paths, default tilings): every query against the
FP64 oracle (the early-exit oracle covers these batches in seconds), plus
properties that hold at any size.  Arm MV: 65,536 motions; FFC on arms +
rectangles: 16,384 path sets; 16-robot team in the 200k-point cloud: 131,072 MV
and 131,072 FFC queries."""
import numpy as np
import pytest
import torch

import oracle
from paper_2604_23960_amd import mrv
from paper_2604_23960_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = mrv.Context(0)
    yield c
    c.close()


def mv_dev(ctx, team, env, dp, n, flags):
    out = torch.full((n,), 7, dtype=torch.uint8, device="cuda")
    ctx.mv_device(team, env, dp, flags, out.data_ptr())
    ctx.sync()
    return out.cpu().numpy()


def ffc_dev(ctx, team, dp, n, flags=0):
    out = torch.full((n, 3), 7, dtype=torch.int32, device="cuda")
    ctx.ffc_device(team, dp, flags, out.data_ptr())
    ctx.sync()
    return out.cpu().numpy()


def test_arms_65536(ctx):
    w = W.arms_workload(65536)
    n = w.paths.n_queries
    ot, oe, op = oracle.Team(w.team), oracle.Env(w.env), oracle.Paths(w.paths)
    team, env = ctx.load_team(w.team), ctx.load_env(w.env)
    dp = mrv.DevicePaths(w.paths)
    say("arms 65536: exhaustive and early-exit MV with obstacles")
    ref = oracle.mv(ot, oe, op, check_env=True)
    assert np.array_equal(mv_dev(ctx, team, env, dp, n, mrv.CHECK_ENV | mrv.EXHAUSTIVE), ref)
    assert np.array_equal(mv_dev(ctx, team, env, dp, n, mrv.CHECK_ENV), ref)
    say("arms 65536: MV without obstacles (robot-robot only)")
    ref0 = oracle.mv(ot, oe, op, check_env=False)
    assert 0 < ref0.sum() < n
    got0 = mv_dev(ctx, team, env, dp, n, 0)
    assert np.array_equal(got0, ref0), np.flatnonzero(got0 != ref0)[:10]
    assert np.array_equal(mv_dev(ctx, team, env, dp, n, mrv.EXHAUSTIVE), ref0)
    say("arms 65536: FFC null iff MV without obstacles is valid; sampled FFC")
    f = ffc_dev(ctx, team, dp, n)
    assert np.array_equal(f[:, 0] < 0, got0.astype(bool))
    idx = np.sort(np.random.default_rng(11).choice(n, 512, replace=False))
    assert np.array_equal(f[idx], oracle.ffc(ot, oracle.Paths(w.paths.subset(idx))))
    ctx.unload(team)
    ctx.unload(env)


def test_ffc_16384(ctx):
    w = W.ffc_workload(16384)
    n = w.paths.n_queries
    ot, op = oracle.Team(w.team), oracle.Paths(w.paths)
    team = ctx.load_team(w.team)
    dp = mrv.DevicePaths(w.paths)
    say("arms + rectangles 16384: FFC, early and exhaustive")
    ref = oracle.ffc(ot, op)
    got = ffc_dev(ctx, team, dp, n)
    assert np.array_equal(got, ref), np.flatnonzero(np.any(got != ref, axis=1))[:10]
    assert np.array_equal(ffc_dev(ctx, team, dp, n, mrv.EXHAUSTIVE), ref)
    ctx.unload(team)


def test_cloud_262144(ctx):
    team_d, env_d, mvp, ffcp = W.big_hetero_workload(262_144)
    ot, oe = oracle.Team(team_d), oracle.Env(env_d)
    team, env = ctx.load_team(team_d), ctx.load_env(env_d)
    say("cloud: 131072 MV queries")
    dmv = mrv.DevicePaths(mvp)
    ref = oracle.mv(ot, oe, oracle.Paths(mvp))
    assert np.array_equal(mv_dev(ctx, team, env, dmv, mvp.n_queries, mrv.CHECK_ENV), ref)
    say("cloud: 131072 FFC queries")
    dffc = mrv.DevicePaths(ffcp)
    fref = oracle.ffc(ot, oracle.Paths(ffcp))
    got = ffc_dev(ctx, team, dffc, ffcp.n_queries)
    assert np.array_equal(got, fref), np.flatnonzero(np.any(got != fref, axis=1))[:10]
    say("cloud: exhaustive MV on the first 8192 motions")
    sub = mvp.subset(np.arange(8192))
    assert np.array_equal(mv_dev(ctx, team, env, mrv.DevicePaths(sub), 8192, mrv.CHECK_ENV | mrv.EXHAUSTIVE),
                          ref[:8192])
    ctx.unload(team)
    ctx.unload(env)
