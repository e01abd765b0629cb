"""GPU parity on the 16-robot heterogeneous team with the 200k-point obstacle
cloud (points on 40 box surfaces, uniform grid on the device, k-d tree in the
oracle), with and without focus sets; on a single arm inside the cloud where
only the cloud and self collisions decide; and on a cloud of three points,
whose blocks read into the padding past the cloud's end, in host and served
forms."""
import numpy as np
import pytest

import oracle
from paper_2604_23960_amd import mrv
from paper_2604_23960_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def big():
    team, env, mv, ffc = W.big_hetero_workload(768)
    return team, env, mv, ffc, oracle.Team(team), oracle.Env(env)


def test_hetero_cloud_mv_ffc(big):
    team, env, mv, ffc, ot, oe = big
    say("16-robot cloud MV/FFC")
    ctx = mrv.Context(0)
    try:
        th, eh = ctx.load_team(team), ctx.load_env(env)
        ref = oracle.mv(ot, oe, oracle.Paths(mv))
        for flags in (mrv.CHECK_ENV, mrv.CHECK_ENV | mrv.OBSTACLES_FIRST, mrv.CHECK_ENV | mrv.EXHAUSTIVE, 0):
            got = ctx.mv(th, eh, mv, flags)
            exp = ref if flags & mrv.CHECK_ENV else oracle.mv(ot, oe, oracle.Paths(mv), check_env=False)
            assert np.array_equal(got, exp), (flags, np.nonzero(got != exp)[0][:10])
        fref = oracle.ffc(ot, oracle.Paths(ffc))
        got = ctx.ffc(th, ffc)
        assert np.array_equal(got, fref), np.nonzero(np.any(got != fref, axis=1))[0][:10]
    finally:
        ctx.close()


def test_single_arm_in_cloud():
    say("single arm in cloud")
    team = [W.arm_models(1)[0].with_base(W.arm_base(0.5, 0.5))]
    env = W.box_surface_cloud(4, n_points=200_000)
    rng = np.random.default_rng([9, 3])
    paths = W.straight_line_paths_T(rng, team, rng.integers(16, 300, 512), 7)
    ot, oe = oracle.Team(team), oracle.Env(env)
    ref = oracle.mv(ot, oe, oracle.Paths(paths))
    assert 0 < ref.sum() < len(ref)
    ctx = mrv.Context(0)
    try:
        th, eh = ctx.load_team(team), ctx.load_env(env)
        for flags in (mrv.CHECK_ENV, mrv.CHECK_ENV | mrv.PAIRS_FIRST, mrv.CHECK_ENV | mrv.EXHAUSTIVE,
                      mrv.CHECK_ENV | mrv.HIERARCHICAL):
            got = ctx.mv(th, eh, paths, flags)
            assert np.array_equal(got, ref), (flags, np.nonzero(got != ref)[0][:10])
    finally:
        ctx.close()


@pytest.mark.parametrize("focus", [0x0001, 0x0010, 0x0100, 0x00F0])
def test_cloud_team_focus(big, focus):
    """Prioritised MV with the point cloud (the focus kernels' point-cloud builds):
    one floor arm, one ceiling arm, one rectangle, the ceiling arms; short motions,
    so that the cloud decides many answers; early-terminating in both phase
    orders and exhaustive."""
    team, env, mv, ffc, ot, oe = big
    rng = np.random.default_rng([9, 8])
    paths = W.straight_line_paths_T(rng, team, rng.integers(1, 12, 256), 7)
    ref = oracle.mv(ot, oe, oracle.Paths(paths), check_env=True, focus=focus)
    ctx = mrv.Context(0)
    try:
        th, eh = ctx.load_team(team), ctx.load_env(env)
        for flags in (mrv.CHECK_ENV, mrv.CHECK_ENV | mrv.OBSTACLES_FIRST, mrv.CHECK_ENV | mrv.EXHAUSTIVE):
            say("cloud focus", hex(focus), "flags", flags)
            got = ctx.mv(th, eh, paths, flags, focus=focus)
            assert np.array_equal(got, ref), (focus, flags, np.nonzero(got != ref)[0][:10])
    finally:
        ctx.close()


def test_tiny_cloud_and_served_form():
    """Three points, each at a sphere centre of an arm's state on some motion: the
    sphere-point blocks read past the cloud's end into its padding, and the points
    decide most answers.  Host, exhaustive and served forms equal the oracle."""
    say("tiny cloud")
    team = [W.arm_models(1)[0].with_base(W.arm_base(0.5, 0.5))]
    rng = np.random.default_rng([9, 7])
    paths = W.straight_line_paths_T(rng, team, rng.integers(16, 200, 384), 7)
    ot, op = oracle.Team(team), oracle.Paths(paths)
    centres = []
    for qi in (3, 17, 101):
        s = oracle.team_spheres(ot, op, qi, oracle.horizon(op, qi) // 2)
        centres.append(s[len(s) - 5, :3])
    env = W.Env(points=np.array(centres), point_radius=0.02)
    oe = oracle.Env(env)
    ref = oracle.mv(ot, oe, op)
    free = oracle.mv(ot, oracle.Env(W.Env()), op)
    assert 0 < ref.sum() < len(ref) and (ref != free).sum() > len(ref) // 4
    ctx = mrv.Context(0)
    try:
        th, eh = ctx.load_team(team), ctx.load_env(env)
        for flags in (mrv.CHECK_ENV, mrv.CHECK_ENV | mrv.EXHAUSTIVE, mrv.CHECK_ENV | mrv.OBSTACLES_FIRST):
            got = ctx.mv(th, eh, paths, flags)
            assert np.array_equal(got, ref), (flags, np.nonzero(got != ref)[0][:10])
        hps = [mrv.HostPaths(paths.subset(np.array([i]))) for i in range(64)]
        tickets = [ctx.submit(0, th, eh, hp, mrv.CHECK_ENV) for hp in hps]
        served = np.concatenate([ctx.poll(t, 0, 1, timeout_ms=None) for t in tickets])
        assert np.array_equal(served, ref[:64])
    finally:
        ctx.close()
