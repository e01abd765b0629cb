"""The planner driver with edge checks served on the GPU: every served MV
answer equals the FP64 oracle's on the same edges, so the plan is the same as
with oracle edge checks, and every edge of the path is valid in FP64."""
import numpy as np
import pytest

from paper_2604_23960_amd import mrv, planner

from test_planner import OracleChecker

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


@pytest.mark.parametrize("seed", [1, 2, 6])
def test_served_plan_matches_oracle_plan(seed):
    team, env = planner.two_arm_problem()
    ref_check = OracleChecker(team, env)
    with mrv.Context(0) as ctx:
        th, eh = ctx.load_team(team), ctx.load_env(env)
        check = planner.ServedChecker(ctx, th, eh, team, log=True)
        say("plan seed", seed)
        rng = np.random.default_rng(seed)
        start, goal = planner.sample_free_pair(check, team, rng)
        res = planner.rrt_connect(check, team, start, goal, rng, batch=32, max_step=0.5, max_iters=150)
    for a, b, ok in check.log:
        assert np.array_equal(ok, ref_check(a, b))
    rng = np.random.default_rng(seed)
    s2, g2 = planner.sample_free_pair(ref_check, team, rng)
    ref = planner.rrt_connect(ref_check, team, s2, g2, rng, batch=32, max_step=0.5, max_iters=150)
    assert res.path is not None and ref.path is not None
    assert res.iterations == ref.iterations and len(res.path) == len(ref.path)
    assert all(np.array_equal(x, y) for x, y in zip(res.path, ref.path))
    assert ref_check(np.stack(res.path[:-1]), np.stack(res.path[1:])).all()
