"""Planner driver logic on the CPU: Composite RRT-Connect with an edge check
that the test supplies from the FP64 oracle (the product driver checks edges
with MV requests on the GPU).  Found paths must start and end at the given
states and every edge must be valid when re-checked; a colliding goal fails at
once."""
import numpy as np

import oracle
from paper_2604_23960_amd import planner
from paper_2604_23960_amd import workloads as W


class OracleChecker:
    def __init__(self, team, env, step=1.0 / 32.0):
        self.ot, self.oe = oracle.Team(team), oracle.Env(env)
        self.dofs = [r.dof for r in team]
        self.step = step
        self.calls = 0

    def __call__(self, a, b):
        self.calls += 1
        p = W.straight_line_paths(a, b, self.dofs, self.step, "linf", 7)
        return oracle.mv(self.ot, self.oe, oracle.Paths(p)).astype(bool)


def _disks():
    team = [W.disk_robot(0.05, f"d{k}") for k in range(2)]
    return team, W.circles_env(0, 12)


def test_rrt_connect_finds_valid_path():
    team, env = _disks()
    check = OracleChecker(team, env)
    rng = np.random.default_rng(4)
    start, goal = planner.sample_free_pair(check, team, rng)
    res = planner.rrt_connect(check, team, start, goal, rng, batch=16, max_step=0.3, max_iters=200)
    assert res.path is not None
    assert np.array_equal(res.path[0], start) and np.array_equal(res.path[-1], goal)
    a = np.stack(res.path[:-1])
    b = np.stack(res.path[1:])
    assert check(a, b).all()
    # tree edges respect the step bound (a two-state path is the direct start-goal edge)
    spans = np.abs(b - a).reshape(len(a), -1).max(axis=1)
    assert len(res.path) == 2 or np.all(spans <= 0.3 + 1e-9)


def test_rrt_connect_rejects_colliding_goal():
    team, env = _disks()
    check = OracleChecker(team, env)
    rng = np.random.default_rng(5)
    start, _ = planner.sample_free_pair(check, team, rng)
    goal = start.copy()
    goal[1] = goal[0]                      # both disks on the same spot
    res = planner.rrt_connect(check, team, start, goal, rng)
    assert res.path is None and res.iterations == 0
