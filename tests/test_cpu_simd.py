"""The CPU SIMD baseline in the paper's style (rake, W = 8, FP32; baseline_cpu)
against the FP64 oracle on the arm workload (with and without obstacles, early
exit and exhaustive), the disk workload and an 8-arm ring team.  These inputs
hold no test within FP32 rounding of contact, so the answers must be equal."""
import numpy as np
import pytest

import baseline_cpu as B
import oracle
from paper_2604_23960_amd import workloads as W


@pytest.fixture(scope="module")
def arms():
    return W.arms_workload(768)


@pytest.mark.parametrize("check_env", [True, False])
@pytest.mark.parametrize("exhaustive", [False, True])
def test_arms(arms, check_env, exhaustive):
    w = arms
    sub = w.paths
    ref = oracle.mv(oracle.Team(w.team), oracle.Env(w.env), oracle.Paths(sub), check_env=check_env)
    got, states = B.mv(w.team, w.env, sub, check_env, exhaustive)
    assert np.array_equal(got, ref)
    T = sub.horizon()
    if exhaustive:
        assert states == int(T.sum()) * len(w.team)
    if not check_env:
        assert 0 < ref.sum() < len(ref)


def test_disks():
    w = W.disks_workload(2048)
    ref = oracle.mv(oracle.Team(w.team), oracle.Env(w.env), oracle.Paths(w.paths))
    got, _ = B.mv(w.team, w.env, w.paths)
    assert np.array_equal(got, ref) and 0 < ref.sum() < len(ref)


def test_ring_of_eight_without_obstacles():
    team = W.ring_team(8)
    rng = np.random.default_rng(5)
    s = W.sample_configs(rng, team, 256, 7)
    g = W.sample_configs(rng, team, 256, 7)
    paths = W.straight_line_paths(s, g, [r.dof for r in team], 1.0 / 32, "linf", 7)
    ref = oracle.mv(oracle.Team(team), None, oracle.Paths(paths), check_env=False)
    got, _ = B.mv(team, None, paths, check_env=False)
    assert np.array_equal(got, ref)


def test_point_clouds_rejected():
    w = W.arms_workload(4)
    env = W.Env(points=np.zeros((3, 3)), point_radius=0.01)
    with pytest.raises(ValueError):
        B.mv(w.team, env, w.paths)
