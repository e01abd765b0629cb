"""GPU check of the precision argument: the FP32 sphere centres the kernels start
from stay within a small fraction of the near-contact band (1e-5 m) of the FP64
oracle's, on every workload's team, so a clearance off by less than twice the
centre error can never cross zero unnoticed."""
import numpy as np
import pytest

import oracle
from paper_2604_23960_amd import mrv
from paper_2604_23960_amd import workloads as W

pytestmark = pytest.mark.gpu

EPS = 1e-5


def say(*a):
    print("[case]", *a, flush=True)


def centre_errors(ctx, team, paths, n_states=1500, seed=0):
    rng = np.random.default_rng(seed)
    T = paths.horizon()
    q = rng.integers(0, paths.n_queries, n_states)
    t = (rng.random(n_states) * T[q]).astype(np.int64)
    th = ctx.load_team(team)
    ot, op = oracle.Team(team), oracle.Paths(paths)
    got = ctx.spheres(th, paths, q, t, ot.total_spheres).astype(np.float64)
    err = []
    for k in range(n_states):
        ref = oracle.team_spheres(ot, op, int(q[k]), int(t[k]))
        assert np.array_equal(got[k, :, 3], ref[:, 3].astype(np.float32).astype(np.float64))
        err.append(np.linalg.norm(got[k, :, :3] - ref[:, :3], axis=1))
    return np.concatenate(err)


@pytest.mark.parametrize("name", ["disks", "arms", "arms_rects", "cloud_team"])
def test_fp32_centre_error_within_band(name):
    say("fp32 centre error", name)
    if name == "disks":
        w = W.disks_workload(512)
        team, paths = w.team, w.paths
    elif name == "arms":
        w = W.arms_workload(512)
        team, paths = w.team, w.paths
    elif name == "arms_rects":
        w = W.ffc_workload(128)
        team, paths = w.team, w.paths
    else:
        team, env, mv, ffc = W.big_hetero_workload(256)
        paths = ffc
    ctx = mrv.Context(0)
    try:
        e = centre_errors(ctx, team, paths)
    finally:
        ctx.close()
    q = np.quantile(e, [0.5, 0.99, 1.0])
    print(f"[fp32-centre-error] {name}: median {q[0]:.3e} m, p99 {q[1]:.3e} m, max {q[2]:.3e} m", flush=True)
    # clearance error <= 2 x centre error + obstacle/test rounding (< 1e-6 m)
    assert q[2] <= EPS / 5
