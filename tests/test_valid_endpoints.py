"""Valid-endpoint motions (the valid-endpoint protocol of the paper's experiments,
§IV-A): workloads.valid_configs keeps configurations valid for each robot alone,
then for the team; the validity test is passed in, so the generator holds no
collision arithmetic.  On the CPU the oracle decides and every endpoint is
checked against it; on the GPU the library decides (as bench.py does) and the
generated motions must equal the oracle-decided ones exactly, since both take
the same decisions on the same seeded candidates."""
import numpy as np
import pytest

import oracle
from paper_2604_23960_amd import workloads as W


def oracle_decide(robots, env, cfg):
    one = W.straight_line_paths(cfg, cfg, [r.dof for r in robots], 1.0, "linf", cfg.shape[2])
    return oracle.mv(oracle.Team(robots), oracle.Env(env), oracle.Paths(one)).astype(bool)


def endpoints(paths):
    """Start and goal configuration of each query, [Q, n_robots, dof_stride] each."""
    nr = paths.n_robots
    b = paths.wp_begin
    first = paths.wp_q[b[:-1]].reshape(paths.n_queries, nr, -1)
    last = paths.wp_q[b[1:] - 1].reshape(paths.n_queries, nr, -1)
    return first, last


@pytest.mark.parametrize("make", [W.arms_workload, W.disks_workload])
def test_endpoints_valid_alone_and_as_team(make):
    w = make(300, decide=oracle_decide)
    assert "valid endpoints" in w.notes
    s, g = endpoints(w.paths)
    for cfg in (s, g):
        assert oracle_decide(w.team, w.env, cfg).all()
        for r, rob in enumerate(w.team):
            assert oracle_decide([rob], w.env, cfg[:, r:r + 1, :]).all()
    # seeded: the same workload again
    w2 = make(300, decide=oracle_decide)
    assert np.array_equal(w.paths.wp_q, w2.paths.wp_q) and np.array_equal(w.paths.wp_t, w2.paths.wp_t)


def test_rejection_is_real():
    # without the decider a sizeable share of the arm endpoints collide
    w = W.arms_workload(300)
    s, _ = endpoints(w.paths)
    assert oracle_decide(w.team, w.env, s).mean() < 0.5


def test_decider_sees_every_candidate_batch():
    calls = []

    def spy(robots, env, cfg):
        calls.append((len(robots), len(cfg)))
        return oracle_decide(robots, env, cfg)
    W.disks_workload(64, decide=spy)
    assert calls[0] == (1, 8192) and calls[1] == (1, 8192) and calls[2][0] == 2


@pytest.mark.gpu
def test_library_decisions_equal_oracle_decisions():
    import bench
    from paper_2604_23960_amd import mrv
    ctx = mrv.Context(0)
    try:
        decide, release = bench.library_decider(ctx)
        for make, n in ((W.arms_workload, 2000), (W.disks_workload, 2000)):
            print("[case] library-decided endpoints", make.__name__, n, flush=True)
            a = make(n, decide=decide)
            b = make(n, decide=oracle_decide)
            assert np.array_equal(a.paths.wp_q, b.paths.wp_q) and np.array_equal(a.paths.wp_t, b.paths.wp_t)
            assert a.notes == b.notes
        release()
    finally:
        ctx.close()
