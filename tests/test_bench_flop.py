"""bench.py's FLOP figure counts executed tests: with the counters of a full
scan of the four-arm workload it gives the per-timestep total of a full scan
(4 arms x 60 spheres, 20 boxes + 8 cylinders, 2,918 self pairs: 425,060 FLOP
per timestep of the team: 216,000 robot-robot, 174,720 obstacle, 29,180 self,
5,160 FK and placement), culled obstacle tests drop out of it, and the split
puts robot-robot, self and sphere-point tests on the matrix cores, the rest on
the vector unit; sphere-point tests count 10 each."""
import bench
from paper_2604_23960_amd import workloads as W


def test_full_scan_counts_give_the_per_timestep_total():
    w = W.arms_workload(8)
    ts = 1000
    n_self = sum(len(r.self_pairs) for r in w.team)
    assert n_self == 2918
    full = dict(states_evaluated=4 * ts, rr_tests=6 * 60 * 60 * ts, self_tests=n_self * ts,
                env_tests=4 * 60 * 28 * ts)
    f = bench.executed_flop(w.team, w.env, full)
    assert f["total"] == ts * 425_060
    assert f["mfma"] == ts * (216_000 + 29_180) and f["valu"] == ts * (174_720 + 5_160)
    culled = dict(full, env_tests=full["env_tests"] // 10)
    drop = (full["env_tests"] - culled["env_tests"]) * bench.FLOP_SPHERE_BOX
    assert bench.executed_flop(w.team, w.env, culled)["total"] == ts * 425_060 - drop
    pts = dict(full, point_tests=777)
    fp = bench.executed_flop(w.team, w.env, pts)
    assert fp["mfma"] == f["mfma"] + 7770 and fp["valu"] == f["valu"]
