"""Benchmark of the MV/FFC hot path on one MI355X.

Headline: MotionValidation with robot-obstacle, self and robot-robot checks on
the four-arm workload (4 seeded 7-R arms x 60 spheres, 20 boxes + 8 cylinders,
65,536 straight-line motions at 1/32 rad max-joint step), every state evaluated
(exhaustive mode), inputs resident in HBM.  One step = one mrv_mv_device call
over all 65,536 motions.  ``value`` = robot-states validated per second.

Also reported (``extra``): early-exit MV on the same motions, FFC on the
4-arm + 4-rectangle decoupled-path workload (16,384 path sets), the disk
workload, the FP32 roofline of the validation kernel and the FP64 oracle on the
host cores (``cpu_baseline``).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# FLOP per unit of work: add, subtract and multiply count 1, a fused multiply-add 2;
# comparisons, minima and selects count none.
FLOP_SPHERE_SPHERE = 10     # 3 sub, |d|^2 5, (ra+rb)^2 2
FLOP_SPHERE_BOX = 26
FLOP_SPHERE_CYL = 26
FLOP_REV_JOINT = 30         # interpolation 3, translation 9, Rz composition 18
FLOP_PRI_JOINT = 12
FLOP_SPHERE_PLACE = 18
PEAK_FP32_VALU = 157.3e12   # MI355X FP32 vector peak (published)


PROFILE = os.path.join(ROOT, "profiles", "k_validate_mv_arms65536_exhaustive.md")
KERNEL_SRC = os.path.join(ROOT, "paper_2604_23960_amd", "csrc", "mrv_kernels.hip")


def profiled_traffic():
    """HBM bytes per launch from the committed rocprofv3 summary, only while the kernel
    source is the one that was profiled (else None)."""
    import hashlib
    try:
        text = open(PROFILE).read()
    except OSError:
        return None
    want = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    vals = dict(line.split(": ", 1) for line in text.splitlines()
                if line.startswith(("traffic_bytes_per_launch: ", "kernel_source_sha256: ")))
    if vals.get("kernel_source_sha256", "").strip() != want:
        return None
    return float(vals["traffic_bytes_per_launch"])


def executed_flop(team, env, stats):
    """FLOP of one exhaustive MV launch from its executed-test counters: FK and
    sphere placement of every robot-state, 10 per sphere-sphere test (robot-robot,
    self, sphere obstacles), 26 per box or cylinder test actually run (the kernel
    skips those whose world box misses a row of 16 spheres by more than the near
    band; that skip is comparisons only and counts no FLOP)."""
    from paper_2604_23960_amd import workloads as W
    assert FLOP_SPHERE_BOX == FLOP_SPHERE_CYL        # one counter covers both
    ts = stats["states_evaluated"] / len(team)
    fk = 0
    for r in team:
        fk += sum(FLOP_REV_JOINT if jt == W.REV_Z else FLOP_PRI_JOINT for jt in r.joint_type)
        fk += r.n_spheres * FLOP_SPHERE_PLACE
    sph_tests = ts * sum(r.n_spheres for r in team) * len(env.spheres)
    return (ts * fk + (stats["rr_tests"] + stats["self_tests"] + sph_tests) * FLOP_SPHERE_SPHERE +
            (stats["env_tests"] - sph_tests) * FLOP_SPHERE_BOX)


def run_device(ctx, team, env, dp, kind, flags, out, steps, warmup, focus=0):
    import torch
    call = (lambda: ctx.mv_device(team, env, dp, flags, out.data_ptr(), focus)) if kind == 0 else \
        (lambda: ctx.ffc_device(team, dp, flags, out.data_ptr()))
    for _ in range(warmup):
        call()
    ctx.sync()
    torch.cuda.synchronize()
    kernel_ms = []
    stats = None
    t0 = time.perf_counter()
    for _ in range(steps):
        call()
        stats = ctx.last_stats()          # waits for the step; reads the kernel's HIP-event time
        kernel_ms.append(stats["kernel_ms"])
    ctx.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, kernel_ms, stats


def ordering_study(log, n_motions=4096, step=1.0 / 128, max_rounds=64):
    """Early-termination orders on ring teams of 4, 8 and 16 arms, with the arm
    workload's obstacle field inside the ring and without obstacles (self tests
    still on), over random
    straight-line motions whose endpoints are valid (each robot moves at most
    `step` in L2 per timestep, the composite motion time-scaled to the slowest).
    Endpoint validity is decided by this library (MV of single-state motions).
    For every order: kernel time per call, effort (robot-states evaluated per
    robot-state covered) and the valid fraction; exhaustive MV for reference.
    Endpoints are composed from per-robot configurations that are valid alone
    (self and obstacle tests of a one-robot team), then kept if the whole team's
    state is valid."""
    import torch
    from paper_2604_23960_amd import mrv
    from paper_2604_23960_amd import workloads as W
    orders = [("combined-bisect", 0), ("combined-rake", mrv.ORDER_RAKE), ("combined-linear", mrv.ORDER_LINEAR),
              ("hierarchical-bisect", mrv.HIERARCHICAL), ("hierarchical-rake", mrv.HIERARCHICAL | mrv.ORDER_RAKE),
              ("hierarchical-linear", mrv.HIERARCHICAL | mrv.ORDER_LINEAR)]
    ctx = mrv.Context(0)
    rows = []
    for n_arms in (4, 8, 16):
        team = W.ring_team(n_arms)
        th = ctx.load_team(team)
        dofs = [r.dof for r in team]
        for env_name in ("obstacles", "empty"):
            env = W.cube_env(1) if env_name == "obstacles" else W.Env()     # obstacles inside the ring
            eh = ctx.load_env(env)
            rng = np.random.default_rng(1000 + n_arms)
            alone = []
            for rob in team:                     # configurations valid for the robot alone
                h1 = ctx.load_team([rob])
                good = np.zeros((0, 1, 7))
                for _ in range(max_rounds):
                    if len(good) >= 4 * n_motions:
                        break
                    cand = W.sample_configs(rng, [rob], 8192, 7)
                    ok = ctx.mv(h1, eh, W.straight_line_paths(cand, cand, [rob.dof], step, "l2", 7),
                                mrv.CHECK_ENV).astype(bool)
                    good = np.concatenate([good, cand[ok]])
                ctx.unload(h1)
                alone.append(good[:, 0, :])
            pool, tried = [], 0
            if min(len(a) for a in alone) > 0:
                for _ in range(max_rounds):
                    if len(pool) >= 2 * n_motions:
                        break
                    cand = np.stack([a[rng.integers(0, len(a), 8192)] for a in alone], axis=1)
                    one = W.straight_line_paths(cand, cand, dofs, step, "l2", 7)     # single-state motions
                    ok = ctx.mv(th, eh, one, mrv.CHECK_ENV).astype(bool)
                    tried += len(cand)
                    pool.extend(cand[ok])
            m = min(n_motions, len(pool) // 2)
            row = dict(arms=n_arms, env=env_name, motions=m, endpoint_acceptance=len(pool) / max(tried, 1))
            if m == 0:
                log(f"ordering study: {n_arms} arms, {env_name}: no valid endpoints")
                rows.append(row)
                ctx.unload(eh)
                continue
            pool = np.asarray(pool)
            paths = W.straight_line_paths(pool[:m], pool[m:2 * m], dofs, step, "l2", 7)
            row["mean_T"] = float(paths.horizon().mean())
            dp = mrv.DevicePaths(paths)
            out = torch.zeros(m, dtype=torch.uint8, device="cuda")
            for name, fl in orders:
                _, kms, st = run_device(ctx, th, eh, dp, 0, mrv.CHECK_ENV | fl, out, 3, 1)
                row[name] = dict(kernel_ms=float(np.median(kms)),
                                 effort=st["states_evaluated"] / max(st["states_covered"], 1))
            row["valid_fraction"] = float(out.float().mean().item())
            _, kms, st = run_device(ctx, th, eh, dp, 0, mrv.CHECK_ENV | mrv.EXHAUSTIVE, out, 3, 1)
            row["exhaustive"] = dict(kernel_ms=float(np.median(kms)), effort=1.0)
            best = min((n for n, _ in orders), key=lambda n: row[n]["kernel_ms"])
            log(f"ordering study: {n_arms} arms, {env_name}: {m} motions, valid {row['valid_fraction']:.3f}, "
                f"fastest {best} {row[best]['kernel_ms']:.3f} ms, exhaustive {row['exhaustive']['kernel_ms']:.3f} ms")
            rows.append(row)
            ctx.unload(eh)
        ctx.unload(th)
    ctx.close()
    return rows


def serving_bench(log, n_requests=3000, n_plain=400):
    """Served (mrv_submit/mrv_wait, continuous batching) vs plain (one synchronous
    call per query) on 64 simulated clients with resident teams of 2-8 robots."""
    from paper_2604_23960_amd import loadgen, mrv
    from paper_2604_23960_amd import workloads as W
    teams, env, reqs = W.serving_workload(n_requests)
    ctx = mrv.Context(0)
    handles = [ctx.load_team(t) for t in teams]
    e = ctx.load_env(env)
    hps = loadgen.prepare(reqs)
    # warm both forms; the served warm-up uses the whole request set so that the
    # slots' scratch has grown to the batch sizes of the timed runs
    loadgen.run_plain(ctx, handles, e, reqs[:20], hps[:20], float("inf"))
    loadgen.run_served(ctx, handles, e, reqs, hps, float("inf"))
    log("serving: saturation throughput (median of three runs each)")

    def median_run(fn):
        runs = sorted((fn()[0] for _ in range(3)), key=lambda r: r["qps"])
        return runs[1]
    plain_sat = median_run(lambda: loadgen.run_plain(ctx, handles, e, reqs[:n_plain], hps[:n_plain], float("inf")))
    served_sat = median_run(lambda: loadgen.run_served(ctx, handles, e, reqs, hps, float("inf")))
    # the served answers equal the plain ones
    _, res_served = loadgen.run_served(ctx, handles, e, reqs[:n_plain], hps[:n_plain], float("inf"))
    _, res_plain = loadgen.run_plain(ctx, handles, e, reqs[:n_plain], hps[:n_plain], float("inf"))
    same = all(np.array_equal(np.asarray(a).reshape(-1), np.asarray(b).reshape(-1)) for a, b in zip(res_served, res_plain))
    rate = 0.8 * plain_sat["qps"]
    log(f"serving: Poisson load at {rate:.0f} req/s (0.8 x plain saturation) and at 5x that")
    plain_at, _ = loadgen.run_plain(ctx, handles, e, reqs[:n_plain], hps[:n_plain], rate, seed=1)
    served_at, _ = loadgen.run_served(ctx, handles, e, reqs[:n_plain], hps[:n_plain], rate, seed=1)
    n5 = min(len(reqs), 5 * n_plain)
    served_5x, _ = loadgen.run_served(ctx, handles, e, reqs[:n5], hps[:n5], 5 * rate, seed=2)
    ctx.close()
    return dict(clients=len(teams), requests=len(reqs), mv_fraction=float(np.mean([r.kind == 0 for r in reqs])),
                plain_saturated=plain_sat, served_saturated=served_sat,
                offered_rate=rate, plain_at_rate=plain_at, served_at_rate=served_at,
                served_at_5x_rate=served_5x,
                served_over_plain_throughput=served_sat["qps"] / plain_sat["qps"], served_answers_equal_plain=same)


def cloud_bench(log, n_queries=262_144, tune_sample=2048, exhaustive_queries=8192):
    """16-robot team in a 200k-point cloud: early-exit MV and FFC over the whole
    batch, exhaustive MV on a slice, default vs autotuned tiling, and one-launch
    graph replay vs the plain multi-kernel launch for small batches."""
    import torch
    from paper_2604_23960_amd import mrv
    from paper_2604_23960_amd import workloads as W
    team, env, mvp, ffcp = W.big_hetero_workload(n_queries)
    ctx = mrv.Context(0)
    th, eh = ctx.load_team(team), ctx.load_env(env)
    res = dict(queries=n_queries, robots=len(team), spheres=sum(r.n_spheres for r in team),
               points=len(env.points))
    dmv, dffc = mrv.DevicePaths(mvp), mrv.DevicePaths(ffcp)
    o_mv = torch.zeros(mvp.n_queries, dtype=torch.uint8, device="cuda")
    o_ffc = torch.zeros((ffcp.n_queries, 3), dtype=torch.int32, device="cuda")
    sub = mvp.subset(np.arange(exhaustive_queries))
    dsub = mrv.DevicePaths(sub)
    o_sub = torch.zeros(sub.n_queries, dtype=torch.uint8, device="cuda")

    def measure(tag):
        out = {}
        w1, _, s1 = run_device(ctx, th, eh, dmv, 0, mrv.CHECK_ENV, o_mv, 3, 1)
        out["mv_early_exit"] = dict(ms_per_call=w1 / 3 * 1e3, covered_states_per_s=s1["states_covered"] * 3 / w1)
        w2, _, s2 = run_device(ctx, th, -1, dffc, 1, 0, o_ffc, 3, 1)
        out["ffc"] = dict(ms_per_call=w2 / 3 * 1e3, covered_states_per_s=s2["states_covered"] * 3 / w2,
                          evaluated_states_per_s=s2["states_evaluated"] * 3 / w2)
        w3, k3, s3 = run_device(ctx, th, eh, dsub, 0, mrv.CHECK_ENV | mrv.EXHAUSTIVE, o_sub, 2, 1)
        out["mv_exhaustive_slice"] = dict(queries=sub.n_queries, ms_per_call=w3 / 2 * 1e3,
                                          kernel_ms=float(np.mean(k3)),
                                          states_per_s=s3["states_evaluated"] * 2 / w3)
        out["tiling"] = dict(mv_early=ctx.get_tiling(th, 0), mv_exhaustive=ctx.get_tiling(th, 0, mrv.EXHAUSTIVE),
                             ffc=ctx.get_tiling(th, 1))
        log(f"cloud {tag}: {out['mv_exhaustive_slice']['states_per_s']:.3g} states/s exhaustive")
        return out

    res["default_tiling"] = measure("default")
    t0 = time.perf_counter()
    ctx.autotune(th, eh, 0, sub.subset(np.arange(tune_sample)), mrv.CHECK_ENV | mrv.EXHAUSTIVE)
    ctx.autotune(th, -1, 1, ffcp.subset(np.arange(tune_sample)), 0)
    res["autotune_seconds"] = time.perf_counter() - t0
    res["autotuned"] = measure("autotuned")
    # graph replay vs plain launch on small batches
    lat = {}
    for nq in (16, 256):
        small = mvp.subset(np.arange(nq))
        ds = mrv.DevicePaths(small)
        o = torch.zeros(nq, dtype=torch.uint8, device="cuda")
        g = ctx.graph_create(th, eh, 0, ds, mrv.CHECK_ENV, o.data_ptr())
        plain, graph = [], []
        for _ in range(5):
            ctx.mv_device(th, eh, ds, mrv.CHECK_ENV, o.data_ptr())
            ctx.graph_launch(g)
        ctx.sync()
        for _ in range(50):
            t1 = time.perf_counter()
            ctx.mv_device(th, eh, ds, mrv.CHECK_ENV, o.data_ptr())
            ctx.sync()
            plain.append(time.perf_counter() - t1)
            t1 = time.perf_counter()
            ctx.graph_launch(g)
            ctx.sync()
            graph.append(time.perf_counter() - t1)
        ctx.graph_destroy(g)
        lat[str(nq)] = dict(plain_p50_ms=float(np.median(plain) * 1e3), graph_p50_ms=float(np.median(graph) * 1e3),
                            plain_p99_ms=float(np.percentile(plain, 99) * 1e3),
                            graph_p99_ms=float(np.percentile(graph, 99) * 1e3))
    res["graph_vs_plain_launch"] = lat
    ctx.close()
    return res


def simd_baseline(w, value, n_sample=16384):
    """The paper's own design on the host cores (baseline_cpu: rake packing of
    W = 8 timesteps per batch, FP32, early exit; all host threads): exhaustive MV
    on the first n_sample motions and early-exit MV on all of them."""
    import baseline_cpu as B
    sub = w.paths.subset(np.arange(min(n_sample, w.paths.n_queries)))
    B.mv(w.team, w.env, w.paths.subset(np.arange(64)), True, True)          # build and start the threads
    t0 = time.perf_counter()
    _, states = B.mv(w.team, w.env, sub, True, True)
    dt = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, st_early = B.mv(w.team, w.env, w.paths, True, False)
    dt_early = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    rate = states / dt
    return dict(kind="cpu SIMD rake, W = 8, FP32", threads=threads,
                exhaustive=dict(robot_states_per_s=rate, sample=f"first {sub.n_queries} motions, {states} robot-states",
                                seconds=dt),
                early_exit=dict(ms_per_call=dt_early * 1e3, motions=w.paths.n_queries,
                                robot_states_evaluated=st_early),
                gpu_over_simd_exhaustive=value / rate)


def cpu_baseline(w, max_queries, target_s=15.0):
    """The FP64 oracle on the host cores, on the same work as the headline: MV with
    robot-obstacle, self and robot-robot checks, every relation at every state
    (its exhaustive scan), over the first motions of the workload; the sample is
    sized from a short calibration run to take about target_s seconds."""
    import oracle
    ot, oe = oracle.Team(w.team), oracle.Env(w.env)
    n = w.paths.n_queries
    cal = w.paths.subset(np.arange(min(n, 256)))
    oracle.mv(ot, oe, oracle.Paths(cal.subset(np.arange(min(8, cal.n_queries)))), exhaustive=True)   # warm
    t0 = time.perf_counter()
    oracle.mv(ot, oe, oracle.Paths(cal), exhaustive=True)
    dt_cal = max(time.perf_counter() - t0, 1e-6)
    m = int(min(n, max_queries, max(cal.n_queries, cal.n_queries * target_s / dt_cal)))
    sub = w.paths.subset(np.arange(m))
    op = oracle.Paths(sub)
    t0 = time.perf_counter()
    valid = oracle.mv(ot, oe, op, exhaustive=True)
    dt = time.perf_counter() - t0
    states = float(np.sum(sub.horizon()) * len(w.team))
    return dict(value=states / dt, unit="robot-states/s", cores=int(oracle.threads()), kind="oracle",
                sample=(f"exhaustive MV (robot-obstacle, self, robot-robot; every relation at every state) over "
                        f"the first {m} of the {n} motions; {states:.4g} robot-states in {dt:.1f} s wall; "
                        f"{valid.mean() * 100:.1f}% valid"))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--queries", type=int, default=65536)
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-queries", type=int, default=65536, help="upper bound on the oracle sample")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="first run a plain device copy of this many MiB (HBM counter calibration)")
    ap.add_argument("--ordering-study", type=int, default=0, metavar="MOTIONS",
                    help="only run the early-termination ordering study with this many motions per team")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path (asked for --gpus {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2604_23960_amd import mrv
    from paper_2604_23960_amd import workloads as W

    def log(*a):
        print("[bench]", *a, file=sys.stderr, flush=True)

    if args.ordering_study > 0:
        print(json.dumps(dict(study="mv-ordering", step_l2=1.0 / 128,
                              rows=ordering_study(log, args.ordering_study))), flush=True)
        return

    if args.copy_calib_mib > 0:
        n = args.copy_calib_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {args.copy_calib_mib} MiB read + written")
        del src, dst
    log("generating the four-arm workload")
    w = W.arms_workload(args.queries)
    ctx = mrv.Context(0)
    team, env = ctx.load_team(w.team), ctx.load_env(w.env)
    dp = mrv.DevicePaths(w.paths)
    out = torch.zeros(w.paths.n_queries, dtype=torch.uint8, device="cuda")
    flags = mrv.CHECK_ENV | mrv.EXHAUSTIVE
    log("timing exhaustive MV")
    wall, kms, st = run_device(ctx, team, env, dp, 0, flags, out, args.steps, args.warmup)
    states = st["states_evaluated"]
    value = states * args.steps / wall
    ms_per_step = wall / args.steps * 1e3
    kernel_ms = float(np.mean(kms))
    flop = executed_flop(w.team, w.env, st)
    achieved = flop / (kernel_ms * 1e-3)
    roofline = dict(bound="alu", achieved=achieved / 1e12, peak=PEAK_FP32_VALU / 1e12, unit="TFLOP/s",
                    frac=achieved / PEAK_FP32_VALU, traffic=profiled_traffic(), kernel="k_validate<3> (exhaustive MV)",
                    kernel_ms=kernel_ms, flop_per_launch=flop)
    extra = dict(states_covered=st["states_covered"], rr_tests=st["rr_tests"], env_tests=st["env_tests"],
                 self_tests=st["self_tests"], near_rechecks=st["near_rechecks"],
                 pair_tests_per_s=(st["rr_tests"] + st["env_tests"] + st["self_tests"]) / (kernel_ms * 1e-3),
                 valid_fraction=float(out.float().mean().item()))
    if not args.no_extra:
        log("timing early-exit MV")
        wall2, kms2, st2 = run_device(ctx, team, env, dp, 0, mrv.CHECK_ENV, out, 5, 1)
        extra["mv_early_exit"] = dict(covered_states_per_s=st2["states_covered"] * 5 / wall2,
                                      evaluated_states_per_s=st2["states_evaluated"] * 5 / wall2,
                                      ms_per_call=wall2 / 5 * 1e3, effort=st2["states_evaluated"] / st2["states_covered"])
        log("timing prioritised MV (focus on arm 0)")
        wall4, kms4, st4 = run_device(ctx, team, env, dp, 0, mrv.CHECK_ENV | mrv.EXHAUSTIVE, out, 3, 1, focus=1)
        wall5, _, st5 = run_device(ctx, team, env, dp, 0, mrv.CHECK_ENV, out, 5, 1, focus=1)
        extra["mv_focus_arm0"] = dict(
            exhaustive=dict(kernel_ms=float(np.mean(kms4)), states_per_s=st4["states_evaluated"] * 3 / wall4,
                            rr_tests=st4["rr_tests"], env_tests=st4["env_tests"], self_tests=st4["self_tests"]),
            early_exit=dict(ms_per_call=wall5 / 5 * 1e3, covered_states_per_s=st5["states_covered"] * 5 / wall5))
        log("timing FFC on the arm + rectangle workload")
        wf = W.ffc_workload(16384)
        tf = ctx.load_team(wf.team)
        dpf = mrv.DevicePaths(wf.paths)
        cf = torch.zeros((wf.paths.n_queries, 3), dtype=torch.int32, device="cuda")
        wall3, kms3, st3 = run_device(ctx, tf, -1, dpf, 1, 0, cf, 5, 1)
        extra["ffc_hetero"] = dict(queries=wf.paths.n_queries, ms_per_call=wall3 / 5 * 1e3,
                                   covered_states_per_s=st3["states_covered"] * 5 / wall3,
                                   evaluated_states_per_s=st3["states_evaluated"] * 5 / wall3,
                                   null_fraction=float((cf[:, 0] < 0).float().mean().item()))
        wall4, kms4, st4 = run_device(ctx, tf, -1, dpf, 1, mrv.EXHAUSTIVE, cf, 3, 1)
        extra["ffc_hetero_exhaustive"] = dict(ms_per_call=wall4 / 3 * 1e3,
                                              states_per_s=st4["states_evaluated"] * 3 / wall4)
        log("serving loop vs plain launches")
        extra["serving"] = serving_bench(log)
        log("16-robot point-cloud workload")
        extra["cloud"] = cloud_bench(log)
        log("Composite RRT-Connect with served edge checks")
        from paper_2604_23960_amd import planner
        extra["planner"] = planner.plan_study(ctx)
    cpu = None
    if not args.no_cpu:
        log("timing the FP64 oracle on the host")
        cpu = cpu_baseline(w, args.cpu_queries)
        log("timing the SIMD rake baseline on the host")
        extra["cpu_simd_rake"] = simd_baseline(w, value)
        extra["gpu_covered_states_per_s_early_exit_same_metric"] = extra.get("mv_early_exit", {}).get(
            "covered_states_per_s")
    line = dict(metric="robot-states validated/s", value=value, unit="robot-states/s", n_gpus=1,
                steps=args.steps, warmup=args.warmup, ms_per_step=ms_per_step, higher_is_better=True,
                scaling="weak", vs_baseline=None, dtype="f32", data="synthetic",
                config=dict(workload="arms-4x7R-60sph-20box-8cyl MV exhaustive (env+self+robot-robot)",
                            motions=w.paths.n_queries, robots=len(w.team), spheres_per_robot=60,
                            boxes=20, cylinders=8, step="1/32 rad Linf", precision="fp32 + fp64 near-contact recheck"),
                roofline=roofline, cpu_baseline=cpu, extra=extra)
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
