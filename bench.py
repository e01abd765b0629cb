"""Benchmark of the MV/FFC hot path on one MI355X.

Headline: MotionValidation with robot-obstacle, self and robot-robot checks on
the four-arm workload (4 seeded 7-R arms x 60 spheres, 20 boxes + 8 cylinders,
65,536 straight-line motions at 1/32 rad max-joint step), every state evaluated
(exhaustive mode), inputs resident in HBM.  One step = one mrv_mv_device call
over all 65,536 motions.  ``value`` = robot-states validated per second.

Also reported (``extra``): early-exit MV on the same motions, FFC on the
4-arm + 4-rectangle decoupled-path workload (16,384 path sets), the disk
workload, the FP32 roofline of the validation kernel and the FP64 oracle on the
host cores (``cpu_baseline``).  ``--cloud-exhaustive N`` and ``--ffc-only N``
run only the profiled configurations of the point-cloud and FFC kernels.
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
    """FLOP of one MV/FFC launch from its executed-test counters, split by the pipe
    that runs it.  Matrix cores: 10 per robot-robot, self and sphere-point test (the
    Gram form's 16 x 16 x 4 products plus the vector unit's minimum; sphere-point
    tests are the pairs of a 16-sphere group's active spheres and the points its
    blocks take, 16 at a time from the cell rows its spheres reach).  Vector unit: FK and sphere placement of every evaluated robot-state, 10
    per sphere-obstacle test, 26 per box or cylinder test actually run (the kernel
    skips those whose world box misses a row of 16 spheres by more than the near
    band; that skip is comparisons only and counts no FLOP)."""
    from paper_2604_23960_amd import workloads as W
    assert FLOP_SPHERE_BOX == FLOP_SPHERE_CYL        # one counter covers both
    ts = stats["states_evaluated"] / len(team)
    fk = 0
    for r in team:
        fk += sum(FLOP_REV_JOINT if jt == W.REV_Z else FLOP_PRI_JOINT for jt in r.joint_type)
        fk += r.n_spheres * FLOP_SPHERE_PLACE
    n_sph = len(env.spheres) if env is not None else 0
    sph_tests = ts * sum(r.n_spheres for r in team) * n_sph if stats["env_tests"] else 0.0
    mfma = (stats["rr_tests"] + stats["self_tests"] + stats.get("point_tests", 0)) * FLOP_SPHERE_SPHERE
    valu = ts * fk + sph_tests * FLOP_SPHERE_SPHERE + (stats["env_tests"] - sph_tests) * FLOP_SPHERE_BOX
    return dict(total=mfma + valu, mfma=mfma, valu=valu)


def roofline_of(team, env, stats, kernel_ms, kernel):
    """Executed FLOP of a launch over its kernel time against the FP32 peak."""
    f = executed_flop(team, env, stats)
    achieved = f["total"] / (kernel_ms * 1e-3)
    return dict(bound="alu", achieved=achieved / 1e12, peak=PEAK_FP32_VALU / 1e12, unit="TFLOP/s",
                frac=achieved / PEAK_FP32_VALU, kernel=kernel, kernel_ms=kernel_ms, flop_per_launch=f["total"],
                flop_on_matrix_cores=f["mfma"], flop_on_vector_unit=f["valu"])


def library_decider(ctx):
    """Endpoint validity decided by this library: MV with obstacle and self tests of
    single-state motions.  Returns decide(robots, env, configs) for
    workloads.valid_configs and a function that unloads what it loaded."""
    from paper_2604_23960_amd import mrv
    from paper_2604_23960_amd import workloads as W
    teams, envs = {}, {}

    def decide(robots, env, cfg):
        kt = tuple(id(r) for r in robots)
        if kt not in teams:
            teams[kt] = (ctx.load_team(robots), robots)
        if id(env) not in envs:
            envs[id(env)] = (ctx.load_env(env), env)
        one = W.straight_line_paths(cfg, cfg, [r.dof for r in robots], 1.0, "linf", cfg.shape[2])
        return ctx.mv(teams[kt][0], envs[id(env)][0], one, mrv.CHECK_ENV).astype(bool)

    def release():
        for h, _ in list(teams.values()) + list(envs.values()):
            ctx.unload(h)
        teams.clear()
        envs.clear()
    return decide, release


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
    The orders: combined or hierarchical (all obstacle tiles before robot-robot
    tiles, Alg. 1) with the golden-ratio bisection, rake or linear tile order;
    robot-robot tests before obstacle tests within a tile; and the
    pair-prioritised order (adjacent bases first within a tile, §III-A).
    Endpoints are composed from per-robot configurations that are valid alone
    (self and obstacle tests of a one-robot team), then kept if the whole team's
    state is valid."""
    import torch
    from paper_2604_23960_amd import mrv
    from paper_2604_23960_amd import workloads as W
    orders = [("combined-bisect", 0), ("combined-rake", mrv.ORDER_RAKE), ("combined-linear", mrv.ORDER_LINEAR),
              ("hierarchical-bisect", mrv.HIERARCHICAL), ("hierarchical-rake", mrv.HIERARCHICAL | mrv.ORDER_RAKE),
              ("hierarchical-linear", mrv.HIERARCHICAL | mrv.ORDER_LINEAR),
              ("pairs-first-bisect", mrv.PAIRS_FIRST),
              ("combined-bisect-pair-priority", mrv.PAIR_PRIORITY),
              ("pairs-first-bisect-pair-priority", mrv.PAIRS_FIRST | mrv.PAIR_PRIORITY),
              ("combined-linear-pair-priority", mrv.ORDER_LINEAR | mrv.PAIR_PRIORITY)]
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


def serving_bench(log, n_requests=20000, n_sat=4000, n_streams=4):
    """Served (mrv_submit/mrv_wait, continuous batching) vs plain (one synchronous
    call per query, one host thread and stream; also n_streams threads, each with
    its own context and stream) for 64 simulated clients with resident teams of
    2-8 robots.  Saturation throughput (all requests at once), then Poisson sweeps
    of n_requests requests per offered rate: the plain forms at fractions of their
    saturation rate, the served form at multiples of the plain form's largest
    sustained rate.  A run is sustained when its queue does not grow (loadgen)."""
    from paper_2604_23960_amd import loadgen, mrv
    from paper_2604_23960_amd import workloads as W
    teams, env, reqs = W.serving_workload(n_requests)
    hps = loadgen.prepare(reqs)
    ctxs = [mrv.Context(0) for _ in range(n_streams)]
    ctx = ctxs[0]
    hs = [[c.load_team(t) for t in teams] for c in ctxs]
    es = [c.load_env(env) for c in ctxs]
    handles, e = hs[0], es[0]
    res = dict(clients=len(teams), requests_per_point=n_requests,
               mv_fraction=float(np.mean([r.kind == 0 for r in reqs])),
               binding_overhead_us_per_call=loadgen.binding_overhead_us(ctx, handles[0], 7))
    # warm-up: the served slots' scratch grows to the batch sizes of the timed runs
    loadgen.run_plain(ctx, handles, e, reqs[:50], hps[:50], float("inf"))
    loadgen.run_plain_streams(ctxs, hs, es, reqs[:200], hps[:200], float("inf"))
    loadgen.run_served(ctx, handles, e, reqs, hps, float("inf"))
    log("serving: saturation")
    res["plain_saturated"] = loadgen.run_plain(ctx, handles, e, reqs[:n_sat], hps[:n_sat], float("inf"))[0]
    res["plain_4stream_saturated"] = loadgen.run_plain_streams(ctxs, hs, es, reqs[:n_sat], hps[:n_sat],
                                                               float("inf"))[0]
    res["served_saturated"] = loadgen.run_served(ctx, handles, e, reqs, hps, float("inf"))[0]
    # answers: served equal plain equal 4-stream plain
    _, a = loadgen.run_served(ctx, handles, e, reqs[:n_sat], hps[:n_sat], float("inf"))
    _, b = loadgen.run_plain(ctx, handles, e, reqs[:n_sat], hps[:n_sat], float("inf"))
    _, c = loadgen.run_plain_streams(ctxs, hs, es, reqs[:n_sat], hps[:n_sat], float("inf"))
    flat = lambda x: np.asarray(x).reshape(-1)
    res["served_answers_equal_plain"] = all(np.array_equal(flat(x), flat(y)) and np.array_equal(flat(x), flat(z))
                                            for x, y, z in zip(a, b, c))
    sweep = []

    def point(form, rate, seed):
        if form == "plain":
            r = loadgen.run_plain(ctx, handles, e, reqs, hps, rate, seed=seed)[0]
        elif form == "plain_4stream":
            r = loadgen.run_plain_streams(ctxs, hs, es, reqs, hps, rate, seed=seed)[0]
        else:
            r = loadgen.run_served(ctx, handles, e, reqs, hps, rate, seed=seed)[0]
        r.update(form=form, offered_rate=rate)
        sweep.append(r)
        log(f"serving: {form} at {rate:.0f}/s: {r['qps']:.0f}/s, p50 {r['p50_ms']:.2f} ms, "
            f"p99 {r['p99_ms']:.2f} ms, sustained {r['sustained']}")
        return r

    best = {}
    for form in ("plain", "plain_4stream"):
        sat = res[form + "_saturated"]["qps"]
        for k, f in enumerate((0.5, 0.8, 0.95)):
            r = point(form, f * sat, 10 + k)
            if r["sustained"]:
                best[form] = r
    plain_best = best.get("plain")
    base = plain_best["offered_rate"] if plain_best else res["plain_saturated"]["qps"]
    served_best = None
    for k, m in enumerate((1, 2, 5, 8, 12)):
        r = point("served", m * base, 20 + k)
        if r["sustained"]:
            served_best = r
    res["sweep"] = sweep
    res["plain_max_sustained"] = plain_best
    res["plain_4stream_max_sustained"] = best.get("plain_4stream")
    res["served_max_sustained"] = served_best
    at5 = next((r for r in sweep if r["form"] == "served" and abs(r["offered_rate"] - 5 * base) < 1e-6), None)
    res["served_at_5x_plain"] = at5
    if plain_best and served_best:
        res["served_over_plain_sustained_rate"] = served_best["offered_rate"] / plain_best["offered_rate"]
        res["five_x_criterion"] = bool(at5 is not None and at5["sustained"] and
                                       at5["p99_ms"] <= plain_best["p99_ms"])
    res["served_over_plain_saturation"] = res["served_saturated"]["qps"] / res["plain_saturated"]["qps"]
    for c in ctxs:
        c.close()
    return res


def disks_bench(ctx, n_queries=4096, reps=20):
    """The disk workload with valid endpoints: MV (obstacles on) and FFC over all
    4,096 motions per call, the call's wall time (latency-bound: about 0.2 G FLOP)."""
    import torch
    from paper_2604_23960_amd import mrv
    from paper_2604_23960_amd import workloads as W
    decide, release = library_decider(ctx)
    w = W.disks_workload(n_queries, decide=decide)
    release()
    th, eh = ctx.load_team(w.team), ctx.load_env(w.env)
    dp = mrv.DevicePaths(w.paths)
    o = torch.zeros(n_queries, dtype=torch.uint8, device="cuda")
    c = torch.zeros((n_queries, 3), dtype=torch.int32, device="cuda")
    w1, k1, s1 = run_device(ctx, th, eh, dp, 0, mrv.CHECK_ENV, o, reps, 3)
    valid = float(o.float().mean().item())
    w2, k2, s2 = run_device(ctx, th, -1, dp, 1, 0, c, reps, 3)
    res = dict(queries=n_queries, endpoints=w.notes, valid_fraction=valid,
               null_ffc_fraction=float((c[:, 0] < 0).float().mean().item()),
               mv=dict(ms_per_call=w1 / reps * 1e3, kernel_ms=float(np.median(k1)),
                       covered_states_per_s=s1["states_covered"] * reps / w1),
               ffc=dict(ms_per_call=w2 / reps * 1e3, kernel_ms=float(np.median(k2)),
                        covered_states_per_s=s2["states_covered"] * reps / w2))
    ctx.unload(th)
    ctx.unload(eh)
    return res


def cloud_bench(log, n_queries=262_144, tune_sample=8192, exhaustive_tune_sample=1024, exhaustive_queries=8192,
                tune_budget_s=15.0):
    """16-robot team in a 200k-point cloud: early-exit MV and FFC over the whole
    batch, exhaustive MV on a slice (each with its roofline), default vs autotuned
    tiling (the tuner held to a time budget), and one-launch graph replay vs the
    plain multi-kernel launch for small batches."""
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
        w1, k1, s1 = run_device(ctx, th, eh, dmv, 0, mrv.CHECK_ENV, o_mv, 3, 1)
        out["mv_early_exit"] = dict(ms_per_call=w1 / 3 * 1e3, covered_states_per_s=s1["states_covered"] * 3 / w1,
                                    roofline=roofline_of(team, env, s1, float(np.mean(k1)), "k_validate<0, true> (early-terminating MV, point cloud)"))
        w2, k2, s2 = run_device(ctx, th, -1, dffc, 1, 0, o_ffc, 3, 1)
        out["ffc"] = dict(ms_per_call=w2 / 3 * 1e3, covered_states_per_s=s2["states_covered"] * 3 / w2,
                          evaluated_states_per_s=s2["states_evaluated"] * 3 / w2,
                          roofline=roofline_of(team, None, s2, float(np.mean(k2)), "k_validate<1, false> (early-terminating FFC)"))
        w3, k3, s3 = run_device(ctx, th, eh, dsub, 0, mrv.CHECK_ENV | mrv.EXHAUSTIVE, o_sub, 2, 1)
        out["mv_exhaustive_slice"] = dict(queries=sub.n_queries, ms_per_call=w3 / 2 * 1e3,
                                          kernel_ms=float(np.mean(k3)),
                                          states_per_s=s3["states_evaluated"] * 2 / w3,
                                          point_tests=s3["point_tests"], rr_tests=s3["rr_tests"],
                                          roofline=roofline_of(team, env, s3, float(np.mean(k3)), "k_validate<3, true> (exhaustive MV, point cloud)"))
        out["tiling"] = dict(mv_early=ctx.get_tiling(th, 0), mv_exhaustive=ctx.get_tiling(th, 0, mrv.EXHAUSTIVE),
                             ffc=ctx.get_tiling(th, 1))
        log(f"cloud {tag}: {out['mv_exhaustive_slice']['states_per_s']:.3g} states/s exhaustive")
        return out

    res["default_tiling"] = measure("default")
    t0 = time.perf_counter()
    # exhaustive work per query does not depend on the batch, so a small sample
    # serves; early-terminating FFC prunes by what other queries' tiles found, which
    # a sample much smaller than the batch misrepresents (tuned on 1,024 path sets,
    # the chosen tiling took 80.7 ms on the 131,072 against 51.1 ms for the default;
    # on 8,192 the tuner keeps the default)
    ctx.autotune(th, eh, 0, sub.subset(np.arange(exhaustive_tune_sample)), mrv.CHECK_ENV | mrv.EXHAUSTIVE)
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


def calibration_copy(mib, log):
    """A plain device copy of mib MiB (read and written once): the reference the HBM
    counters of a profile are scaled by."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    log(f"copy calibration: {mib} MiB read + written")


def cloud_exhaustive(n_motions, steps, warmup, log):
    """Exhaustive MV with obstacles of the 16-robot point-cloud team over its first
    n_motions MV motions (the profiled configuration of the point-cloud kernel)."""
    import torch
    from paper_2604_23960_amd import mrv
    from paper_2604_23960_amd import workloads as W
    team, env, mvp, _ = W.big_hetero_workload(max(2 * n_motions, 1024))
    sub = mvp.subset(np.arange(n_motions))
    ctx = mrv.Context(0)
    th, eh = ctx.load_team(team), ctx.load_env(env)
    dp = mrv.DevicePaths(sub)
    out = torch.zeros(n_motions, dtype=torch.uint8, device="cuda")
    log(f"timing exhaustive MV of the cloud team over {n_motions} motions")
    wall, kms, st = run_device(ctx, th, eh, dp, 0, mrv.CHECK_ENV | mrv.EXHAUSTIVE, out, steps, warmup)
    kms_mean = float(np.mean(kms))
    res = dict(workload="cloud-16r-576sph-200kpts MV exhaustive", motions=n_motions, steps=steps,
               ms_per_step=wall / steps * 1e3, states_per_s=st["states_evaluated"] * steps / wall,
               point_tests=st["point_tests"], rr_tests=st["rr_tests"], self_tests=st["self_tests"],
               roofline=roofline_of(team, env, st, kms_mean, "k_validate<3, true> (exhaustive MV, point cloud)"))
    ctx.close()
    return res


def ffc_only(n_paths, steps, warmup, log):
    """Early-terminating and exhaustive FFC of the arm + rectangle team over n_paths
    path sets (the profiled configuration of the FFC kernels)."""
    import torch
    from paper_2604_23960_amd import mrv
    from paper_2604_23960_amd import workloads as W
    wf = W.ffc_workload(n_paths)
    ctx = mrv.Context(0)
    tf = ctx.load_team(wf.team)
    dpf = mrv.DevicePaths(wf.paths)
    cf = torch.zeros((wf.paths.n_queries, 3), dtype=torch.int32, device="cuda")
    res = dict(workload="arms4+rects4 FFC", path_sets=wf.paths.n_queries, steps=steps)
    for name, flags, kname in (("early", 0, "k_validate<1, false> (early-terminating FFC)"),
                               ("exhaustive", mrv.EXHAUSTIVE, "k_validate<4, false> (exhaustive FFC)")):
        log(f"timing {name} FFC over {wf.paths.n_queries} path sets")
        wall, kms, st = run_device(ctx, tf, -1, dpf, 1, flags, cf, steps, warmup)
        res[name] = dict(ms_per_step=wall / steps * 1e3, states_evaluated=st["states_evaluated"],
                         rr_tests=st["rr_tests"],
                         roofline=roofline_of(wf.team, None, st, float(np.mean(kms)), kname))
    ctx.close()
    return res


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, max_queries, target_s=15.0):
    """The FP64 oracle on the host cores, on the same work as the headline: MV with
    robot-obstacle, self and robot-robot checks, every relation at every state
    (its exhaustive scan), over the first motions of the workload; the sample is
    sized from a short calibration run to take about target_s seconds.  Also the
    oracle on one thread over a 1/64 subsample (every 64th motion)."""
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
    cores = int(oracle.threads())
    one = w.paths.subset(np.arange(0, n, 64))
    t0 = time.perf_counter()
    oracle.mv(ot, oe, oracle.Paths(one), exhaustive=True, nthreads=1)
    dt1 = time.perf_counter() - t0
    states1 = float(np.sum(one.horizon()) * len(w.team))
    return dict(value=states / dt, unit="robot-states/s", cores=cores, kind="oracle",
                cpu_model=cpu_model(), host_threads=os.cpu_count(),
                sample=(f"exhaustive MV (robot-obstacle, self, robot-robot; every relation at every state) over "
                        f"the first {m} of the {n} motions; {states:.4g} robot-states in {dt:.1f} s wall; "
                        f"{valid.mean() * 100:.1f}% valid"),
                single_thread=dict(value=states1 / dt1, motions=one.n_queries, seconds=dt1,
                                   sample=f"every 64th of the {n} motions (1/64), one thread"))


def precision_vs_oracle(ctx, cases, n_states=256, seed=5):
    """FP32 against FP64: for sampled (query, timestep) states of each workload, the
    sphere centres the kernels compute (mrv_spheres, relative to the team origin,
    the origin then added in FP32) against the oracle's FP64 centres; the largest
    centre error and the largest change of any robot-robot clearance
    |p_a - p_b| - (r_a + r_b) evaluated in FP64 from the two sets of centres
    (|delta32 - delta64| of the FK the tests see).  The Gram-form sums of the
    matrix-core tests add at most 32 u (rho^2 + r_max^2) to a squared distance
    (u = 2^-24, rho = largest |centre - origin|), stated beside it."""
    import oracle
    rng = np.random.default_rng(seed)
    out = {}
    for name, team, paths in cases:
        th = ctx.load_team(team)
        ot, op = oracle.Team(team), oracle.Paths(paths)
        T = paths.horizon()
        qs = rng.integers(0, paths.n_queries, n_states)
        ts = np.array([rng.integers(0, T[q]) for q in qs])
        S = sum(r.n_spheres for r in team)
        got = ctx.spheres(th, paths, qs, ts, S).astype(np.float64)
        rob = np.concatenate([[k] * r.n_spheres for k, r in enumerate(team)])
        cerr, derr, rho = 0.0, 0.0, 0.0
        for k, (q, t) in enumerate(zip(qs, ts)):
            ref = oracle.team_spheres(ot, op, int(q), int(t))
            cerr = max(cerr, float(np.abs(got[k, :, :3] - ref[:, :3]).max()))
            rho = max(rho, float(np.linalg.norm(ref[:, :3] - ref[:, :3].mean(0), axis=1).max()))
            a, b = np.nonzero(rob[:, None] < rob[None, :])
            d64 = np.linalg.norm(ref[a, :3] - ref[b, :3], axis=1) - (ref[a, 3] + ref[b, 3])
            d32 = np.linalg.norm(got[k, a, :3] - got[k, b, :3], axis=1) - (ref[a, 3] + ref[b, 3])
            if len(a):
                derr = max(derr, float(np.abs(d32 - d64).max()))
        rmax = max(float(np.max(r.sphere_xyzr[:, 3])) for r in team)
        u = 2.0 ** -24
        out[name] = dict(states=n_states, max_centre_err_m=cerr, max_rr_clearance_err_m=derr,
                         gram_bound_sq_m2=32 * u * (rho ** 2 + rmax ** 2))
        ctx.unload(th)
    return out


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
    ap.add_argument("--ordering-out", default="",
                    help="also write the ordering study's JSON record to this file")
    ap.add_argument("--cloud-exhaustive", type=int, default=0, metavar="MOTIONS",
                    help="only time exhaustive MV of the 16-robot point-cloud team over this many motions")
    ap.add_argument("--ffc-only", type=int, default=0, metavar="PATH_SETS",
                    help="only time FFC (early-terminating and exhaustive) of the arm + rectangle team")
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
        rec = dict(study="mv-ordering", step_l2=1.0 / 128, motions=args.ordering_study,
                   rows=ordering_study(log, args.ordering_study))
        if args.ordering_out:
            with open(args.ordering_out, "w") as f:
                json.dump(rec, f, indent=1)
        print(json.dumps(rec), flush=True)
        return

    if args.cloud_exhaustive > 0:
        if args.copy_calib_mib > 0:
            calibration_copy(args.copy_calib_mib, log)
        print(json.dumps(cloud_exhaustive(args.cloud_exhaustive, args.steps, args.warmup, log)), flush=True)
        return

    if args.ffc_only > 0:
        if args.copy_calib_mib > 0:
            calibration_copy(args.copy_calib_mib, log)
        print(json.dumps(ffc_only(args.ffc_only, args.steps, args.warmup, log)), flush=True)
        return

    if args.copy_calib_mib > 0:
        calibration_copy(args.copy_calib_mib, log)
    ctx = mrv.Context(0)
    decide, release = library_decider(ctx)
    log("generating the four-arm workload (endpoints valid, decided by this library)")
    w = W.arms_workload(args.queries, decide=decide)
    release()
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
    roofline = roofline_of(w.team, w.env, st, kernel_ms, "k_validate<3, false> (exhaustive MV)")
    roofline["traffic"] = profiled_traffic()
    extra = dict(states_covered=st["states_covered"], rr_tests=st["rr_tests"], env_tests=st["env_tests"],
                 self_tests=st["self_tests"], near_rechecks=st["near_rechecks"],
                 pair_tests_per_s=(st["rr_tests"] + st["env_tests"] + st["self_tests"]) / (kernel_ms * 1e-3),
                 valid_fraction=float(out.float().mean().item()), endpoints=w.notes)
    if not args.no_extra:
        log("timing early-exit MV")
        wall2, kms2, st2 = run_device(ctx, team, env, dp, 0, mrv.CHECK_ENV, out, 5, 1)
        extra["mv_early_exit"] = dict(covered_states_per_s=st2["states_covered"] * 5 / wall2,
                                      evaluated_states_per_s=st2["states_evaluated"] * 5 / wall2,
                                      ms_per_call=wall2 / 5 * 1e3, effort=st2["states_evaluated"] / st2["states_covered"],
                                      roofline=roofline_of(w.team, w.env, st2, float(np.mean(kms2)),
                                                           "k_validate<0, false> (early-terminating MV)"))
        log("timing prioritised MV (focus on arm 0)")
        wall4, kms4, st4 = run_device(ctx, team, env, dp, 0, mrv.CHECK_ENV | mrv.EXHAUSTIVE, out, 3, 1, focus=1)
        wall5, _, st5 = run_device(ctx, team, env, dp, 0, mrv.CHECK_ENV, out, 5, 1, focus=1)
        extra["mv_focus_arm0"] = dict(
            exhaustive=dict(kernel_ms=float(np.mean(kms4)), states_per_s=st4["states_evaluated"] * 3 / wall4,
                            rr_tests=st4["rr_tests"], env_tests=st4["env_tests"], self_tests=st4["self_tests"]),
            early_exit=dict(ms_per_call=wall5 / 5 * 1e3, covered_states_per_s=st5["states_covered"] * 5 / wall5))
        log("disk workload (valid endpoints)")
        extra["disks"] = disks_bench(ctx)
        log("timing FFC on the arm + rectangle workload")
        wf = W.ffc_workload(16384)
        tf = ctx.load_team(wf.team)
        dpf = mrv.DevicePaths(wf.paths)
        cf = torch.zeros((wf.paths.n_queries, 3), dtype=torch.int32, device="cuda")
        wall3, kms3, st3 = run_device(ctx, tf, -1, dpf, 1, 0, cf, 5, 1)
        extra["ffc_hetero"] = dict(queries=wf.paths.n_queries, ms_per_call=wall3 / 5 * 1e3,
                                   covered_states_per_s=st3["states_covered"] * 5 / wall3,
                                   evaluated_states_per_s=st3["states_evaluated"] * 5 / wall3,
                                   null_fraction=float((cf[:, 0] < 0).float().mean().item()),
                                   roofline=roofline_of(wf.team, None, st3, float(np.mean(kms3)),
                                                        "k_validate<1, false> (early-terminating FFC)"))
        wall4, kms4, st4 = run_device(ctx, tf, -1, dpf, 1, mrv.EXHAUSTIVE, cf, 3, 1)
        extra["ffc_hetero_exhaustive"] = dict(ms_per_call=wall4 / 3 * 1e3,
                                              states_per_s=st4["states_evaluated"] * 3 / wall4,
                                              roofline=roofline_of(wf.team, None, st4, float(np.mean(kms4)),
                                                                   "k_validate<4, false> (exhaustive FFC)"))
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
        log("FP32 against FP64 sphere centres and clearances")
        cases = [("arms", w.team, w.paths.subset(np.arange(512)))]
        if not args.no_extra:
            wd = W.disks_workload(512)
            cases.insert(0, ("disks", wd.team, wd.paths))
            cases.append(("arms_rects", wf.team, wf.paths.subset(np.arange(512))))
            bt, _, bmv, _ = W.big_hetero_workload(1024)
            cases.append(("cloud_team", bt, bmv.subset(np.arange(256))))
        extra["precision_vs_oracle"] = precision_vs_oracle(ctx, cases)
        log("timing the SIMD rake baseline on the host")
        extra["cpu_simd_rake"] = simd_baseline(w, value)
        extra["gpu_covered_states_per_s_early_exit_same_metric"] = extra.get("mv_early_exit", {}).get(
            "covered_states_per_s")
    line = dict(metric="robot-states validated/s", value=value, unit="robot-states/s", n_gpus=1,
                steps=args.steps, warmup=args.warmup, ms_per_step=ms_per_step, higher_is_better=True,
                scaling="weak", vs_baseline=None, dtype="f32", data="synthetic",
                config=dict(workload="arms-4x7R-60sph-20box-8cyl MV exhaustive (env+self+robot-robot)",
                            motions=w.paths.n_queries, robots=len(w.team), spheres_per_robot=60,
                            boxes=20, cylinders=8, step="1/32 rad Linf",
                            endpoints="valid alone and as a team, decided by this library",
                            obstacle_cull=("box and cylinder tests skipped where the obstacle's world box misses "
                                           "a 16-sphere row's box by more than the near band; answers are the full "
                                           "scan's and only executed tests count as FLOP"),
                            precision="fp32 + fp64 near-contact recheck"),
                roofline=roofline, cpu_baseline=cpu, extra=extra)
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
