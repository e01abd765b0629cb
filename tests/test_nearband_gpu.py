"""GPU parity where the FP32 arithmetic is least sure of itself.

* Sphere pairs run on the matrix cores in the Gram form D = w_a + w_b -
  2 (p_a, r_a).(p_b, r_b), whose rounding bound grows with |p|^2, the squared
  distance from the team origin.  Pairs placed 1.5-2.3 m from the origin at
  clearances from -3 eps to +6 eps land in the bound's uncertain band, so the
  kernel must revisit them in the direct form and re-evaluate the near ones in
  FP64.  Robot-robot pairs (a probe robot against an arm of the four-arm team and
  of the 16-robot team) and self pairs (two spheres of one robot, one on its base
  frame) are placed so that collision iff the clearance is negative holds by
  construction; the test asserts that on the oracle too.
* Sphere-point tests also run on the matrix cores in a Gram form, D = |c|^2 -
  R^2 - 2 c.p + |p|^2, whose bound grows with |p|^2 relative to the cloud's
  origin.  A probe sphere is placed 1.6-3.0 m from it at clearances -3 eps to
  +6 eps from one point of a cloud (the point amid a cluster of points that stay
  clear), so the kernel decides some of them from the bound and revisits the rest
  in the direct form, re-evaluating the near ones in FP64.
* Teams and environments far from the world origin (hundreds of metres): the
  kernels work relative to the team's and the environment's origins, so answers
  equal the oracle's there too; where a query's relative coordinates are large
  (a disk driven 300 m from its base) the near band widens and answers still
  equal the oracle's.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2604_23960_amd import mrv
from paper_2604_23960_amd import workloads as W

pytestmark = pytest.mark.gpu

EPS = 1e-5
DELTAS = np.array([-3.0, -1.0, -0.1, 0.1, 1.0, 3.0, 6.0]) * EPS
R_PROBE = 0.05


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = mrv.Context(0)
    yield c
    c.close()


def team_origin(team):
    b = np.array([r.base.reshape(3, 4)[:, 3] for r in team])
    return 0.5 * (b.min(axis=0) + b.max(axis=0))


def probe_robot(locals_xyz, base_xyz=(0.0, 0.0, 0.0), base_spheres=(), self_pairs=(), radius=R_PROBE):
    """Three prismatic joints (x, y, z) on an unrotated base: a sphere with local
    centre c on frame 3 sits at base + q + c.  base_spheres are (centre, radius)
    on frame 0 (they do not move)."""
    frames = [0] * len(base_spheres) + [3] * len(locals_xyz)
    xyzr = [list(c) + [r] for c, r in base_spheres] + [list(c) + [radius] for c in locals_xyz]
    return W.Robot("probe", np.array([W.PRI_X, W.PRI_Y, W.PRI_Z], np.int32), np.stack([W.IDENTITY12] * 3),
                   np.array(frames, np.int32), np.array(xyzr, np.float64),
                   np.array(self_pairs, np.int32).reshape(-1, 2), W.frame12(np.eye(3), base_xyz),
                   np.full(3, -5.0), np.full(3, 5.0))


def single_state_paths(configs, dof_stride=7, T=1):
    """One query per row of configs [Q, n_robots, dof]: every robot holds its
    configuration for T states."""
    rows = []
    for cfg in configs:
        ts = np.array([0]) if T == 1 else np.array([0, T - 1])
        rows.append([(ts, np.repeat(c[None, :], len(ts), axis=0)) for c in cfg])
    return W.paths_from_lists(rows, dof_stride)


def free_states(team, n_try, seed):
    """Configurations of `team` free of robot-robot and self contact by more than
    the decoy margin, decided by the oracle (test infrastructure)."""
    rng = np.random.default_rng(seed)
    cand = W.sample_configs(rng, team, n_try, 7)
    ot = oracle.Team(team)
    ok = oracle.mv(ot, oracle.Env(W.Env()), oracle.Paths(single_state_paths(cand)), check_env=True).astype(bool)
    return cand[ok]


def place_probe(team, cfg, rng, slot, n_probe=20, lo=1.5, hi=2.3):
    """Find an exposed sphere s of `team` in state cfg whose centre lies lo..hi m
    from the team origin o.  The probe (base at o) carries sphere `slot` at the
    local centre where, with zero joint values, it touches s radially outward of
    it, and its other spheres further out; a joint vector delta * v then sets the
    clearance to delta.  Returns (probe, v, |s - o|) or None."""
    ot = oracle.Team(team)
    sp = oracle.team_spheres(ot, oracle.Paths(single_state_paths(cfg[None])), 0, 0)
    o = team_origin(team)
    d = np.linalg.norm(sp[:, :3] - o, axis=1)
    cand = np.nonzero((d >= lo) & (d <= hi))[0]
    rng.shuffle(cand)
    for s in cand:
        v = (sp[s, :3] - o) / d[s]
        c0 = sp[s, :3] + (sp[s, 3] + R_PROBE) * v - o
        locs = [c0 if j == slot else c0 + (0.25 + 0.01 * j) * v for j in range(n_probe)]
        # every probe sphere must be clear of every team sphere but s by a wide margin
        pts = o[None, :] + np.array(locs)
        gap = np.linalg.norm(pts[:, None, :] - sp[None, :, :3], axis=2) - sp[None, :, 3] - R_PROBE
        gap[slot, s] = np.inf
        if gap.min() > 0.02:
            return probe_robot(locs, base_xyz=tuple(o)), v, float(d[s])
    return None


def robot_robot_cases(team, seed, slots=(0, 9, 15, 17)):
    """Per probe slot: (slot, team + probe, configurations over DELTAS, |p|)."""
    rng = np.random.default_rng(seed)
    states = free_states(team, 20000, seed)
    assert len(states) > 0, "no collision-free state found"
    cases = []
    for slot in slots:
        for cfg in states[rng.permutation(len(states))]:
            got = place_probe(team, cfg, rng, slot)
            if got is None:
                continue
            probe, v, dist = got
            full = team + [probe]
            cfgs = np.zeros((len(DELTAS), len(full), 7))
            cfgs[:, :len(team)] = cfg
            cfgs[:, len(team), :3] = DELTAS[:, None] * v[None, :]
            cases.append((slot, full, cfgs, dist))
            break
    assert len(cases) == len(slots)
    return cases


def check_robot_robot_oracle(full, paths):
    """The oracle's answers, asserted against the construction: collision iff the
    clearance is negative, FFC = (0, owner of the touched sphere, probe)."""
    n = len(full)
    ot, op = oracle.Team(full), oracle.Paths(paths)
    expect_valid = (DELTAS >= 0).astype(np.uint8)
    ref_mv = oracle.mv(ot, None, op, check_env=False)
    ref_self = oracle.mv(ot, oracle.Env(W.Env()), op, check_env=True)
    ref_ffc = oracle.ffc(ot, op)
    assert np.array_equal(ref_mv, expect_valid) and np.array_equal(ref_self, expect_valid)
    for f, d in zip(ref_ffc, DELTAS):
        assert (f[0] == 0 and f[2] == n - 1 and 0 <= f[1] < n - 1) if d < 0 else tuple(f) == (-1, -1, -1)
    return ref_mv, ref_ffc


@pytest.mark.parametrize("which", ["arms", "cloud_team"])
def test_gram_near_band_robot_robot(ctx, which):
    team = W.arm_team(1) if which == "arms" else W.hetero_team(1, 8, 8, 1.0, ceiling=True)
    for slot, full, cfgs, dist in robot_robot_cases(team, 21 if which == "arms" else 22):
        for T in (1, 6):
            paths = single_state_paths(cfgs, T=T)
            ref_mv, ref_ffc = check_robot_robot_oracle(full, paths)
            th = ctx.load_team(full)
            for flags in (0, mrv.EXHAUSTIVE, mrv.CHECK_ENV, mrv.CHECK_ENV | mrv.EXHAUSTIVE,
                          mrv.CHECK_ENV | mrv.PAIRS_FIRST):
                say(which, "probe slot", slot, f"|p|={dist:.2f} m", "T", T, "MV flags", flags)
                got = ctx.mv(th, -1, paths, flags)
                assert np.array_equal(got, ref_mv), (slot, flags, got, ref_mv)
            for flags in (0, mrv.EXHAUSTIVE):
                say(which, "probe slot", slot, "T", T, "FFC flags", flags)
                got = ctx.ffc(th, paths, flags)
                assert np.array_equal(got, ref_ffc), (slot, flags, got, ref_ffc)
            ctx.unload(th)


def self_case(ia, ib, dist, seed, n_sph=20):
    """A robot whose self pair (ia, ib) joins a base-frame sphere `dist` m from the
    team origin (its base) and a frame-3 sphere that touches it, radially outward,
    at zero joint values; joint vector delta * w sets the clearance to delta.  The
    other spheres are decoys far from both (the frame-3 ones also listed as self
    pairs of ia).  Returns (robot, configurations over DELTAS)."""
    rng = np.random.default_rng(seed)
    w = rng.normal(size=3)
    w /= np.linalg.norm(w)
    side = np.cross(w, [0.0, 0.0, 1.0])
    side = side / np.linalg.norm(side) if np.linalg.norm(side) > 1e-3 else np.array([1.0, 0.0, 0.0])
    c_a, r_a = dist * w, 0.07
    c_b = c_a + (r_a + R_PROBE) * w
    order = []
    for j in range(n_sph):
        if j == ia:
            order.append((0, c_a, r_a))
        elif j == ib:
            order.append((3, c_b, R_PROBE))
        elif j % 2:
            order.append((0, -0.5 * w + 0.05 * j * side, 0.04))
        else:
            order.append((3, c_b + (0.3 + 0.02 * j) * w, R_PROBE))
    frames = np.array([f for f, _, _ in order], np.int32)
    xyzr = np.array([list(c) + [r] for _, c, r in order])
    pairs = [(ia, ib)] + [(ia, j) for j in range(n_sph) if j not in (ia, ib) and frames[j] == 3]
    robot = W.Robot("selfprobe", np.array([W.PRI_X, W.PRI_Y, W.PRI_Z], np.int32), np.stack([W.IDENTITY12] * 3),
                    frames, xyzr, np.array(pairs, np.int32), W.IDENTITY12.copy(), np.full(3, -5.0), np.full(3, 5.0))
    cfgs = (DELTAS[:, None] * w[None, :])[:, None, :]
    return robot, cfgs


@pytest.mark.parametrize("ia,ib", [(2, 9), (3, 18), (17, 0)])
def test_gram_near_band_self(ctx, ia, ib):
    for k, dist in enumerate((1.6, 2.2)):
        robot, cfgs = self_case(ia, ib, dist, 100 * ia + 10 * ib + k)
        paths = single_state_paths(cfgs, dof_stride=3, T=4)
        ot, op = oracle.Team([robot]), oracle.Paths(paths)
        ref = oracle.mv(ot, oracle.Env(W.Env()), op, check_env=True)
        assert np.array_equal(ref, (DELTAS >= 0).astype(np.uint8))      # by construction
        th = ctx.load_team([robot])
        for flags in (mrv.CHECK_ENV, mrv.CHECK_ENV | mrv.EXHAUSTIVE, mrv.CHECK_ENV | mrv.PAIRS_FIRST,
                      mrv.CHECK_ENV | mrv.HIERARCHICAL):
            say("self pair", ia, ib, f"|p|={dist}", "flags", flags)
            got = ctx.mv(th, -1, paths, flags)
            assert np.array_equal(got, ref), (ia, ib, dist, flags, got, ref)
        ctx.unload(th)


def point_case(dist, seed):
    """A probe robot (one sphere of radius R_PROBE on three prismatic joints) and a
    cloud (radius RP_PROBE) whose bounding box is centred at the world origin: the
    probe point p0 lies `dist` m from it along a random unit w, the sphere's centre
    at zero joint values at p0 - (R_PROBE + RP_PROBE) w, so joint vector -delta w
    sets the clearance to delta.  The other points are the box's corners and a
    cluster of 200 around p0, all clear of the sphere by at least 2 mm.
    Returns (robot, env, configurations over DELTAS)."""
    rng = np.random.default_rng(seed)
    w = rng.normal(size=3)
    w /= np.linalg.norm(w)
    p0 = dist * w
    c0 = p0 - (R_PROBE + RP_PROBE) * w
    corners = np.array([[sx, sy, sz] for sx in (-3.1, 3.1) for sy in (-3.1, 3.1) for sz in (-3.1, 3.1)])
    # cluster: directions mostly towards p0, at R + r_p + 2..30 mm from c0
    u = rng.normal(size=(200, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    u = np.where((u @ w)[:, None] < 0.2, u + 1.2 * w, u)
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    cl = c0 + (R_PROBE + RP_PROBE + rng.uniform(0.002, 0.03, (200, 1))) * u
    pts = np.concatenate([corners, cl, p0[None, :]])
    robot = probe_robot([(0.0, 0.0, 0.0)], base_xyz=c0)
    cfgs = (-DELTAS[:, None] * w[None, :])[:, None, :]
    return robot, W.Env(points=pts, point_radius=RP_PROBE), cfgs


RP_PROBE = 0.005


@pytest.mark.parametrize("dist", [1.6, 2.3, 3.0])
def test_gram_near_band_points(ctx, dist):
    robot, env, cfgs = point_case(dist, int(dist * 10))
    paths = single_state_paths(cfgs, dof_stride=3, T=4)
    ot, oe, op = oracle.Team([robot]), oracle.Env(env), oracle.Paths(paths)
    ref = oracle.mv(ot, oe, op, check_env=True)
    assert np.array_equal(ref, (DELTAS >= 0).astype(np.uint8))      # by construction
    th, eh = ctx.load_team([robot]), ctx.load_env(env)
    for flags in (mrv.CHECK_ENV, mrv.CHECK_ENV | mrv.EXHAUSTIVE, mrv.CHECK_ENV | mrv.PAIRS_FIRST,
                  mrv.CHECK_ENV | mrv.HIERARCHICAL):
        say("sphere-point probe", f"|p|={dist}", "flags", flags)
        got = ctx.mv(th, eh, paths, flags)
        assert np.array_equal(got, ref), (dist, flags, got, ref)
    ctx.unload(th)
    ctx.unload(eh)


def shifted(w, shift):
    """The workload moved rigidly by `shift` metres: bases and obstacles; joint
    values are relative to the bases and do not change."""
    shift = np.asarray(shift, np.float64)
    team = []
    for r in w.team:
        b = r.base.copy().reshape(3, 4)
        b[:, 3] += shift
        team.append(r.with_base(b.reshape(-1)))
    e = w.env
    env = W.Env(spheres=e.spheres.copy(), boxes=e.boxes.copy(), cylinders=e.cylinders.copy(),
                points=e.points.copy(), point_radius=e.point_radius)
    env.spheres[:, :3] += shift
    env.boxes[:, :3] += shift
    env.cylinders[:, :3] += shift
    if len(env.points):
        env.points += shift
    return dataclasses.replace(w, team=team, env=env)


@pytest.mark.parametrize("shift", [(300.0, -200.0, 50.0), (-750.0, 420.0, 3.0)])
def test_far_from_world_origin(ctx, shift):
    """The arm workload moved hundreds of metres away: MV (every mode) and FFC
    equal the oracle's on the moved inputs."""
    w = shifted(W.arms_workload(512), shift)
    ot, oe, op = oracle.Team(w.team), oracle.Env(w.env), oracle.Paths(w.paths)
    th, eh = ctx.load_team(w.team), ctx.load_env(w.env)
    for flags in (mrv.CHECK_ENV, mrv.CHECK_ENV | mrv.EXHAUSTIVE, 0, mrv.EXHAUSTIVE):
        say("arms moved by", shift, "MV flags", flags)
        ref = oracle.mv(ot, oe, op, check_env=bool(flags & mrv.CHECK_ENV))
        assert np.array_equal(ctx.mv(th, eh, w.paths, flags), ref), flags
    say("arms moved by", shift, "FFC")
    assert np.array_equal(ctx.ffc(th, w.paths), oracle.ffc(ot, op))
    ctx.unload(eh)
    ctx.unload(th)


def test_far_grazing_and_large_joint_values(ctx):
    """Exactly touching disks 600 m from the world origin (their bases there too),
    and the disk workload driven 300 m from the bases by its prismatic joints
    (relative coordinates of 300 m: the near band widens) among circles moved
    with it."""
    g = W.grazing_disks(90, 24)
    far = [r.with_base(W.frame12(np.eye(3), (600.0, -600.0, 0.0))) for r in g.team]
    ot, op = oracle.Team(far), oracle.Paths(g.paths)
    th = ctx.load_team(far)
    for flags in (0, mrv.EXHAUSTIVE):
        say("grazing disks 600 m away, flags", flags)
        assert np.array_equal(ctx.mv(th, -1, g.paths, flags), oracle.mv(ot, None, op, check_env=False))
        assert np.array_equal(ctx.ffc(th, g.paths, flags), oracle.ffc(ot, op))
    ctx.unload(th)

    d = W.disks_workload(1024)
    paths = dataclasses.replace(d.paths, wp_q=d.paths.wp_q + np.array([300.0, -300.0]))
    env = W.Env(spheres=d.env.spheres + np.array([300.0, -300.0, 0.0, 0.0]))
    ot, oe, op = oracle.Team(d.team), oracle.Env(env), oracle.Paths(paths)
    th, eh = ctx.load_team(d.team), ctx.load_env(env)
    for flags in (mrv.CHECK_ENV, mrv.CHECK_ENV | mrv.EXHAUSTIVE):
        say("disks driven 300 m by their joints, flags", flags)
        assert np.array_equal(ctx.mv(th, eh, paths, flags), oracle.mv(ot, oe, op))
    assert np.array_equal(ctx.ffc(th, paths), oracle.ffc(ot, op))
    ctx.unload(eh)
    ctx.unload(th)
