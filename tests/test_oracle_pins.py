"""Pins for the FP64 oracle: closed forms, hand-worked clearances, an independent
brute force on tiny teams, and invariants the definitions of MV (paper §III-A,
Alg. 1) and FFC (§III-B, Alg. 2) force.  CPU only."""
import math

import numpy as np
import pytest

import brute
import oracle
from paper_2604_23960_amd import workloads as W


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.lib()


def planar_2link(l1, l2, base=None):
    """Two REV_Z joints; F_2 = Tx(l1); spheres at the elbow (frame 1) and the tip (frame 2)."""
    f2 = W.frame12(np.eye(3), (l1, 0.0, 0.0))
    return W.Robot("p2", np.array([W.REV_Z, W.REV_Z], np.int32), np.stack([W.IDENTITY12, f2]),
                   np.array([1, 2], np.int32), np.array([[l1, 0, 0, 0.1], [l2, 0, 0, 0.1]]),
                   np.zeros((0, 2), np.int32), W.IDENTITY12.copy() if base is None else base,
                   -np.pi * np.ones(2), np.pi * np.ones(2))


# ----------------------------------------------------------------------------- FK

def test_fk_planar_two_link_closed_form():
    rng = np.random.default_rng(0)
    l1, l2 = 0.7, 0.45
    team = oracle.Team([planar_2link(l1, l2)])
    for _ in range(200):
        q = rng.uniform(-3, 3, 2)
        s = oracle.fk_robot(team, 0, q)
        c1, s1, c12, s12 = math.cos(q[0]), math.sin(q[0]), math.cos(q[0] + q[1]), math.sin(q[0] + q[1])
        assert np.allclose(s[0, :3], [l1 * c1, l1 * s1, 0.0], atol=1e-14)
        assert np.allclose(s[1, :3], [l1 * c1 + l2 * c12, l1 * s1 + l2 * s12, 0.0], atol=1e-14)


def test_fk_prismatic_chain_is_offset():
    rob = W.Robot("xyz", np.array([W.PRI_X, W.PRI_Y, W.PRI_Z], np.int32), np.stack([W.IDENTITY12] * 3),
                  np.array([3, 0], np.int32), np.array([[0.1, -0.2, 0.3, 0.05], [0.5, 0.5, 0.5, 0.05]]),
                  np.zeros((0, 2), np.int32), W.frame12(np.eye(3), (1.0, 2.0, 3.0)),
                  -np.ones(3), np.ones(3))
    team = oracle.Team([rob])
    q = np.array([0.25, -0.5, 0.125])
    s = oracle.fk_robot(team, 0, q)
    assert np.array_equal(s[0, :3], np.array([1.1, 1.8, 3.3]) + q) or np.allclose(
        s[0, :3], np.array([1.1, 1.8, 3.3]) + q, atol=1e-15)
    assert np.allclose(s[1, :3], [1.5, 2.5, 3.5], atol=1e-15)


def dh_reference(meta, base, q):
    """Standard DH product Base * T_1 ... T_k with T = Rz(q) Tz(d) Tx(a) Rx(alpha)."""
    a, d, alpha = meta["a"], meta["d"], meta["alpha"]
    M = brute.h4(base)
    frames_before_link = []
    for k in range(len(q)):
        Rz = np.eye(4)
        Rz[:2, :2] = [[math.cos(q[k]), -math.sin(q[k])], [math.sin(q[k]), math.cos(q[k])]]
        frames_before_link.append(M @ Rz)            # link k+1 geometry lives here
        T = np.eye(4)
        T[:3, :3] = W.rot_x(alpha[k])
        T[:3, 3] = [0.0, 0.0, 0.0]
        Tz = np.eye(4); Tz[2, 3] = d[k]
        Tx = np.eye(4); Tx[0, 3] = a[k]
        M = M @ Rz @ Tz @ Tx @ T
    return frames_before_link, M


def test_fk_dh_arm_matches_standard_dh_product():
    team_models = W.arm_team(1)
    team = oracle.Team(team_models)
    rng = np.random.default_rng(5)
    for r, rob in enumerate(team_models):
        for _ in range(20):
            q = rng.uniform(-2.9, 2.9, 7)
            sph, fr = oracle.fk_robot(team, r, q, frames=True)
            ref_frames, _ = dh_reference(rob.meta, rob.base, q)
            for k in range(7):
                assert np.allclose(fr[k + 1].reshape(3, 4), ref_frames[k][:3, :], atol=1e-13)
            for s in range(rob.n_spheres):
                f = int(rob.sphere_frame[s])
                ref = (ref_frames[f - 1] @ np.append(rob.sphere_xyzr[s, :3], 1.0))[:3]
                assert np.allclose(sph[s, :3], ref, atol=1e-13)


def test_fk_frames_orthonormal():
    team = oracle.Team(W.hetero_team(1, 8, 4, 1.0, ceiling=True))
    rng = np.random.default_rng(3)
    for r, rob in enumerate(team.robots):
        for _ in range(10):
            q = rng.uniform(rob.q_lo, rob.q_hi)
            _, fr = oracle.fk_robot(team, r, q, frames=True)
            for F in fr:
                R = F.reshape(3, 4)[:, :3]
                assert np.allclose(R.T @ R, np.eye(3), atol=1e-14)
                assert abs(np.linalg.det(R) - 1.0) < 1e-14


def test_fk_base_transform_applies_to_all_centres():
    rob = W.arm_models(1)[2]
    B = W.frame12(W.random_rotation(np.random.default_rng(9)), (0.3, -1.2, 0.7))
    t_id = oracle.Team([rob])
    t_b = oracle.Team([rob.with_base(B)])
    q = np.random.default_rng(1).uniform(-2.9, 2.9, 7)
    s0 = oracle.fk_robot(t_id, 0, q)
    s1 = oracle.fk_robot(t_b, 0, q)
    Bm = B.reshape(3, 4)
    assert np.allclose(s1[:, :3], s0[:, :3] @ Bm[:, :3].T + Bm[:, 3], atol=1e-13)
    assert np.array_equal(s0[:, 3], s1[:, 3])


def test_fk_matches_brute_force_homogeneous_products():
    team_models = W.hetero_team(1, 4, 3, 0.5)
    team = oracle.Team(team_models)
    rng = np.random.default_rng(11)
    for r, rob in enumerate(team_models):
        q = rng.uniform(rob.q_lo, rob.q_hi)
        assert np.allclose(oracle.fk_robot(team, r, q), brute.spheres_world(rob, q), atol=1e-13)


# ----------------------------------------------------------------------------- clearances

def test_clearance_box_hand_worked():
    box = np.concatenate([[0, 0, 0], np.eye(3).ravel(), [1, 1, 1]])
    assert oracle.clear_sphere_box([2, 0, 0], 0.5, box) == pytest.approx(0.5, abs=1e-15)
    assert oracle.clear_sphere_box([2, 2, 0], 0.5, box) == pytest.approx(math.sqrt(2) - 0.5, abs=1e-15)
    assert oracle.clear_sphere_box([2, 2, 2], 0.5, box) == pytest.approx(math.sqrt(3) - 0.5, abs=1e-15)
    assert oracle.clear_sphere_box([0, 0, 0], 0.5, box) == pytest.approx(-1.5, abs=1e-15)
    assert oracle.clear_sphere_box([0.75, 0.2, 0], 0.1, box) == pytest.approx(-0.35, abs=1e-15)
    # rotated and translated: a box rotated 45 degrees about z, long axis along (1,1)/sqrt2
    R = W.rot_z(math.pi / 4)
    box2 = np.concatenate([[1, 1, 0], R.ravel(), [2, 0.5, 0.5]])
    u = np.array([1, 1, 0]) / math.sqrt(2)
    assert oracle.clear_sphere_box(np.array([1, 1, 0]) + 3.0 * u, 0.25, box2) == pytest.approx(0.75, abs=1e-14)


def test_clearance_cylinder_hand_worked():
    cyl = np.array([0, 0, 0, 0, 0, 1, 1.0, 1.0])
    rho = 0.25
    assert oracle.clear_sphere_cylinder([3, 0, 0], rho, cyl) == pytest.approx(2 - rho, abs=1e-15)
    assert oracle.clear_sphere_cylinder([0, 0, 3], rho, cyl) == pytest.approx(2 - rho, abs=1e-15)
    assert oracle.clear_sphere_cylinder([2, 0, 2], rho, cyl) == pytest.approx(math.sqrt(2) - rho, abs=1e-15)
    assert oracle.clear_sphere_cylinder([0, 0, 0], rho, cyl) == pytest.approx(-1 - rho, abs=1e-15)
    assert oracle.clear_sphere_cylinder([0.5, 0, 0.9], rho, cyl) == pytest.approx(-0.1 - rho, abs=1e-15)
    # tilted axis (x): same geometry rotated
    cylx = np.array([1, 2, 3, 1, 0, 0, 1.0, 1.0])
    assert oracle.clear_sphere_cylinder([1, 5, 3], rho, cylx) == pytest.approx(2 - rho, abs=1e-15)
    assert oracle.clear_sphere_cylinder([4, 2, 3], rho, cylx) == pytest.approx(2 - rho, abs=1e-15)


def test_clearance_sphere_and_point():
    assert oracle.clear_sphere_sphere([0, 0, 0], 0.5, [3, 4, 0], 1.0) == pytest.approx(3.5, abs=1e-15)
    assert oracle.clear_sphere_point([0, 0, 0], 0.5, [0, 0, 0.6], 0.05) == pytest.approx(0.05, abs=1e-15)


def test_clearances_match_brute_formulation():
    rng = np.random.default_rng(21)
    env = W.cube_env(1)
    for _ in range(300):
        x = rng.uniform([-1.2, -1.2, -0.2], [1.2, 1.2, 2.2])
        r = rng.uniform(0.01, 0.1)
        for b in env.boxes:
            assert oracle.clear_sphere_box(x, r, b) == pytest.approx(brute.box_clear(x, r, b), abs=1e-12)
        for c in env.cylinders:
            assert oracle.clear_sphere_cylinder(x, r, c) == pytest.approx(brute.cyl_clear(x, r, c), abs=1e-12)


def test_point_index_matches_brute_force():
    rng = np.random.default_rng(4)
    pts = rng.uniform(-1, 1, (5000, 3))
    env = oracle.Env(W.Env(points=pts, point_radius=0.005))
    for _ in range(400):
        x = rng.uniform(-1.1, 1.1, 3)
        r = rng.uniform(0.01, 0.12)
        assert oracle.points_any_hit(env, x, r) == oracle.points_any_hit(env, x, r, brute=True)


# ----------------------------------------------------------------------------- paths

def test_path_state_exact_at_waypoints_and_padding():
    times = [0, 5, 9]
    cfgs = np.array([[0.1, -0.3], [0.7, 0.2], [-0.4, 0.9]])
    for t, c in zip(times, cfgs):
        assert np.array_equal(oracle.path_state(times, cfgs, 2, t), c)
    for t in (10, 50, 10_000):
        assert np.array_equal(oracle.path_state(times, cfgs, 2, t), cfgs[-1])
    got = oracle.path_state(times, cfgs, 2, 7)
    assert np.allclose(got, cfgs[1] + 0.5 * (cfgs[2] - cfgs[1]), atol=1e-16)


def test_motion_steps():
    assert oracle.motion_steps([0.3, 0.4], 0.005, "l2") == 100
    assert oracle.motion_steps([0.3, -0.41], 0.1, "linf") == 5
    assert oracle.motion_steps([0.0, 0.0], 0.1, "linf") == 0
    assert oracle.motion_steps([1.0], 1.0 / 32, "linf") == 32
    rng = np.random.default_rng(0)
    for _ in range(100):
        dq = rng.uniform(-1, 1, 7)
        assert oracle.motion_steps(dq, 1 / 32, "linf") == W.steps_for(dq, 1 / 32, "linf")
        assert oracle.motion_steps(dq, 0.005, "l2") == W.steps_for(dq, 0.005, "l2")


# ----------------------------------------------------------------------------- closed-form FFC / MV

def two_disk_paths(SA, GA, SB, GB, n):
    return W.paths_from_lists([[(np.array([0, n]), np.stack([SA, GA])),
                                (np.array([0, n]), np.stack([SB, GB]))]], 2)


def first_integer_in_quadratic(D0, DV, n, R):
    """First integer t in [0, n] with |D0 + (t/n) DV|^2 < R^2, or -1; None if too close to a root."""
    a = DV @ DV / n ** 2
    b = 2 * (D0 @ DV) / n
    c = D0 @ D0 - R * R
    if a == 0:
        return (0 if c < 0 else -1)
    disc = b * b - 4 * a * c
    if disc <= 0:
        return -1
    t1 = (-b - math.sqrt(disc)) / (2 * a)
    t2 = (-b + math.sqrt(disc)) / (2 * a)
    for root in (t1, t2):
        if abs(root - round(root)) < 1e-6:
            return None
    lo = max(0, math.floor(t1) + 1)
    if lo < t2 and lo <= n:
        return lo
    return -1


def test_ffc_two_disks_closed_form():
    rng = np.random.default_rng(7)
    team = [W.disk_robot(0.05, "a"), W.disk_robot(0.05, "b")]
    ot = oracle.Team(team)
    checked = hits = 0
    while checked < 400:
        SA, GA, SB, GB = (rng.uniform(0, 1, 2) for _ in range(4))
        n = W.steps_for(GA - SA, 0.005, "l2")
        n = max(n, W.steps_for(GB - SB, 0.005, "l2"), 1)
        expect = first_integer_in_quadratic(SA - SB, (GA - SA) - (GB - SB), n, 0.1)
        if expect is None:
            continue
        got = oracle.ffc(ot, oracle.Paths(two_disk_paths(SA, GA, SB, GB, n)))[0]
        if expect < 0:
            assert tuple(got) == (-1, -1, -1)
        else:
            assert tuple(got) == (expect, 0, 1)
            hits += 1
        checked += 1
    assert hits > 20


def test_mv_disk_vs_circle_closed_form():
    rng = np.random.default_rng(8)
    team = [W.disk_robot(0.05, "a")]
    ot = oracle.Team(team)
    checked = 0
    while checked < 300:
        c = rng.uniform(0.3, 0.7, 2)
        rc = rng.uniform(0.02, 0.08)
        env = W.Env(spheres=np.array([[c[0], c[1], 0.0, rc]]))
        S, G = rng.uniform(0, 1, 2), rng.uniform(0, 1, 2)
        n = max(W.steps_for(G - S, 0.005, "l2"), 1)
        expect = first_integer_in_quadratic(S - c, G - S, n, 0.05 + rc)
        if expect is None:
            continue
        p = W.paths_from_lists([[(np.array([0, n]), np.stack([S, G]))]], 2)
        got = oracle.mv(ot, oracle.Env(env), oracle.Paths(p))[0]
        assert got == (1 if expect < 0 else 0)
        checked += 1


# ----------------------------------------------------------------------------- brute force

def tiny_team(rng, n_robots):
    team = []
    for r in range(n_robots):
        kind = rng.integers(0, 3)
        if kind == 0:
            rob = W.disk_robot(rng.uniform(0.05, 0.2), f"d{r}")
        elif kind == 1:
            rob = W.se2_rect(0.0, f"s{r}")
            keep = rng.choice(rob.n_spheres, size=int(rng.integers(1, 9)), replace=False)
            rob.sphere_frame = rob.sphere_frame[keep]
            rob.sphere_xyzr = rob.sphere_xyzr[keep]
        else:
            rob = planar_2link(rng.uniform(0.1, 0.4), rng.uniform(0.1, 0.4),
                               W.frame12(W.rot_z(rng.uniform(-3, 3)), (rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5), 0)))
            rob.sphere_xyzr[:, 3] = rng.uniform(0.03, 0.12, 2)
            rob.self_pairs = np.array([[0, 1]], np.int32) if rng.random() < 0.3 else np.zeros((0, 2), np.int32)
        team.append(rob)
    return team


def tiny_env(rng):
    sph = np.column_stack([rng.uniform(-1, 1, (3, 2)), np.zeros(3), rng.uniform(0.02, 0.1, 3)])
    boxes = np.zeros((2, 15))
    for i in range(2):
        boxes[i, :3] = rng.uniform(-1, 1, 3) * [1, 1, 0.1]
        boxes[i, 3:12] = W.random_rotation(rng).ravel()
        boxes[i, 12:] = rng.uniform(0.05, 0.2, 3)
    cyl = np.zeros((1, 8))
    cyl[0, :3] = rng.uniform(-1, 1, 3) * [1, 1, 0.1]
    cyl[0, 3:6] = W.random_unit(rng)
    cyl[0, 6:] = rng.uniform(0.05, 0.3, 2)
    return W.Env(spheres=sph, boxes=boxes, cylinders=cyl, points=rng.uniform(-1, 1, (20, 3)) * [1, 1, 0.05],
                 point_radius=0.01)


def tiny_paths(rng, team, nq, t_max):
    per_q = []
    for _ in range(nq):
        rows = []
        for rob in team:
            L = int(rng.integers(1, t_max + 1))
            K = int(rng.integers(1, 4))
            if L == 1 or K == 1:
                times = np.array([0]) if L == 1 or rng.random() < 0.5 else np.array([0, L - 1])
            else:
                inner = np.sort(rng.choice(np.arange(1, L - 1), size=min(K - 2, L - 2), replace=False)) if K > 2 and L > 2 else []
                times = np.concatenate([[0], inner, [L - 1]]).astype(int)
            lo = np.where(rob.joint_type == W.REV_Z, -3.0, -1.0)
            hi = -lo
            rows.append((times, rng.uniform(lo, hi, (len(times), rob.dof))))
        per_q.append(rows)
    return W.paths_from_lists(per_q, 3)


@pytest.mark.parametrize("seed", range(6))
def test_oracle_matches_brute_force_tiny(seed):
    rng = np.random.default_rng(100 + seed)
    n_checked_hits = 0
    for _ in range(6):
        team = tiny_team(rng, int(rng.integers(1, 4)))
        env = tiny_env(rng)
        paths = tiny_paths(rng, team, 12, 16)
        ot, oe, op = oracle.Team(team), oracle.Env(env), oracle.Paths(paths)
        mv_env = oracle.mv(ot, oe, op, check_env=True)
        mv_noenv = oracle.mv(ot, oe, op, check_env=False)
        ff = oracle.ffc(ot, op)
        for q in range(paths.n_queries):
            assert bool(mv_env[q]) == brute.mv(team, env, paths, q, True)
            assert bool(mv_noenv[q]) == brute.mv(team, env, paths, q, False)
            assert tuple(ff[q]) == brute.ffc(team, paths, q)
            n_checked_hits += int(ff[q, 0] >= 0)
    assert n_checked_hits > 0


# ----------------------------------------------------------------------------- invariants

@pytest.fixture(scope="module")
def arms_small():
    w = W.arms_workload(192)
    return w, oracle.Team(w.team), oracle.Env(w.env), oracle.Paths(w.paths)


def test_invariant_mv_noenv_iff_ffc_null_and_conflict_implies_invalid(arms_small):
    w, ot, oe, op = arms_small
    v_noenv = oracle.mv(ot, oe, op, check_env=False)
    v_env = oracle.mv(ot, oe, op, check_env=True)
    ff = oracle.ffc(ot, op)
    assert np.array_equal(v_noenv.astype(bool), ff[:, 0] < 0)
    assert not np.any(v_env.astype(bool) & (ff[:, 0] >= 0))
    assert 0 < (ff[:, 0] >= 0).sum() < len(ff)


def test_invariant_robot_swap_symmetry(arms_small):
    w, ot, oe, op = arms_small
    ff = oracle.ffc(ot, op)
    perm = [2, 0, 3, 1]
    team2 = [w.team[i] for i in perm]
    p2 = W.paths_from_lists([[w.paths.path(q, i) for i in perm] for q in range(w.paths.n_queries)], 7)
    ff2 = oracle.ffc(oracle.Team(team2), oracle.Paths(p2))
    assert np.array_equal(ff[:, 0], ff2[:, 0])
    v1 = oracle.mv(ot, oe, op)
    v2 = oracle.mv(oracle.Team(team2), oe, oracle.Paths(p2))
    assert np.array_equal(v1, v2)
    # the conflicting pair at t* is a colliding pair in both labelings
    inv = {p: k for k, p in enumerate(perm)}
    for q in np.nonzero(ff[:, 0] >= 0)[0][:20]:
        i2, j2 = ff2[q, 1], ff2[q, 2]
        a, b = sorted((perm[i2], perm[j2]))
        t = ff[q, 0]
        sph = oracle.team_spheres(ot, op, int(q), int(t))
        hits = brute.rr_hits([sph[ot.sphere_off[r]:ot.sphere_off[r + 1]] for r in range(4)])
        assert (a, b) in hits and (ff[q, 1], ff[q, 2]) == min(hits)
        assert inv[a] < 4


def dense(paths, q, team):
    rows = []
    T = int(paths.horizon()[q])
    for r, rob in enumerate(team):
        times, cfgs = paths.path(q, r)
        L = int(times[-1]) + 1
        states = np.stack([oracle.path_state(times, cfgs, paths.dof_stride, t) for t in range(L)])
        rows.append((np.arange(L), states))
    return rows, T


def test_invariant_prefix_truncation_and_time_shift(arms_small):
    w, ot, oe, op = arms_small
    ff = oracle.ffc(ot, op)
    hit_q = [q for q in range(len(ff)) if ff[q, 0] > 2][:12]
    assert hit_q
    trunc, shifted, shift = [], [], []
    for q in hit_q:
        rows, T = dense(w.paths, q, w.team)
        ts = int(ff[q, 0])
        trunc.append([(np.arange(min(ts, len(t))), c[:min(ts, len(t))]) if min(ts, len(t)) > 0
                      else (np.arange(1), c[:1]) for (t, c) in rows])
        k = int(1 + q % 5)
        shift.append(k)
        sh = []
        for r in range(len(w.team)):
            times, cfgs = w.paths.path(q, r)
            sh.append((np.concatenate([[0], times + k]), np.concatenate([cfgs[:1], cfgs])))
        shifted.append(sh)
    f_tr = oracle.ffc(ot, oracle.Paths(W.paths_from_lists(trunc, 7)))
    assert np.all(f_tr[:, 0] == -1)
    f_sh = oracle.ffc(ot, oracle.Paths(W.paths_from_lists(shifted, 7)))
    assert np.array_equal(f_sh[:, 0], ff[hit_q, 0] + np.array(shift))
    assert np.array_equal(f_sh[:, 1:], ff[hit_q, 1:])
    # dense resampling reproduces the same states, hence the same answer
    dense_q = [dense(w.paths, q, w.team)[0] for q in hit_q]
    f_dn = oracle.ffc(ot, oracle.Paths(W.paths_from_lists(dense_q, 7)))
    assert np.array_equal(f_dn, ff[hit_q])


def test_invariant_zero_length_and_single_robot():
    w = W.arms_workload(64)
    ot, oe = oracle.Team(w.team), oracle.Env(w.env)
    rows = [[(np.array([0]), w.paths.path(q, r)[1][:1]) for r in range(4)] for q in range(64)]
    p0 = W.paths_from_lists(rows, 7)
    v = oracle.mv(ot, oe, oracle.Paths(p0))
    for q in range(64):
        sph = oracle.team_spheres(ot, oracle.Paths(p0), q, 0)
        per = [sph[ot.sphere_off[r]:ot.sphere_off[r + 1]] for r in range(4)]
        env_bad = any(brute.env_hit(w.team, w.env, per, r) for r in range(4))
        assert bool(v[q]) == (not env_bad and not brute.rr_hits(per))
    one = oracle.Team(w.team[:1])
    p1 = W.paths_from_lists([[w.paths.path(q, 0)] for q in range(64)], 7)
    assert np.all(oracle.ffc(one, oracle.Paths(p1))[:, 0] == -1)
    assert np.all(oracle.mv(one, oe, oracle.Paths(p1), check_env=False) == 1)


def test_touching_is_not_a_collision_and_first_overlap_closed_form():
    """Contact at clearance exactly 0 is free (a collision needs a negative
    clearance, §II-B); the first overlapping step of a linear approach and the
    lexicographic order of FFC's (t, i, j) follow by hand."""
    T = 64
    w = W.grazing_disks(9, T)
    ot, op = oracle.Team(w.team), oracle.Paths(w.paths)
    v = oracle.mv(ot, None, op, check_env=False)
    assert list(v) == [1, 0, 0] * 3
    f = oracle.ffc(ot, op)
    # disk 1 at x = 0.5 - 0.25 (t - T/2) / (T/2 - 1) clears disk 0 by x - 0.5 < 0 from t = T/2 + 1
    want = [(-1, -1, -1), (T // 2 + 1, 0, 1), (0, 0, 2)] * 3
    assert [tuple(r) for r in f] == want


def test_exhaustive_scan_gives_the_same_answers():
    """Evaluating every relation at every state (exhaustive validation) changes
    the work, not MV's answer or the first colliding timestep."""
    w = W.arms_workload(96)
    ot, oe, op = oracle.Team(w.team), oracle.Env(w.env), oracle.Paths(w.paths)
    for check_env in (True, False):
        v0, f0 = oracle.mv(ot, oe, op, check_env=check_env, first_hit=True)
        v1, f1 = oracle.mv(ot, oe, op, check_env=check_env, first_hit=True, exhaustive=True)
        assert np.array_equal(v0, v1) and np.array_equal(f0, f1)


# ----------------------------------------------------------------------------- prioritised MV

def _mask(robots):
    return sum(1 << r for r in robots)


@pytest.mark.parametrize("seed", range(4))
def test_focus_matches_brute_force_tiny(seed):
    """Prioritised MV (§III-C, PP-ST-RRT): the oracle against the brute-force
    definition (obstacle and self tests of the robots in focus, robot pairs with
    a robot in focus) for random focus sets."""
    rng = np.random.default_rng(700 + seed)
    n_diff = 0
    for _ in range(5):
        n = int(rng.integers(2, 4))
        team = tiny_team(rng, n)
        env = tiny_env(rng)
        paths = tiny_paths(rng, team, 10, 14)
        ot, oe, op = oracle.Team(team), oracle.Env(env), oracle.Paths(paths)
        full = oracle.mv(ot, oe, op, check_env=True)
        for _ in range(3):
            F = [r for r in range(n) if rng.random() < 0.5] or [int(rng.integers(0, n))]
            for check_env in (True, False):
                got = oracle.mv(ot, oe, op, check_env=check_env, focus=_mask(F))
                for q in range(paths.n_queries):
                    assert bool(got[q]) == brute.mv(team, env, paths, q, check_env, focus=F)
            n_diff += int(np.sum(oracle.mv(ot, oe, op, focus=_mask(F)) != full))
    assert n_diff > 0       # some focus sets must drop a collision the full check sees


def test_focus_decomposes_full_mv(arms_small):
    """Every relation of MV belongs to the focus set of one of its robots, so a
    motion is valid iff it is valid with each single robot in focus; a larger
    focus set can only invalidate more."""
    w, ot, oe, op = arms_small
    for check_env in (True, False):
        full = oracle.mv(ot, oe, op, check_env=check_env)
        single = [oracle.mv(ot, oe, op, check_env=check_env, focus=1 << r) for r in range(4)]
        assert np.array_equal(full, np.logical_and.reduce(single).astype(np.uint8))
        pair01 = oracle.mv(ot, oe, op, check_env=check_env, focus=0b0011)
        assert np.all(pair01 <= single[0]) and np.all(pair01 <= single[1])
        assert np.array_equal(oracle.mv(ot, oe, op, check_env=check_env, focus=0b1111), full)
        assert np.array_equal(oracle.mv(ot, oe, op, check_env=check_env, focus=0), full)
        assert any(not np.array_equal(s, full) for s in single)


def test_focus_skips_pairs_of_fixed_robots():
    """Three disks of radius 0.1 (contact at centre distance 0.2): disks 1 and 2
    overlap at every step (fixed, higher-priority paths that collide with each
    other); disk 0 sweeps along y = y0 and passes disk 1 at t = 5 at distance
    0.5 - y0: clear for y0 = 0.25, a collision for y0 = 0.35."""
    team = [W.disk_robot(0.1, f"d{k}") for k in range(3)]
    ot = oracle.Team(team)

    def paths(y0):
        rows = [(np.array([0, 10]), np.array([[-1.0, y0], [1.0, y0]])),     # disk 0 sweeps x in [-1, 1]
                (np.array([0]), np.array([[0.0, 0.5]])),                    # disk 1 rests at (0, 0.5)
                (np.array([0]), np.array([[0.05, 0.5]]))]                   # disk 2 rests 0.05 from disk 1
        return W.paths_from_lists([rows], 2)

    clear, hit = oracle.Paths(paths(0.25)), oracle.Paths(paths(0.35))
    assert oracle.mv(ot, None, clear, check_env=False, focus=0b001)[0] == 1
    assert oracle.mv(ot, None, clear, check_env=False, focus=0b011)[0] == 0       # pair (1, 2) collides
    assert oracle.mv(ot, None, clear, check_env=False, focus=0b010)[0] == 0
    assert oracle.mv(ot, None, clear, check_env=False)[0] == 0
    assert oracle.mv(ot, None, hit, check_env=False, focus=0b001)[0] == 0
    assert oracle.mv(ot, None, hit, check_env=False, focus=0b100)[0] == 0      # pair (1, 2)
