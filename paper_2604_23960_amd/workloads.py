"""Seeded synthetic workloads for multi-robot motion validation.

This module builds *inputs only*: robot sphere models, obstacle sets and timed
waypoint paths.  It performs no forward kinematics and no collision test, so
it shares none of the validation arithmetic with either the FP64 oracle or
the GPU path; both of them consume what it produces.

Problem shape (paper §III-A, Alg. 1 input; §III-B, Alg. 2 input): a team of
robots, each a set of spheres attached to the links of a kinematic chain
(§II-B), an obstacle set, and one path per robot.  A path is a list of timed
waypoints ``(tau_k, Q_k)``; the robot's state at integer timestep ``t`` is the
linear interpolation between the waypoints around ``t`` and the last waypoint
once ``t`` passes the end (padding, §III-A).  Straight-line motions are
discretised so that no robot moves more than ``step`` per timestep and all
robots start and stop together (§IV-A, implementations).

Model conventions (shared by every consumer of these arrays):

* joint types: ``REV_Z`` rotation about the local z axis by ``q``;
  ``PRI_X/PRI_Y/PRI_Z`` translation by ``q`` along the local axis.
* ``joint_fixed[k]`` is a 3x4 row-major transform ``F_k`` applied before the
  joint motion: ``Frame_0 = base``, ``Frame_k = Frame_{k-1} F_k J_k(q_k)``.
* ``sphere_frame[s]`` in ``0..n_joints`` (0 = base) and ``sphere_xyzr[s]`` the
  sphere centre in that frame plus its radius.
* ``self_pairs`` lists sphere index pairs (within one robot) that count as
  self-collision.

Every array is generated from ``numpy.random.default_rng([seed, stream])``
with separate streams for the team, the environment and the workload.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

REV_Z, PRI_X, PRI_Y, PRI_Z = 0, 1, 2, 3
STREAM_TEAM, STREAM_ENV, STREAM_WORK = 1, 2, 3

ARM_SPHERES = 60
ARM_LIMIT = 2.9
RECT_DIMS = (0.4, 0.2)
RECT_GRID = (6, 2)


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([seed, stream])


# ----------------------------------------------------------------------------
# small transform builders (model construction, not kinematics)

def rot_x(a: float) -> np.ndarray:
    c, s = math.cos(a), math.sin(a)
    return np.array([[1.0, 0.0, 0.0], [0.0, c, -s], [0.0, s, c]])


def rot_z(a: float) -> np.ndarray:
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def frame12(R: np.ndarray, p) -> np.ndarray:
    out = np.zeros(12)
    out.reshape(3, 4)[:, :3] = R
    out.reshape(3, 4)[:, 3] = p
    return out


IDENTITY12 = frame12(np.eye(3), (0.0, 0.0, 0.0))


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform random rotation from a normalised Gaussian quaternion."""
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def random_unit(rng: np.random.Generator) -> np.ndarray:
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


# ----------------------------------------------------------------------------
# robot models

@dataclass
class Robot:
    name: str
    joint_type: np.ndarray          # int32 [nj]
    joint_fixed: np.ndarray         # float64 [nj, 12]
    sphere_frame: np.ndarray        # int32 [ns]
    sphere_xyzr: np.ndarray         # float64 [ns, 4]
    self_pairs: np.ndarray          # int32 [np, 2]
    base: np.ndarray                # float64 [12]
    q_lo: np.ndarray                # float64 [nj]
    q_hi: np.ndarray                # float64 [nj]
    meta: dict = field(default_factory=dict)

    @property
    def dof(self) -> int:
        return int(self.joint_type.shape[0])

    @property
    def n_spheres(self) -> int:
        return int(self.sphere_xyzr.shape[0])

    def with_base(self, base: np.ndarray, name: str | None = None) -> "Robot":
        return Robot(name or self.name, self.joint_type.copy(), self.joint_fixed.copy(),
                     self.sphere_frame.copy(), self.sphere_xyzr.copy(), self.self_pairs.copy(),
                     np.asarray(base, dtype=np.float64).copy(), self.q_lo.copy(), self.q_hi.copy(),
                     dict(self.meta))


def _largest_remainder(weights: np.ndarray, total: int, minimum: int) -> np.ndarray:
    n = len(weights)
    counts = np.full(n, minimum, dtype=np.int64)
    rest = total - minimum * n
    share = weights / weights.sum() * rest
    base = np.floor(share).astype(np.int64)
    counts += base
    left = rest - int(base.sum())
    order = np.argsort(-(share - base), kind="stable")
    counts[order[:left]] += 1
    return counts


def dh_arm(rng: np.random.Generator, name: str, n_spheres: int = ARM_SPHERES) -> Robot:
    """Seeded 7-revolute arm in standard DH form (a, d ~ U[0, 0.35], alpha in {0, +-pi/2}).

    Standard DH ``T_k = Rz(theta_k) Tz(d_k) Tx(a_k) Rx(alpha_k)`` written in
    chain form: ``F_1 = I`` and ``F_k = Tz(d_{k-1}) Tx(a_{k-1}) Rx(alpha_{k-1})``,
    so link k's geometry lives in ``Frame_k`` on the polyline
    (0,0,0) -> (0,0,d_k) -> (a_k,0,d_k).  Spheres are spread over the links by
    arc length (largest remainder, at least one per link), evenly spaced, with
    radii U[0.03, 0.08].
    """
    nj = 7
    a = rng.uniform(0.0, 0.35, nj)
    d = rng.uniform(0.0, 0.35, nj)
    alpha = rng.choice(np.array([0.0, math.pi / 2, -math.pi / 2]), nj)
    joint_fixed = np.zeros((nj, 12))
    joint_fixed[0] = IDENTITY12
    for k in range(1, nj):
        joint_fixed[k] = frame12(rot_x(alpha[k - 1]), (a[k - 1], 0.0, d[k - 1]))
    lengths = a + d
    counts = _largest_remainder(lengths, n_spheres, 1)
    frames, xyzr = [], []
    for k in range(nj):
        n_k = int(counts[k])
        for m in range(n_k):
            s = (m + 0.5) / n_k * lengths[k]
            if s <= d[k]:
                c = (0.0, 0.0, s)
            else:
                c = (s - d[k], 0.0, d[k])
            frames.append(k + 1)
            xyzr.append((c[0], c[1], c[2], rng.uniform(0.03, 0.08)))
    sphere_frame = np.asarray(frames, dtype=np.int32)
    sphere_xyzr = np.asarray(xyzr, dtype=np.float64)
    # Self-collision pairs: spheres on links at least three joints apart.
    ia, ib = np.nonzero(sphere_frame[None, :] - sphere_frame[:, None] >= 3)
    self_pairs = np.stack([ia, ib], axis=1).astype(np.int32)
    return Robot(name, np.full(nj, REV_Z, np.int32), joint_fixed, sphere_frame, sphere_xyzr,
                 self_pairs, IDENTITY12.copy(), np.full(nj, -ARM_LIMIT), np.full(nj, ARM_LIMIT),
                 dict(kind="arm", a=a, d=d, alpha=alpha))


def disk_robot(radius: float = 0.05, name: str = "disk") -> Robot:
    """Planar disk: PRI_X, PRI_Y, one sphere at the origin (mobile robot at z=0)."""
    return Robot(name, np.array([PRI_X, PRI_Y], np.int32), np.stack([IDENTITY12, IDENTITY12]),
                 np.array([2], np.int32), np.array([[0.0, 0.0, 0.0, radius]]),
                 np.zeros((0, 2), np.int32), IDENTITY12.copy(), np.zeros(2), np.ones(2),
                 dict(kind="disk"))


def se2_rect(z: float, name: str = "rect") -> Robot:
    """SE(2) rectangle 0.4 x 0.2 m covered by a 6 x 2 grid of spheres.

    Joints PRI_X, PRI_Y, REV_Z on a base at height ``z``; each sphere covers its
    grid cell (radius = half the cell diagonal).
    """
    lx, ly = RECT_DIMS
    nx, ny = RECT_GRID
    cx, cy = lx / nx, ly / ny
    rad = math.hypot(cx / 2, cy / 2)
    xyzr = []
    for i in range(nx):
        for j in range(ny):
            xyzr.append((-lx / 2 + cx * (i + 0.5), -ly / 2 + cy * (j + 0.5), 0.0, rad))
    return Robot(name, np.array([PRI_X, PRI_Y, REV_Z], np.int32),
                 np.stack([IDENTITY12] * 3), np.full(nx * ny, 3, np.int32),
                 np.asarray(xyzr), np.zeros((0, 2), np.int32), frame12(np.eye(3), (0, 0, z)),
                 np.array([-1.0, -1.0, -math.pi]), np.array([1.0, 1.0, math.pi]),
                 dict(kind="rect"))


def arm_base(x: float, y: float, z: float = 0.0, ceiling: bool = False) -> np.ndarray:
    """Base on (x, y, z) facing the square's centre; ceiling mounts are flipped by Rx(pi)."""
    yaw = math.atan2(-y, -x)
    if ceiling:
        # flipped about x: the arm hangs down; yaw is applied in the flipped frame so the
        # arm still faces the centre.
        R = rot_x(math.pi) @ rot_z(-yaw)
    else:
        R = rot_z(yaw)
    return frame12(R, (x, y, z))


CORNERS = [(0.5, 0.5), (-0.5, 0.5), (-0.5, -0.5), (0.5, -0.5)]


def arm_models(seed: int = 1) -> list[Robot]:
    """The four seeded 7-R arm models of the arm workload (seed 1)."""
    rng = _rng(seed, STREAM_TEAM)
    return [dh_arm(rng, f"arm{k}") for k in range(4)]


def arm_team(seed: int = 1) -> list[Robot]:
    return [m.with_base(arm_base(x, y)) for m, (x, y) in zip(arm_models(seed), CORNERS)]


def ring_radius(n_arms: int) -> float:
    """Base circle of a ring team: the arm workload's corner distance for four
    arms, else about 1 m between neighbouring bases."""
    return max(math.hypot(*CORNERS[0]), n_arms / (2.0 * math.pi))


def ring_team(n_arms: int, seed: int = 1) -> list[Robot]:
    """n_arms copies of the four seeded arm models (cycled) on a circle, facing
    its centre; four arms sit on the arm workload's corners."""
    models = arm_models(seed)
    R = ring_radius(n_arms)
    team = []
    for k in range(n_arms):
        ang = math.pi / 4 + 2.0 * math.pi * k / n_arms
        x, y = R * math.cos(ang), R * math.sin(ang)
        team.append(models[k % 4].with_base(arm_base(x, y), f"arm{k}"))
    return team


# ----------------------------------------------------------------------------
# environments

@dataclass
class Env:
    spheres: np.ndarray = field(default_factory=lambda: np.zeros((0, 4)))     # [n,4] xyz r
    boxes: np.ndarray = field(default_factory=lambda: np.zeros((0, 15)))      # [n,15] c, R(9), h(3)
    cylinders: np.ndarray = field(default_factory=lambda: np.zeros((0, 8)))   # [n,8] c, u, hl, R
    points: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))      # [n,3]
    point_radius: float = 0.0


def circles_env(seed: int = 0, n: int = 16) -> Env:
    rng = _rng(seed, STREAM_ENV)
    c = rng.uniform(0.0, 1.0, (n, 2))
    r = rng.uniform(0.02, 0.08, n)
    return Env(spheres=np.column_stack([c, np.zeros(n), r]))


def cube_env(seed: int = 1, n_boxes: int = 20, n_cyl: int = 8) -> Env:
    """Boxes and cylinders in the cube [-1,1]^2 x [0,2]."""
    rng = _rng(seed, STREAM_ENV)
    lo, hi = np.array([-1.0, -1.0, 0.0]), np.array([1.0, 1.0, 2.0])
    boxes = np.zeros((n_boxes, 15))
    for i in range(n_boxes):
        boxes[i, 0:3] = rng.uniform(lo, hi)
        boxes[i, 3:12] = random_rotation(rng).reshape(-1)
        boxes[i, 12:15] = rng.uniform(0.05, 0.25, 3)
    cyl = np.zeros((n_cyl, 8))
    for i in range(n_cyl):
        cyl[i, 0:3] = rng.uniform(lo, hi)
        cyl[i, 3:6] = random_unit(rng)
        cyl[i, 6] = rng.uniform(0.1, 0.5)
        cyl[i, 7] = rng.uniform(0.03, 0.10)
    return Env(boxes=boxes, cylinders=cyl)


# ----------------------------------------------------------------------------
# paths

@dataclass
class Paths:
    """Query-major CSR over per-robot waypoint lists."""
    n_queries: int
    n_robots: int
    dof_stride: int
    wp_begin: np.ndarray   # int64 [n_queries * n_robots + 1]
    wp_t: np.ndarray       # int32 [n_wp]
    wp_q: np.ndarray       # float64 [n_wp, dof_stride]

    def path(self, q: int, r: int):
        b, e = self.wp_begin[q * self.n_robots + r], self.wp_begin[q * self.n_robots + r + 1]
        return self.wp_t[b:e], self.wp_q[b:e]

    def horizon(self) -> np.ndarray:
        """Per-query T = max over robots of (last waypoint time + 1)."""
        last = self.wp_t[self.wp_begin[1:] - 1].astype(np.int64) + 1
        return last.reshape(self.n_queries, self.n_robots).max(axis=1)

    def subset(self, queries) -> "Paths":
        queries = np.asarray(queries, dtype=np.int64)
        return paths_from_lists([[self.path(q, r) for r in range(self.n_robots)] for q in queries],
                                self.dof_stride)


def paths_from_lists(per_query, dof_stride: int) -> Paths:
    """Build CSR paths from ``per_query[q][r] = (times, configs)``."""
    nq = len(per_query)
    nr = len(per_query[0]) if nq else 0
    begin = [0]
    ts, qs = [], []
    for qi in per_query:
        for (t, c) in qi:
            t = np.asarray(t, dtype=np.int32)
            c = np.asarray(c, dtype=np.float64).reshape(len(t), -1)
            pad = np.zeros((len(t), dof_stride))
            pad[:, :c.shape[1]] = c
            ts.append(t)
            qs.append(pad)
            begin.append(begin[-1] + len(t))
    wp_t = np.concatenate(ts) if ts else np.zeros(0, np.int32)
    wp_q = np.concatenate(qs) if qs else np.zeros((0, dof_stride))
    return Paths(nq, nr, dof_stride, np.asarray(begin, dtype=np.int64), wp_t.astype(np.int32),
                 np.ascontiguousarray(wp_q))


def steps_for(dq: np.ndarray, step: float, metric: str) -> int:
    """Timesteps needed so a robot moves at most ``step`` per timestep (L2 or Linf)."""
    if metric == "l2":
        d = math.sqrt(float(np.sum(np.asarray(dq, dtype=np.float64) ** 2)))
    else:
        d = float(np.max(np.abs(dq))) if len(dq) else 0.0
    return int(math.ceil(d / step))


def straight_line_paths(starts: np.ndarray, goals: np.ndarray, dofs, step: float, metric: str,
                        dof_stride: int) -> Paths:
    """Composite straight-line motions: every robot moves S_i -> G_i over the same n steps.

    ``starts``/``goals`` are [Q, n_robots, dof_stride]; n = max_i ceil(d_i/step).
    n = 0 gives a single waypoint (one state).
    """
    nq, nr = starts.shape[:2]
    per_query = []
    for q in range(nq):
        n = max(steps_for(goals[q, r, :dofs[r]] - starts[q, r, :dofs[r]], step, metric)
                for r in range(nr))
        if n == 0:
            per_query.append([(np.array([0]), starts[q, r:r + 1, :dofs[r]]) for r in range(nr)])
        else:
            per_query.append([(np.array([0, n]), np.stack([starts[q, r, :dofs[r]],
                                                          goals[q, r, :dofs[r]]]))
                              for r in range(nr)])
    return paths_from_lists(per_query, dof_stride)


def sample_configs(rng: np.random.Generator, team: list[Robot], n: int, dof_stride: int) -> np.ndarray:
    out = np.zeros((n, len(team), dof_stride))
    for r, rob in enumerate(team):
        out[:, r, :rob.dof] = rng.uniform(rob.q_lo, rob.q_hi, (n, rob.dof))
    return out


def valid_configs(rng: np.random.Generator, team: list[Robot], n: int, dof_stride: int, decide,
                  batch: int = 8192, max_rounds: int = 256) -> tuple[np.ndarray, dict]:
    """n team configurations valid as single states, by the valid-endpoint protocol
    of the paper's experiments (§IV-A): per-robot configurations uniform in the
    joint limits are kept when valid for that robot alone (its self and obstacle
    tests), then composed at random and kept when the whole team's state is
    valid.  ``decide(robots, configs)`` returns, for configs [m, len(robots),
    dof_stride], whether each state is valid; it is the caller's validity test
    (the library or the oracle), so this module holds no collision arithmetic.
    Returns [n, len(team), dof_stride] and the acceptance rates."""
    alone, acc_alone = [], []
    for rob in team:
        good, tried = [], 0
        while sum(len(g) for g in good) < min(n, batch) and tried < max_rounds * batch:
            cand = sample_configs(rng, [rob], batch, dof_stride)
            good.append(cand[np.asarray(decide([rob], cand), bool)])
            tried += batch
        pool = np.concatenate(good)[:, 0, :]
        if len(pool) == 0:
            raise RuntimeError(f"no configuration of {rob.name} is valid alone")
        alone.append(pool)
        acc_alone.append(len(pool) / tried)
    kept, tried = [], 0
    while sum(len(k) for k in kept) < n and tried < max_rounds * batch:
        cand = np.stack([a[rng.integers(0, len(a), batch)] for a in alone], axis=1)
        kept.append(cand[np.asarray(decide(team, cand), bool)])
        tried += batch
    out = np.concatenate(kept)
    if len(out) < n:
        raise RuntimeError(f"only {len(out)} of {n} valid team configurations found")
    return out[:n], dict(alone=acc_alone, team=len(out) / tried)


def random_timed_paths(rng: np.random.Generator, team: list[Robot], n_queries: int,
                       len_lo: int, len_hi: int, k_lo: int, k_hi: int, dof_stride: int,
                       lengths: np.ndarray | None = None) -> Paths:
    """Independent piecewise-linear timed paths (decoupled planners' output shape).

    Per robot: L ~ U{len_lo..len_hi} states (or ``lengths[q, r]``), K ~ U{k_lo..k_hi}
    waypoints uniform in C-space, first at t=0, last at t=L-1, interior times
    distinct integers drawn uniformly from (0, L-1) and sorted.
    """
    per_query = []
    for q in range(n_queries):
        rows = []
        for r, rob in enumerate(team):
            L = int(lengths[q, r]) if lengths is not None else int(rng.integers(len_lo, len_hi + 1))
            K = int(rng.integers(k_lo, k_hi + 1))
            K = max(1, min(K, L))
            if L == 1 or K == 1:
                times = np.array([0]) if L == 1 else np.array([0, L - 1])
            else:
                inner = np.sort(rng.choice(np.arange(1, L - 1), size=min(K - 2, max(L - 2, 0)),
                                           replace=False)) if K > 2 else np.zeros(0, np.int64)
                times = np.concatenate([[0], inner, [L - 1]])
            cfg = rng.uniform(rob.q_lo, rob.q_hi, (len(times), rob.dof))
            rows.append((times, cfg))
        per_query.append(rows)
    return paths_from_lists(per_query, dof_stride)


# ----------------------------------------------------------------------------
# named workloads

@dataclass
class Workload:
    name: str
    team: list
    env: Env
    paths: Paths
    ops: str
    notes: str = ""


def _endpoints(rng, team, n, dof_stride, decide):
    """Start and goal configurations: uniform in the joint limits, or (decide given)
    valid team states drawn by valid_configs, starts first."""
    if decide is None:
        return sample_configs(rng, team, n, dof_stride), sample_configs(rng, team, n, dof_stride), None
    both, acc = valid_configs(rng, team, 2 * n, dof_stride, decide)
    return both[:n], both[n:], acc


def disks_workload(n_queries: int = 4096, seed: int = 0, decide=None) -> Workload:
    """Two disks (r=0.05) in the unit square among 16 circles; straight lines at 0.005
    L2 per step.  With ``decide`` (see valid_configs) the endpoints are valid states,
    uniform in collision-free space."""
    team = [disk_robot(0.05, "disk0"), disk_robot(0.05, "disk1")]
    env = circles_env(seed)
    rng = _rng(seed, STREAM_WORK)
    s, g, acc = _endpoints(rng, team, n_queries, 2, decide and (lambda rs, c: decide(rs, env, c)))
    paths = straight_line_paths(s, g, [2, 2], 0.005, "l2", 2)
    return Workload("disks-2r-16circles", team, env, paths, "mv+ffc",
                    notes="" if acc is None else f"valid endpoints, acceptance {acc}")


def arms_workload(n_queries: int = 65536, seed: int = 1, decide=None) -> Workload:
    """Four 7-R arms facing inward on a 1 m square; straight lines at 1/32 rad
    max-joint step.  With ``decide`` (see valid_configs) the endpoints are valid
    states (alone, then as a team)."""
    team = arm_team(seed)
    env = cube_env(seed)
    rng = _rng(seed, STREAM_WORK)
    s, g, acc = _endpoints(rng, team, n_queries, 7, decide and (lambda rs, c: decide(rs, env, c)))
    paths = straight_line_paths(s, g, [7] * 4, 1.0 / 32.0, "linf", 7)
    return Workload("arms-4x7R-60sph-20box-8cyl", team, env, paths, "mv",
                    notes="" if acc is None else f"valid endpoints, acceptance {acc}")


def hetero_team(seed_arms: int = 1, n_arms: int = 4, n_rects: int = 4, rect_z: float = 0.5,
                ceiling: bool = False) -> list[Robot]:
    models = arm_models(seed_arms)
    team = []
    for k in range(n_arms):
        x, y = CORNERS[k % 4]
        ceil_mount = ceiling and k >= 4
        team.append(models[k % 4].with_base(arm_base(x, y, 2.0 if ceil_mount else 0.0, ceil_mount),
                                            f"arm{k}"))
    for k in range(n_rects):
        team.append(se2_rect(rect_z, f"rect{k}"))
    return team


def ffc_workload(n_queries: int = 16384, seed: int = 2) -> Workload:
    """4 arms + 4 SE(2) rectangles with decoupled timed paths of 200-2000 states."""
    team = hetero_team(1, 4, 4, 0.5)
    env = cube_env(1)
    rng = _rng(seed, STREAM_WORK)
    paths = random_timed_paths(rng, team, n_queries, 200, 2000, 2, 8, 7)
    return Workload("ffc-4arm-4rect-200to2000", team, env, paths, "ffc")


def grazing_disks(n_queries: int = 300, T: int = 64) -> Workload:
    """Three disks of radius 0.25 with exact touching contacts, so most tests fall
    in the near-contact band.  Disk 0 rests at the origin; disks 1 and 2 touch it
    at (0.5, 0) and (0, 0.5) (clearance exactly 0, not a collision).  By query
    index mod 3: (0) all rest for T steps; (1) disk 1 rests until T/2, then moves
    to (0.25, 0), overlapping disk 0 from step T/2 + 1; (2) disk 2 overlaps disk 0
    at (0, 0.3) throughout."""
    team = [disk_robot(0.25, f"disk{k}") for k in range(3)]
    env = Env()
    rest0 = ([0, T - 1], [[0.0, 0.0], [0.0, 0.0]])
    touch1 = ([0, T - 1], [[0.5, 0.0], [0.5, 0.0]])
    touch2 = ([0, T - 1], [[0.0, 0.5], [0.0, 0.5]])
    move1 = ([0, T // 2, T - 1], [[0.5, 0.0], [0.5, 0.0], [0.25, 0.0]])
    over2 = ([0, T - 1], [[0.0, 0.3], [0.0, 0.3]])
    per = []
    for q in range(n_queries):
        per.append([rest0, touch1, touch2] if q % 3 == 0 else
                   [rest0, move1, touch2] if q % 3 == 1 else [rest0, touch1, over2])
    return Workload("grazing-3disks", team, env, paths_from_lists(per, 2), "mv+ffc")


def small(w_fn, n_queries: int, **kw) -> Workload:
    return w_fn(n_queries=n_queries, **kw)


# ----------------------------------------------------------------------------
# serving workload: many planner clients with resident teams

@dataclass
class ServeRequest:
    client: int
    kind: int            # 0 MV, 1 FFC
    paths: Paths         # one query
    horizon: int


def serving_workload(n_requests: int, n_clients: int = 64, seed: int = 3, mv_fraction: float = 0.7,
                     t_lo: int = 8, t_hi: int = 4096):
    """Clients with teams of 2-8 robots drawn from the arm models (distinct corners)
    and SE(2) rectangles, the cube obstacles, and single-query requests:
    MV straight-line motions with T ~ round(log-uniform[t_lo, t_hi]) states, FFC
    timed paths with per-robot lengths U[ceil(T/2), T] (one robot exactly T).
    Returns (teams, env, requests)."""
    rng_t = _rng(seed, STREAM_TEAM)
    models = arm_models(1)
    teams = []
    for _ in range(n_clients):
        n = int(rng_t.integers(2, 9))
        n_arms = int(rng_t.integers(0, min(4, n) + 1))
        corners = rng_t.permutation(4)[:n_arms]
        team = []
        for k, c in enumerate(corners):
            x, y = CORNERS[int(c)]
            team.append(models[int(c)].with_base(arm_base(x, y), f"arm{k}"))
        for k in range(n - n_arms):
            team.append(se2_rect(0.5, f"rect{k}"))
        teams.append(team)
    env = cube_env(1)
    rng = _rng(seed, STREAM_WORK)
    reqs = []
    for _ in range(n_requests):
        client = int(rng.integers(0, n_clients))
        team = teams[client]
        T = int(round(math.exp(rng.uniform(math.log(t_lo), math.log(t_hi)))))
        if rng.random() < mv_fraction:
            s = sample_configs(rng, team, 1, 7)[0]
            g = sample_configs(rng, team, 1, 7)[0]
            rows = [(np.array([0, T - 1]), np.stack([s[r, :rob.dof], g[r, :rob.dof]])) for r, rob in enumerate(team)]
            reqs.append(ServeRequest(client, 0, paths_from_lists([rows], 7), T))
        else:
            lengths = rng.integers((T + 1) // 2, T + 1, (1, len(team)))
            lengths[0, int(rng.integers(0, len(team)))] = T
            p = random_timed_paths(rng, team, 1, 0, 0, 2, 4, 7, lengths=lengths)
            reqs.append(ServeRequest(client, 1, p, T))
    return teams, env, reqs


# ----------------------------------------------------------------------------
# large heterogeneous workload (vectorised generation)

def box_surface_cloud(seed: int = 4, n_boxes: int = 40, n_points: int = 200_000,
                      point_radius: float = 0.005) -> Env:
    """Points uniform over the surfaces of random boxes (area-weighted) in the cube
    [-1,1]^2 x [0,2]; box centres uniform, half-extents U[0.05, 0.3], random rotation."""
    rng = _rng(seed, STREAM_ENV)
    lo, hi = np.array([-1.0, -1.0, 0.0]), np.array([1.0, 1.0, 2.0])
    cen = rng.uniform(lo, hi, (n_boxes, 3))
    ext = rng.uniform(0.05, 0.3, (n_boxes, 3))
    rot = np.stack([random_rotation(rng) for _ in range(n_boxes)])
    # faces: axis k, sign +-1; area of a face normal to k = 4 * h_j * h_l
    face_area = np.zeros((n_boxes, 6))
    for k in range(3):
        j, l = [a for a in range(3) if a != k]
        face_area[:, 2 * k] = face_area[:, 2 * k + 1] = 4.0 * ext[:, j] * ext[:, l]
    w = face_area.ravel() / face_area.sum()
    pick = rng.choice(len(w), size=n_points, p=w)
    b, f = pick // 6, pick % 6
    k, sgn = f // 2, np.where(f % 2 == 0, 1.0, -1.0)
    local = rng.uniform(-1.0, 1.0, (n_points, 3)) * ext[b]
    local[np.arange(n_points), k] = sgn * ext[b, k]
    pts = np.einsum("nij,nj->ni", rot[b], local) + cen[b]
    return Env(points=pts, point_radius=point_radius)


def _csr_from_times(times_list, cfg_list, dof_stride):
    """Concatenate per-path waypoint arrays (already in query-major path order)."""
    counts = np.array([len(t) for t in times_list], dtype=np.int64)
    begin = np.concatenate([[0], np.cumsum(counts)])
    wp_t = np.concatenate(times_list).astype(np.int32)
    wp_q = np.concatenate(cfg_list)
    return begin, wp_t, wp_q


def straight_line_paths_T(rng, team, T: np.ndarray, dof_stride: int) -> Paths:
    """Straight lines with given per-query horizons T (states): waypoints (0, S), (T-1, G)."""
    nq, nr = len(T), len(team)
    s = sample_configs(rng, team, nq, dof_stride)
    g = sample_configs(rng, team, nq, dof_stride)
    two = T > 1
    counts = np.where(two, 2, 1)
    per_path = np.repeat(counts, nr)
    begin = np.concatenate([[0], np.cumsum(per_path)]).astype(np.int64)
    n_wp = int(begin[-1])
    wp_t = np.zeros(n_wp, np.int32)
    wp_q = np.zeros((n_wp, dof_stride))
    first = begin[:-1]
    wp_q[first] = s.reshape(nq * nr, dof_stride)
    sec = first[np.repeat(two, nr)] + 1
    wp_t[sec] = np.repeat(T[two] - 1, nr)
    wp_q[sec] = g[two].reshape(-1, dof_stride)
    return Paths(nq, nr, dof_stride, begin, wp_t, wp_q)


def stratified_timed_paths(rng, team, lengths: np.ndarray, k_lo: int, k_hi: int, dof_stride: int) -> Paths:
    """Timed paths with given per-(query, robot) lengths L: K ~ U{k_lo..k_hi}
    waypoints, times 0 = tau_0 < ... < tau_{K-1} = L-1 placed one per equal slice
    of [0, L-1] with a uniform jitter inside the slice, configurations uniform in
    C-space."""
    nq, nr = lengths.shape
    L = lengths.reshape(-1).astype(np.int64)
    K = rng.integers(k_lo, k_hi + 1, L.shape[0])
    # at least two states per slice so the jittered times stay strictly increasing
    K = np.minimum(K, (L - 1) // 2 + 1)
    K = np.where(L == 1, 1, np.maximum(K, 2))
    begin = np.concatenate([[0], np.cumsum(K)]).astype(np.int64)
    n_wp = int(begin[-1])
    path = np.repeat(np.arange(L.shape[0]), K)
    idx = np.arange(n_wp) - begin[path]
    Kp, Lp = K[path], L[path]
    seg = (Lp - 1) / np.maximum(Kp - 1, 1)
    jitter = rng.uniform(-0.2, 0.2, n_wp) * seg
    t = np.floor(idx * seg + jitter).astype(np.int64)
    t = np.where(idx == Kp - 1, Lp - 1, t)
    t = np.where(idx == 0, 0, t)
    wp_q = np.zeros((n_wp, dof_stride))
    robot = path % nr
    for r, rob in enumerate(team):
        sel = robot == r
        wp_q[sel, :rob.dof] = rng.uniform(rob.q_lo, rob.q_hi, (int(sel.sum()), rob.dof))
    return Paths(nq, nr, dof_stride, begin, t.astype(np.int32), wp_q)


def big_hetero_workload(n_queries: int = 262_144, seed: int = 4):
    """16 robots (the four arm models on floor and ceiling corners + 8 SE(2)
    rectangles at z = 1.0), a 200k-point box-surface cloud, horizons
    T ~ U{16..1024}; half MV straight lines (environment on), half FFC timed paths
    with per-robot lengths U{16..T} (one robot exactly T).
    Returns (team, env, mv_paths, ffc_paths)."""
    team = hetero_team(1, 8, 8, 1.0, ceiling=True)
    env = box_surface_cloud(seed)
    rng = _rng(seed, STREAM_WORK)
    n_mv = n_queries // 2
    n_ffc = n_queries - n_mv
    T_mv = rng.integers(16, 1025, n_mv)
    mv = straight_line_paths_T(rng, team, T_mv, 7)
    T_ffc = rng.integers(16, 1025, n_ffc)
    lengths = rng.integers(16, T_ffc[:, None] + 1, (n_ffc, len(team)))
    lengths[np.arange(n_ffc), rng.integers(0, len(team), n_ffc)] = T_ffc
    ffc = stratified_timed_paths(rng, team, lengths, 2, 8, 7)
    return team, env, mv, ffc
