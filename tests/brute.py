"""Independent numpy brute force for tiny MV/FFC cases (test helper).

Written separately from the C oracle and with a different formulation, so a
slip in either shows up as a disagreement:

* kinematics as products of 4x4 homogeneous matrices built per joint,
* clearances via closest-point clamping (box) and a slab/disk split
  (cylinder) instead of the oracle's excess-vector formulas,
* all timesteps and all sphere pairs evaluated at once, with no early exit;
  MV is ``any`` over the collision tensor and FFC the lexicographic minimum
  of the colliding (t, i, j) triples.
"""
from __future__ import annotations

import numpy as np

REV_Z, PRI_X, PRI_Y, PRI_Z = 0, 1, 2, 3


def h4(m12):
    M = np.eye(4)
    M[:3, :] = np.asarray(m12, dtype=np.float64).reshape(3, 4)
    return M


def joint4(jt, q):
    M = np.eye(4)
    if jt == REV_Z:
        M[0, 0], M[0, 1], M[1, 0], M[1, 1] = np.cos(q), -np.sin(q), np.sin(q), np.cos(q)
    else:
        M[jt - 1, 3] = q
    return M


def spheres_world(robot, q):
    frames = [h4(robot.base)]
    for k in range(robot.dof):
        frames.append(frames[-1] @ h4(robot.joint_fixed[k]) @ joint4(int(robot.joint_type[k]), q[k]))
    out = np.zeros((robot.n_spheres, 4))
    for s in range(robot.n_spheres):
        c = np.append(robot.sphere_xyzr[s, :3], 1.0)
        out[s, :3] = (frames[int(robot.sphere_frame[s])] @ c)[:3]
        out[s, 3] = robot.sphere_xyzr[s, 3]
    return out


def state(times, cfgs, t):
    times = np.asarray(times)
    if t >= times[-1]:
        return np.asarray(cfgs[-1], dtype=np.float64)
    k = int(np.searchsorted(times, t, side="right") - 1)
    s = (t - times[k]) / (times[k + 1] - times[k])
    return cfgs[k] + s * (cfgs[k + 1] - cfgs[k])


def box_clear(x, r, box):
    c, R, h = box[:3], box[3:12].reshape(3, 3), box[12:15]
    p = R.T @ (x - c)
    closest = np.clip(p, -h, h)
    gap = np.linalg.norm(p - closest)
    if gap > 0:
        return gap - r
    return float(np.max(np.abs(p) - h)) - r


def cyl_clear(x, r, cyl):
    c, u, hl, R = cyl[:3], cyl[3:6], cyl[6], cyl[7]
    v = x - c
    h = float(v @ u)
    s = float(np.linalg.norm(np.cross(u, v)))
    if abs(h) <= hl and s <= R:
        return max(s - R, abs(h) - hl) - r
    if abs(h) <= hl:
        return (s - R) - r
    if s <= R:
        return (abs(h) - hl) - r
    return float(np.hypot(s - R, abs(h) - hl)) - r


def team_states(team, paths, qi):
    T = int(paths.horizon()[qi])
    per_t = []
    for t in range(T):
        per_t.append([spheres_world(rob, state(*paths.path(qi, r), t)[:rob.dof])
                      for r, rob in enumerate(team)])
    return per_t


def rr_hits(sph_t):
    """List of colliding (i, j) pairs, i<j, at one timestep."""
    n = len(sph_t)
    hits = []
    for i in range(n):
        for j in range(i + 1, n):
            A, B = sph_t[i], sph_t[j]
            d = np.linalg.norm(A[:, None, :3] - B[None, :, :3], axis=2)
            if np.any(d < A[:, None, 3] + B[None, :, 3]):
                hits.append((i, j))
    return hits


def env_hit(team, env, sph_t, r):
    S = sph_t[r]
    for (a, b) in team[r].self_pairs:
        if np.linalg.norm(S[a, :3] - S[b, :3]) < S[a, 3] + S[b, 3]:
            return True
    for x in S:
        for o in env.spheres:
            if np.linalg.norm(x[:3] - o[:3]) < x[3] + o[3]:
                return True
        for b in env.boxes:
            if box_clear(x[:3], x[3], b) < 0:
                return True
        for cy in env.cylinders:
            if cyl_clear(x[:3], x[3], cy) < 0:
                return True
        if len(env.points):
            if np.any(np.linalg.norm(env.points - x[:3], axis=1) < x[3] + env.point_radius):
                return True
    return False


def mv(team, env, paths, qi, check_env=True, focus=None):
    """focus: robots validated (a set of indices; None = all), prioritised MV."""
    F = set(range(len(team))) if focus is None else set(focus)
    for sph_t in team_states(team, paths, qi):
        if check_env and any(env_hit(team, env, sph_t, r) for r in F):
            return False
        if any(i in F or j in F for (i, j) in rr_hits(sph_t)):
            return False
    return True


def ffc(team, paths, qi):
    for t, sph_t in enumerate(team_states(team, paths, qi)):
        h = rr_hits(sph_t)
        if h:
            return (t,) + min(h)
    return (-1, -1, -1)
