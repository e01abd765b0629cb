"""A thin Composite RRT-Connect driver whose edge checks are MV requests through
the serving loop (Composite RRT-C, §III-C: single-robot RRT-Connect run in the
composite configuration space, with multi-robot MV as its edge check; the team
is one composite robot, and every edge is a straight composite motion whose
robots move together, discretised so that no joint moves more than ``step`` per
timestep).

Each iteration extends the current tree toward a batch of random composite
configurations (one MV request for the whole batch of edges), then grows the
other tree toward every new node in steps of at most ``max_step`` (a second
request holding all the steps), keeping each chain's valid prefix, and swaps the
trees: RRT-Connect (Kuffner and LaValle, 2000) with batched EXTEND and CONNECT,
so that one request carries many edges.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import mrv
from . import workloads as W


class ServedChecker:
    """Validates batches of straight composite edges with MV requests submitted
    to a context's serving loop.  ``log`` keeps (starts, goals, answers) of
    every request when set."""

    def __init__(self, ctx: mrv.Context, team_handle: int, env_handle: int, team, step: float = 1.0 / 32.0,
                 metric: str = "linf", dof_stride: int = 7, flags: int = mrv.CHECK_ENV, log: bool = False):
        self.ctx, self.team_handle, self.env_handle = ctx, team_handle, env_handle
        self.dofs = [r.dof for r in team]
        self.step, self.metric, self.dof_stride, self.flags = step, metric, dof_stride, flags
        self.requests = 0
        self.edges = 0
        self.log = [] if log else None

    def __call__(self, starts: np.ndarray, goals: np.ndarray) -> np.ndarray:
        if len(starts) == 0:
            return np.zeros(0, dtype=bool)
        paths = W.straight_line_paths(starts, goals, self.dofs, self.step, self.metric, self.dof_stride)
        ticket = self.ctx.submit(0, self.team_handle, self.env_handle, paths, self.flags)
        ok = self.ctx.poll(ticket, 0, len(starts), timeout_ms=None).astype(bool)
        self.requests += 1
        self.edges += len(starts)
        if self.log is not None:
            self.log.append((starts.copy(), goals.copy(), ok.copy()))
        return ok


@dataclass
class _Tree:
    nodes: list = field(default_factory=list)       # composite configurations [n_robots, dof_stride]
    parent: list = field(default_factory=list)

    def add(self, q, parent: int) -> int:
        self.nodes.append(np.array(q, dtype=np.float64))
        self.parent.append(parent)
        return len(self.nodes) - 1

    def nearest(self, qs: np.ndarray) -> np.ndarray:
        """Index of the nearest node (L-infinity over all joints) for each row of qs."""
        nodes = np.stack(self.nodes)                                    # [N, n, d]
        d = np.abs(qs[:, None] - nodes[None]).reshape(len(qs), len(nodes), -1).max(axis=2)
        return np.argmin(d, axis=1)

    def branch(self, i: int) -> list:
        out = []
        while i >= 0:
            out.append(self.nodes[i])
            i = self.parent[i]
        return out                                                      # node ... root


@dataclass
class PlanResult:
    path: list | None          # composite configurations, start first; None: no path found
    iterations: int
    seconds: float
    tree_sizes: tuple


def rrt_connect(check, team, start: np.ndarray, goal: np.ndarray, rng: np.random.Generator, batch: int = 32,
                max_step: float = 0.5, max_iters: int = 300, dof_stride: int = 7) -> PlanResult:
    """Composite RRT-Connect between two composite configurations
    ([n_robots, dof_stride]).  ``check(starts, goals)`` returns the validity of
    each straight edge.  Fails at once when the start or goal state itself
    collides."""
    t0 = time.perf_counter()
    start = np.asarray(start, dtype=np.float64)
    goal = np.asarray(goal, dtype=np.float64)
    ends = check(np.stack([start, goal]), np.stack([start, goal]))
    if not ends.all():
        return PlanResult(None, 0, time.perf_counter() - t0, (0, 0))
    if check(start[None], goal[None])[0]:
        return PlanResult([start, goal], 0, time.perf_counter() - t0, (1, 1))
    ta, tb = _Tree(), _Tree()
    ta.add(start, -1)
    tb.add(goal, -1)
    a_is_start = True
    for it in range(1, max_iters + 1):
        # extend tree a toward a batch of random composite configurations
        target = W.sample_configs(rng, team, batch, dof_stride)
        near = ta.nearest(target)
        qn = np.stack([ta.nodes[i] for i in near])
        d = target - qn
        span = np.abs(d).reshape(batch, -1).max(axis=1)
        scale = np.minimum(1.0, max_step / np.maximum(span, 1e-12))
        qnew = qn + d * scale[:, None, None]
        ok = check(qn, qnew)
        added = [ta.add(qnew[k], int(near[k])) for k in np.nonzero(ok)[0]]
        if added:
            # connect: grow tree b from its nearest node toward each new node in
            # steps of at most max_step; all steps of all chains go in one request,
            # and each chain keeps its valid prefix
            chains, seg_a, seg_b = [], [], []
            for i in added:
                j = int(tb.nearest(ta.nodes[i][None])[0])
                p0, p1 = tb.nodes[j], ta.nodes[i]
                m = max(1, int(np.ceil(np.abs(p1 - p0).max() / max_step)))
                pts = [p0 + (p1 - p0) * (s / m) for s in range(m)] + [p1]
                chains.append((i, j, pts, len(seg_a)))
                seg_a += pts[:-1]
                seg_b += pts[1:]
            ok = check(np.stack(seg_a), np.stack(seg_b))
            for i, j, pts, o in chains:
                m = len(pts) - 1
                good = ok[o:o + m]
                n_ok = m if good.all() else int(np.argmin(good))
                parent = j
                for s in range(1, n_ok + 1 if n_ok < m else m):
                    parent = tb.add(pts[s], parent)
                if n_ok == m:
                    side_a = ta.branch(i)[::-1]                         # root of a ... new node
                    side_b = tb.branch(parent)                          # last step ... root of b
                    path = side_a + side_b
                    if not a_is_start:
                        path = path[::-1]
                    return PlanResult(path, it, time.perf_counter() - t0, (len(ta.nodes), len(tb.nodes)))
        ta, tb = tb, ta
        a_is_start = not a_is_start
    return PlanResult(None, max_iters, time.perf_counter() - t0, (len(ta.nodes), len(tb.nodes)))


def two_arm_problem(seed: int = 1):
    """Two of the arm workload's 7-R arms on opposite corners of the 1 m square,
    among 4 boxes and 2 cylinders of the cube."""
    m = W.arm_models(1)
    team = [m[0].with_base(W.arm_base(0.5, 0.5), "arm0"), m[2].with_base(W.arm_base(-0.5, -0.5), "arm2")]
    return team, W.cube_env(seed, n_boxes=4, n_cyl=2)


def plan_study(ctx: mrv.Context, n_problems: int = 8, batch: int = 32, max_step: float = 0.5,
               max_iters: int = 150) -> dict:
    """Plans ``n_problems`` seeded start-goal pairs of the two-arm problem with
    edge checks served by ``ctx``; times, requests and edges per plan."""
    team, env = two_arm_problem()
    th, eh = ctx.load_team(team), ctx.load_env(env)
    rows = []
    for seed in range(n_problems):
        check = ServedChecker(ctx, th, eh, team)
        rng = np.random.default_rng(seed)
        start, goal = sample_free_pair(check, team, rng)
        r0, e0 = check.requests, check.edges
        res = rrt_connect(check, team, start, goal, rng, batch=batch, max_step=max_step, max_iters=max_iters)
        rows.append(dict(solved=res.path is not None, ms=res.seconds * 1e3, iterations=res.iterations,
                         requests=check.requests - r0, edges=check.edges - e0,
                         path_states=len(res.path) if res.path else 0))
    ctx.unload(eh)
    ctx.unload(th)
    ok = [r for r in rows if r["solved"]]
    req = sum(r["requests"] for r in rows)
    return dict(problems=n_problems, solved=len(ok),
                median_ms_solved=float(np.median([r["ms"] for r in ok])) if ok else None,
                mean_requests_per_plan=req / n_problems,
                mean_edges_per_request=sum(r["edges"] for r in rows) / max(req, 1),
                ms_per_request=sum(r["ms"] for r in rows) / max(req, 1), per_problem=rows)


def sample_free_pair(check, team, rng: np.random.Generator, dof_stride: int = 7, tries: int = 64):
    """A start and a goal state that ``check`` finds collision-free."""
    c = W.sample_configs(rng, team, tries, dof_stride)
    free = np.nonzero(check(c, c))[0]
    if len(free) < 2:
        raise RuntimeError("no two free states among the samples")
    return c[free[0]], c[free[1]]
