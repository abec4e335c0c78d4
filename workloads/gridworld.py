"""Grid-world agents and reach/avoid task automata, drawn from a seed.

Agent MDP (the labelled MDP of the Preliminaries, "Markov Decision Process"):
the states are the free cells of the largest 4-connected component of a W x H
grid.  Actions are N, S, E, W, stay (indices 0..4).  A move reaches the
intended neighbour with probability 1 - p_slip and otherwise one of the two
perpendicular neighbours, each with probability p_slip / 2.  A move into a
wall, an obstacle or a cell outside the component leaves the agent in place.
"stay" is deterministic.  Successors reached by several outcomes are merged,
listed in order of first appearance among (intended, perpendicular 1,
perpendicular 2).  Every action is enabled in every state.  Each (agent,
action) pair has a cost drawn from U[1, 3]; the agent's reward is its negative.

Task DFA (the DFA of the Preliminaries, accepting locations are sinks):
  * reach-seq(k): locations 0..k, waypoint sets a_1..a_k (2 cells each).  In
    location q < k the letter "a_{q+1}" moves to q+1; every other letter stays.
    Location k accepts and is a sink.
  * avoid-seq(k): as reach-seq(k) plus an avoid set (3 cells) and location
    k+1, a sink that cannot reach acceptance.  The avoid letter sends every
    location q < k to k+1.
A cell carries at most one proposition, so the labelling L_ij(s) of agent i's
state s as seen by task j is a small integer "letter": 0 = no proposition,
l in 1..k = waypoint set a_l, k+1 = avoid (avoid-seq only).

Everything here is input data; nothing computes a product, a value or a
policy.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

ACTIONS = ("N", "S", "E", "W", "stay")
# (dx, dy) per action; y grows southwards.
_DIRS = ((0, -1), (0, 1), (1, 0), (-1, 0), (0, 0))
# perpendicular directions of each move
_PERP = {0: (2, 3), 1: (2, 3), 2: (0, 1), 3: (0, 1)}

BASE_SEED = 230504397


def workload_seed(cfg: int, variant: int = 0) -> int:
    """Seed of configuration ``cfg`` (1-based), variant ``variant``."""
    return BASE_SEED + 1000 * cfg + variant


@dataclass
class Agent:
    """Explicit sparse agent MDP.  Row (s, a) = s * n_actions + a owns
    successors ``succ[sa_ptr[row]:sa_ptr[row+1]]`` with ``prob`` alongside."""
    width: int
    height: int
    cells: np.ndarray          # int32 [n_states]: grid cell (y*W + x) of each state
    init: int                  # initial state index
    p_slip: float
    action_cost: np.ndarray    # float64 [n_actions], positive costs
    n_actions: int
    sa_ptr: np.ndarray         # int32 [n_states*n_actions + 1]
    succ: np.ndarray           # int32 [nnz]
    prob: np.ndarray           # float64 [nnz]
    cost: np.ndarray           # float64 [n_states*n_actions]

    @property
    def n_states(self) -> int:
        return int(self.cells.shape[0])


@dataclass
class Task:
    """A reach-seq / avoid-seq task as a DFA table plus its cells (normalised
    coordinates are kept so each agent can snap them to its own grid)."""
    kind: str                  # "reach" or "avoid"
    k: int
    n_locs: int
    n_letters: int
    q0: int
    delta: np.ndarray          # int32 [n_locs, n_letters]
    accepting: np.ndarray      # uint8 [n_locs]
    waypoints_uv: np.ndarray   # float64 [k, 2, 2]: k sets of 2 cells, (u, v) in [0,1)
    avoid_uv: Optional[np.ndarray]  # float64 [3, 2] or None


@dataclass
class Workload:
    name: str
    agents: List[Agent]
    tasks: List[Task]
    letters: List[List[np.ndarray]]   # letters[i][j]: int32 [agent i n_states]
    meta: dict = field(default_factory=dict)

    @property
    def n_agents(self) -> int:
        return len(self.agents)

    @property
    def n_tasks(self) -> int:
        return len(self.tasks)


# --------------------------------------------------------------------------
# grids
# --------------------------------------------------------------------------

def _largest_component(free: np.ndarray) -> np.ndarray:
    """Boolean mask of the largest 4-connected component of ``free``."""
    H, W = free.shape
    comp = -np.ones((H, W), dtype=np.int64)
    best, best_size, cid = -1, 0, 0
    for y0 in range(H):
        for x0 in range(W):
            if not free[y0, x0] or comp[y0, x0] >= 0:
                continue
            stack = [(y0, x0)]
            comp[y0, x0] = cid
            size = 0
            while stack:
                y, x = stack.pop()
                size += 1
                for dx, dy in _DIRS[:4]:
                    yy, xx = y + dy, x + dx
                    if 0 <= yy < H and 0 <= xx < W and free[yy, xx] and comp[yy, xx] < 0:
                        comp[yy, xx] = cid
                        stack.append((yy, xx))
            if size > best_size:
                best, best_size = cid, size
            cid += 1
    return comp == best


def make_grid(rng: np.random.Generator, width: int, height: int,
              obstacle_frac: float) -> np.ndarray:
    """Free-cell mask (H, W) restricted to the largest component."""
    free = rng.random((height, width)) >= obstacle_frac
    if not free.any():
        free[0, 0] = True
    return _largest_component(free)


def make_agent(rng: np.random.Generator, free: np.ndarray, start_cell: int,
               p_slip: float, action_cost: np.ndarray) -> Agent:
    """Explicit agent MDP on the free cells of ``free`` (see module doc)."""
    H, W = free.shape
    cells = np.flatnonzero(free.ravel()).astype(np.int32)
    index = -np.ones(H * W, dtype=np.int64)
    index[cells] = np.arange(cells.size)
    nA = len(ACTIONS)

    def target(c: int, d: int) -> int:
        y, x = divmod(int(c), W)
        dx, dy = _DIRS[d]
        yy, xx = y + dy, x + dx
        if 0 <= yy < H and 0 <= xx < W and free[yy, xx]:
            return int(index[yy * W + xx])
        return int(index[c])

    sa_ptr = [0]
    succ: List[int] = []
    prob: List[float] = []
    for s, c in enumerate(cells):
        for a in range(nA):
            if a == 4:
                outcomes = [(s, 1.0)]
            else:
                p1, p2 = _PERP[a]
                outcomes = [(target(c, a), 1.0 - p_slip),
                            (target(c, p1), 0.5 * p_slip),
                            (target(c, p2), 0.5 * p_slip)]
            merged: List[List] = []
            for t, p in outcomes:
                if p <= 0.0:
                    continue
                for m in merged:
                    if m[0] == t:
                        m[1] += p
                        break
                else:
                    merged.append([t, p])
            for t, p in merged:
                succ.append(t)
                prob.append(p)
            sa_ptr.append(len(succ))
    n = cells.size
    init = int(index[start_cell])
    assert init >= 0
    return Agent(width=W, height=H, cells=cells, init=init, p_slip=float(p_slip),
                 action_cost=np.asarray(action_cost, dtype=np.float64), n_actions=nA,
                 sa_ptr=np.asarray(sa_ptr, dtype=np.int32),
                 succ=np.asarray(succ, dtype=np.int32),
                 prob=np.asarray(prob, dtype=np.float64),
                 cost=np.tile(np.asarray(action_cost, dtype=np.float64), n))


# --------------------------------------------------------------------------
# tasks
# --------------------------------------------------------------------------

def make_task_dfa(kind: str, k: int) -> tuple:
    """(n_locs, n_letters, q0, delta, accepting) of reach-seq(k) / avoid-seq(k)."""
    if kind == "reach":
        n_locs, n_letters = k + 1, k + 1
    elif kind == "avoid":
        n_locs, n_letters = k + 2, k + 2
    else:
        raise ValueError(kind)
    delta = np.zeros((n_locs, n_letters), dtype=np.int32)
    for q in range(n_locs):
        delta[q, :] = q
    for q in range(k):
        delta[q, q + 1] = q + 1
        if kind == "avoid":
            delta[q, k + 1] = k + 1
    accepting = np.zeros(n_locs, dtype=np.uint8)
    accepting[k] = 1
    return n_locs, n_letters, 0, delta, accepting


def _make_task(rng: np.random.Generator, kind: str, k: int) -> Task:
    n_locs, n_letters, q0, delta, acc = make_task_dfa(kind, k)
    wp = rng.random((k, 2, 2))
    av = rng.random((3, 2)) if kind == "avoid" else None
    return Task(kind=kind, k=k, n_locs=n_locs, n_letters=n_letters, q0=q0,
                delta=delta, accepting=acc, waypoints_uv=wp, avoid_uv=av)


def _snap(free: np.ndarray, uv: np.ndarray, taken: set) -> int:
    """Nearest free cell (Euclidean in cell units, ties by cell index) to the
    normalised point ``uv`` that is not in ``taken``."""
    H, W = free.shape
    x, y = uv[0] * W, uv[1] * H
    cells = np.flatnonzero(free.ravel())
    cy, cx = np.divmod(cells, W)
    d2 = (cx + 0.5 - x) ** 2 + (cy + 0.5 - y) ** 2
    order = np.lexsort((cells, d2))
    for o in order:
        c = int(cells[o])
        if c not in taken:
            return c
    raise ValueError("grid too small for the task cells")


def _letters(agent: Agent, free: np.ndarray, task: Task, start_cell: int) -> np.ndarray:
    taken = {start_cell}
    letter_of_cell = {}
    for l in range(task.k):
        for u in range(2):
            c = _snap(free, task.waypoints_uv[l, u], taken)
            taken.add(c)
            letter_of_cell[c] = l + 1
    if task.avoid_uv is not None:
        for u in range(3):
            c = _snap(free, task.avoid_uv[u], taken)
            taken.add(c)
            letter_of_cell[c] = task.k + 1
    by_cell = np.zeros(free.size, dtype=np.int32)
    for c, l in letter_of_cell.items():
        by_cell[c] = l
    return by_cell[agent.cells]


def _draw_start(rng: np.random.Generator, free: np.ndarray, taken: set) -> int:
    cells = [int(c) for c in np.flatnonzero(free.ravel()) if int(c) not in taken]
    return cells[int(rng.integers(len(cells)))]


# --------------------------------------------------------------------------
# configurations
# --------------------------------------------------------------------------

def _assemble(name, rng, grids, starts, slips, costs, tasks, meta) -> Workload:
    agents = [make_agent(rng, g, s, p, c) for g, s, p, c in zip(grids, starts, slips, costs)]
    letters = [[_letters(a, g, t, s) for t in tasks]
               for a, g, s in zip(agents, grids, starts)]
    return Workload(name=name, agents=agents, tasks=tasks, letters=letters, meta=meta)


def make_workload(cfg: int, variant: int = 0, *, n_agents: Optional[int] = None,
                  n_tasks: Optional[int] = None) -> Workload:
    """Configuration ``cfg`` (1, 2 or 3) drawn from ``workload_seed(cfg, variant)``.

    1: 2 agents on their own obstacle-free 6x6 grids, p_slip 0.1, two
       reach-seq(2) tasks.
    2: 10 agents sharing one 20x20 grid with 15 % obstacles, p_slip ~ U[.05,.2],
       20 tasks of 3-8 DFA locations (reach-seq k in [2,7] or avoid-seq k in
       [1,6], type uniform).
    3: 50 agents, 46 on 32x32 grids and one each on 48x48, 64x64, 96x96 and
       128x128 (20 % obstacles, one grid per agent), p_slip ~ U[.05,.2];
       100 tasks, 90 with 3 locations and 10 with 4,5,...,12,12 locations.
    ``n_agents`` / ``n_tasks`` truncate the agent / task lists (same draws).
    """
    rng = np.random.default_rng(workload_seed(cfg, variant))
    if cfg == 1:
        nI, nJ = 2, 2
        grids = [make_grid(rng, 6, 6, 0.0) for _ in range(nI)]
        slips = [0.1] * nI
        costs = [rng.uniform(1.0, 3.0, size=5) for _ in range(nI)]
        tasks = [_make_task(rng, "reach", 2) for _ in range(nJ)]
        name = "2x2 agents-tasks, 6x6 grids"
    elif cfg == 2:
        nI, nJ = 10, 20
        g = make_grid(rng, 20, 20, 0.15)
        grids = [g] * nI
        slips = list(rng.uniform(0.05, 0.2, size=nI))
        costs = [rng.uniform(1.0, 3.0, size=5) for _ in range(nI)]
        tasks = []
        for _ in range(nJ):
            if rng.random() < 0.5:
                tasks.append(_make_task(rng, "reach", int(rng.integers(2, 8))))
            else:
                tasks.append(_make_task(rng, "avoid", int(rng.integers(1, 7))))
        name = "10x20 agents-tasks, shared 20x20 grid, 15% obstacles"
    elif cfg == 3:
        nI, nJ = 50, 100
        sizes = [32] * 46 + [48, 64, 96, 128]
        grids = [make_grid(rng, s, s, 0.20) for s in sizes]
        slips = list(rng.uniform(0.05, 0.2, size=nI))
        costs = [rng.uniform(1.0, 3.0, size=5) for _ in range(nI)]
        n_locs = [3] * 90 + [4, 5, 6, 7, 8, 9, 10, 11, 12, 12]
        tasks = []
        for nl in n_locs:
            kind = "reach" if rng.random() < 0.5 else "avoid"
            k = nl - 1 if kind == "reach" else nl - 2
            tasks.append(_make_task(rng, kind, k))
        name = "50x100 agents-tasks, 32x32..128x128 grids, 20% obstacles"
    else:
        raise ValueError(f"unknown configuration {cfg}")
    starts = []
    for g in grids:
        starts.append(_draw_start(rng, g, set()))
    nI2 = nI if n_agents is None else min(nI, n_agents)
    nJ2 = nJ if n_tasks is None else min(nJ, n_tasks)
    return _assemble(name, rng, grids[:nI2], starts[:nI2], slips[:nI2], costs[:nI2],
                     tasks[:nJ2], {"cfg": cfg, "variant": variant})


def tiny_workload(seed: int, n_agents: int = 2, n_tasks: int = 2, width: int = 3,
                  height: int = 2, p_slip: float = 0.2, obstacle_frac: float = 0.0,
                  kinds=("reach", "avoid"), k: int = 1) -> Workload:
    """Small instances for brute force / LP / centralised cross-checks."""
    rng = np.random.default_rng(seed)
    grids = [make_grid(rng, width, height, obstacle_frac) for _ in range(n_agents)]
    slips = [p_slip] * n_agents
    costs = [rng.uniform(1.0, 3.0, size=5) for _ in range(n_agents)]
    tasks = [_make_task(rng, kinds[j % len(kinds)], k) for j in range(n_tasks)]
    starts = [_draw_start(rng, g, set()) for g in grids]
    return _assemble(f"tiny-{seed}", rng, grids, starts, slips, costs, tasks, {"seed": seed})


def dirichlet_weights(rng: np.random.Generator, K: int, d: int) -> np.ndarray:
    """K weight vectors drawn from Dirichlet(1_d) (rows >= 0, summing to 1)."""
    W = rng.dirichlet(np.ones(d), size=K)
    return W / W.sum(axis=1, keepdims=True)


def worked_example() -> Workload:
    """The one-agent, one-task MDP of the paper's worked example (Fig. 3a).

    States s0..s3; s1 is labelled x, s3 is labelled y.  At s0, action a goes to
    s0/s1/s2 with probabilities .3/.2/.5 and action b to s1/s3 with .9/.1; s2
    moves to s3; s1 and s3 loop.  Every action has reward -1.  The task is
    "not x until y": letters 0 = {}, 1 = {x}, 2 = {y}; location 0 moves to the
    accepting sink 1 on y and to the trap 2 on x.
    """
    sa_ptr, succ, prob, cost = [0], [], [], []
    rows = {0: [[(0, .3), (1, .2), (2, .5)], [(1, .9), (3, .1)]],
            1: [[(1, 1.0)]], 2: [[(3, 1.0)]], 3: [[(3, 1.0)]]}
    # every state gets two action slots; a missing second action is disabled
    # (an empty row, i.e. probabilities summing to 0)
    for s in range(4):
        for a in range(2):
            if a < len(rows[s]):
                for t, p in rows[s][a]:
                    succ.append(t)
                    prob.append(p)
            cost.append(1.0)
            sa_ptr.append(len(succ))
    agent = Agent(width=4, height=1, cells=np.arange(4, dtype=np.int32), init=0, p_slip=0.0,
                  action_cost=np.array([1.0, 1.0]), n_actions=2,
                  sa_ptr=np.asarray(sa_ptr, dtype=np.int32), succ=np.asarray(succ, dtype=np.int32),
                  prob=np.asarray(prob, dtype=np.float64), cost=np.asarray(cost, dtype=np.float64))
    delta = np.array([[0, 2, 1], [1, 1, 1], [2, 2, 2]], dtype=np.int32)
    task = Task(kind="until", k=1, n_locs=3, n_letters=3, q0=0, delta=delta,
                accepting=np.array([0, 1, 0], dtype=np.uint8),
                waypoints_uv=np.zeros((0, 2, 2)), avoid_uv=None)
    letters = [[np.array([0, 1, 0, 2], dtype=np.int32)]]
    return Workload(name="worked example (Fig. 3a)", agents=[agent], tasks=[task],
                    letters=letters, meta={})
