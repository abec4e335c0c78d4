"""The centralised team MDP of the decentralised model (Sec. 3.1, Def.
teamMDP), in FP64, for small instances only.

TEST INFRASTRUCTURE ONLY (as the rest of this package).  The team MDP is
exponential in the number of agents (Sec. 3.1 states its size); here it is an
independent check of Alg. 2: its scalarised optimum from the joint initial
state equals the best assignment's value (Lemma lem:ct-mdp-prop), with
|I| = |J|.

States are (i, j, s, q, used): agent i works on task j, agent state s, task
location q, and ``used`` the set of agents already committed (a bit mask).
  * Working rows: when agent i is committed and task j is not done at q, the
    agent's own actions move (s, q) as in the product, with agent i's cost
    and task j's first-acceptance mass as rewards.
  * At the start of task j (agent i at its initial state, task at q0, agent
    i not committed): a zero-reward switch commits agent i (b1), and another
    hands task j to the next uncommitted agent after i (b2).
  * When task j is done (accepted or trapped) under a committed agent i, a
    zero-reward switch starts task j + 1 with the first uncommitted agent
    (b3).  States without rows (the last task done) are absorbing with value
    0.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .product import traps


@dataclass
class TeamMDP:
    n_states: int
    state_row: np.ndarray      # int64 [S+1] rows of each state (may be empty)
    row_ptr: np.ndarray        # int64 [R+1]
    col: np.ndarray            # int64 [N]
    prob: np.ndarray           # float64 [N]
    rew: np.ndarray            # float64 [R, |I|+|J|] objective vector of each row
    init: int


def build_team_mdp(wl) -> TeamMDP:
    nI, nJ = wl.n_agents, wl.n_tasks
    agents, tasks = wl.agents, wl.tasks
    d = nI + nJ
    done = [tasks[j].accepting.astype(bool) | traps(tasks[j].n_locs, tasks[j].delta, tasks[j].accepting)
            for j in range(nJ)]
    keys = [(i, j, s, q, used) for i in range(nI) for j in range(nJ) for s in range(agents[i].n_states)
            for q in range(tasks[j].n_locs) for used in range(1 << nI)]
    index = {key: n for n, key in enumerate(keys)}
    state_row, row_ptr, col, prob, rew = [0], [0], [], [], []

    def add_row(succ, r):
        for target, p in succ:
            col.append(target)
            prob.append(p)
        row_ptr.append(len(col))
        rew.append(r)

    for (i, j, s, q, used) in keys:
        ag, tk = agents[i], tasks[j]
        mine = (used >> i) & 1
        if mine and not done[j][q]:
            for a in range(ag.n_actions):
                r = s * ag.n_actions + a
                lo, hi = ag.sa_ptr[r], ag.sa_ptr[r + 1]
                if hi == lo:
                    continue
                succ, mass = [], 0.0
                for e in range(lo, hi):
                    s2 = int(ag.succ[e])
                    q2 = int(tk.delta[q, wl.letters[i][j][s2]])
                    if tk.accepting[q2] and not tk.accepting[q]:
                        mass += ag.prob[e]
                    succ.append((index[(i, j, s2, q2, used)], ag.prob[e]))
                v = np.zeros(d)
                v[i] = -ag.cost[r]
                v[nI + j] = mass
                add_row(succ, v)
        if s == ag.init and q == tk.q0 and not mine:
            add_row([(index[(i, j, s, q, used | (1 << i))], 1.0)], np.zeros(d))                      # b1
            nxt = [k for k in range(i + 1, nI) if not (used >> k) & 1]
            if nxt:
                k = nxt[0]
                add_row([(index[(k, j, agents[k].init, q, used)], 1.0)], np.zeros(d))               # b2
        if mine and done[j][q] and j + 1 < nJ:
            free = [k for k in range(nI) if not (used >> k) & 1]
            if free:
                k = free[0]
                add_row([(index[(k, j + 1, agents[k].init, tasks[j + 1].q0, used)], 1.0)], np.zeros(d))  # b3
        state_row.append(len(row_ptr) - 1)
    return TeamMDP(n_states=len(keys), state_row=np.asarray(state_row, dtype=np.int64),
                   row_ptr=np.asarray(row_ptr, dtype=np.int64), col=np.asarray(col, dtype=np.int64),
                   prob=np.asarray(prob, dtype=np.float64), rew=np.asarray(rew, dtype=np.float64).reshape(-1, d),
                   init=index[(0, 0, agents[0].init, tasks[0].q0, 0)])


def team_value(team: TeamMDP, w: np.ndarray, eps: float = 1e-12, max_sweeps: int = 1_000_000) -> float:
    """Scalarised optimum w . (objectives) from the joint initial state, by
    Jacobi value iteration from 0 (states without rows keep value 0)."""
    S = team.n_states
    R = len(team.row_ptr) - 1
    P = sp.csr_matrix((team.prob, team.col, team.row_ptr), shape=(R, S))
    r = team.rew @ np.asarray(w, dtype=np.float64)
    counts = np.diff(team.state_row)
    has = counts > 0
    starts = team.state_row[:-1][has]
    x = np.zeros(S)
    for _ in range(max_sweeps):
        y = np.zeros(S)
        y[has] = np.maximum.reduceat(r + P @ x, starts)
        if np.abs(y - x).max() <= eps:
            return float(y[team.init])
        x = y
    raise RuntimeError("value iteration did not converge")


def team_value_proper(team: TeamMDP, w: np.ndarray) -> float:
    """Scalarised optimum over proper policies (those that finish every task
    with probability 1) from the joint initial state.

    Where an agent's steps weigh nothing, the team MDP admits an improper
    optimum (that agent takes a task and never finishes it, so the agents
    after it never spend anything); ``team_value`` returns that one.  The
    proper optimum is the least solution v of v >= r_a + P_a v over every row
    a (any such v bounds each proper policy's value from above, and the
    proper optimum satisfies the system with equality), i.e. the linear
    programme min sum_s v(s) over that system; states without rows have
    v >= 0."""
    from scipy.optimize import linprog
    S = team.n_states
    R = len(team.row_ptr) - 1
    r = team.rew @ np.asarray(w, dtype=np.float64)
    row_state = np.repeat(np.arange(S), np.diff(team.state_row))
    P = sp.csr_matrix((team.prob, team.col, team.row_ptr), shape=(R, S))
    own = sp.csr_matrix((np.ones(R), (np.arange(R), row_state)), shape=(R, S))
    empty = np.flatnonzero(np.diff(team.state_row) == 0)
    lone = sp.csr_matrix((np.ones(len(empty)), (np.arange(len(empty)), empty)), shape=(len(empty), S))
    A = sp.vstack([-(own - P), -lone]).tocsr()
    b = np.concatenate([-r, np.zeros(len(empty))])
    res = linprog(np.ones(S), A_ub=A, b_ub=b, bounds=[(None, None)] * S, method="highs")
    if res.status != 0:
        raise RuntimeError("proper team optimum: " + res.message)
    return float(res.x[team.init])


def single_objective_model(team: TeamMDP, w: np.ndarray) -> dict:
    """The team MDP scalarised for one weight vector, laid out as a
    caller-built single-objective model (the reward in the cost column).
    States without rows get an empty one: all mass to done, reward 0, so
    their value is 0."""
    state_row, row_ptr, col, prob, rew = [0], [0], [], [], []
    r = team.rew @ w
    for s in range(team.n_states):
        rows = range(team.state_row[s], team.state_row[s + 1])
        for q in rows:
            lo, hi = team.row_ptr[q], team.row_ptr[q + 1]
            col += team.col[lo:hi].tolist()
            prob += team.prob[lo:hi].tolist()
            row_ptr.append(len(col))
            rew.append((r[q], 0.0))
        if len(rows) == 0:
            row_ptr.append(len(col))
            rew.append((0.0, 0.0))
        state_row.append(len(row_ptr) - 1)
    row_ptr = np.asarray(row_ptr)
    prob = np.asarray(prob)
    sums = np.array([prob[row_ptr[q]:row_ptr[q + 1]].sum() for q in range(len(row_ptr) - 1)])
    return {"state_row": np.asarray(state_row), "row_ptr": row_ptr, "col": np.asarray(col), "prob": prob,
            "rew": np.asarray(rew), "to_done": (sums < 1 - 1e-12).astype(np.uint8), "init": team.init}
