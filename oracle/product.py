"""Agent-task product MDPs (Sec. 2 "Product MDP"; Sec. 3.1, agent-task MDP
M_{i(x)j} with proposition done_j and reward rho_{j+|I|}).

Readings taken here:
  * A location is a trap if no run reaches an accepting location (Sec. 2,
    DFA paragraph).  A product state (s, q) is ``done`` iff q is accepting or a
    trap (Sec. 3.1).  Done states are absorbing with value 0, so they are not
    stored: transitions into them are dropped and the rows of the remaining
    ("live") states become sub-stochastic.
  * The initial product state is (s0, q0) (Sec. 2, product definition).
  * Probability reward (standard reading of the pre-sink construction):
    rho_{j+|I|}(s, q, a) = sum_{s'} P(s, a, s') [delta(q, L(s')) accepting],
    the one-step mass of first acceptance.  Its expected total equals the
    probability of completing the task.  ``presink_literal=True`` instead adds
    the paper's one-off unit reward in a pre-sink location (parity unpinned).
  * Cost reward rho_i(s, q, a) = -c_i(s, a) (costs are negative rewards,
    Sec. 3.1), charged on every action taken in a live state.
  * Enabled actions are those whose successor probabilities sum to 1
    (Sec. 2, MDP definition); a row with no successors is disabled.
  * Canonical order: live reachable states sorted by (q, s); rows in action
    order; a row's entries in the agent's successor order.
"""
from __future__ import annotations

from dataclasses import dataclass
from collections import deque

import numpy as np
import scipy.sparse as sp


@dataclass
class Product:
    n_states: int              # live reachable states S
    states: np.ndarray         # int64 [S, 2] (agent state s, DFA location q)
    state_row: np.ndarray      # int64 [S+1] rows of each state
    row_action: np.ndarray     # int64 [R] agent action of each row
    row_ptr: np.ndarray        # int64 [R+1]
    col: np.ndarray            # int64 [N] live successor index
    prob: np.ndarray           # float64 [N]
    to_done: np.ndarray        # bool [R]: the row moves mass into a done state
    rew_cost: np.ndarray       # float64 [R]  (= -cost)
    rew_prob: np.ndarray       # float64 [R]
    init: int                  # index of (s0, q0), -1 if that state is done

    @property
    def n_rows(self) -> int:
        return int(self.row_action.shape[0])

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def P(self) -> sp.csr_matrix:
        """Row-by-state sparse transition matrix [R, S]."""
        return sp.csr_matrix((self.prob, self.col, self.row_ptr),
                             shape=(self.n_rows, self.n_states))

    def row_state(self) -> np.ndarray:
        return np.repeat(np.arange(self.n_states), np.diff(self.state_row))


def traps(n_locs: int, delta: np.ndarray, accepting: np.ndarray) -> np.ndarray:
    """Boolean mask of trap locations: no run reaches an accepting location."""
    reach = accepting.astype(bool).copy()
    changed = True
    while changed:
        changed = False
        for q in range(n_locs):
            if not reach[q] and reach[delta[q]].any():
                reach[q] = True
                changed = True
    return ~reach


def _with_presink(task):
    """The task automaton with one inserted pre-sink location p: every
    transition into an accepting location is redirected to p, and p moves to
    the first accepting location on every letter (Sec. 3.1, "we can modify
    A_j to include q").  Returns (n_locs, delta, accepting)."""
    n, L = task.n_locs, task.n_letters
    acc = task.accepting.astype(bool)
    target = int(np.flatnonzero(acc)[0])
    delta = np.zeros((n + 1, L), dtype=np.int64)
    for q in range(n):
        for l in range(L):
            q2 = int(task.delta[q, l])
            delta[q, l] = n if (acc[q2] and not acc[q]) else q2
    delta[n, :] = target
    return n + 1, delta, np.concatenate([task.accepting, [0]]).astype(np.uint8)


def build_product(agent, task, letters, presink_literal: bool = False) -> Product:
    """Live reachable part of M_i (x) A_j in CSR form (see module doc)."""
    if presink_literal:
        n_locs, delta, accepting = _with_presink(task)
    else:
        n_locs, delta, accepting = task.n_locs, task.delta, task.accepting
    acc = accepting.astype(bool)
    done_loc = acc | traps(n_locs, delta, accepting)
    if presink_literal:
        # rho = 1 exactly in locations outside Q_F all of whose successors accept
        presink = np.array([(not acc[q]) and bool(acc[delta[q]].all()) for q in range(n_locs)])
    nA = agent.n_actions
    sa_ptr, succ, prob = agent.sa_ptr, agent.succ, agent.prob

    def enabled(s, a):
        r = s * nA + a
        return sa_ptr[r + 1] > sa_ptr[r]

    start = (int(agent.init), int(task.q0))
    if done_loc[start[1]]:
        z = np.zeros(0, dtype=np.int64)
        return Product(0, np.zeros((0, 2), np.int64), np.zeros(1, np.int64), z,
                       np.zeros(1, np.int64), z, np.zeros(0), np.zeros(0, bool),
                       np.zeros(0), np.zeros(0), -1)
    # breadth-first exploration of live states from (s0, q0)
    seen = {start}
    queue = deque([start])
    while queue:
        s, q = queue.popleft()
        for a in range(nA):
            r = s * nA + a
            for e in range(sa_ptr[r], sa_ptr[r + 1]):
                s2 = int(succ[e])
                q2 = int(delta[q, letters[s2]])
                if not done_loc[q2] and (s2, q2) not in seen:
                    seen.add((s2, q2))
                    queue.append((s2, q2))
    states = sorted(seen, key=lambda sq: (sq[1], sq[0]))
    index = {sq: n for n, sq in enumerate(states)}
    state_row, row_action, row_ptr = [0], [], [0]
    col, pr, to_done, rc, rp = [], [], [], [], []
    for (s, q) in states:
        for a in range(nA):
            if not enabled(s, a):
                continue
            r = s * nA + a
            mass_acc = 0.0
            hits_done = False
            for e in range(sa_ptr[r], sa_ptr[r + 1]):
                s2 = int(succ[e])
                q2 = int(delta[q, letters[s2]])
                if done_loc[q2]:
                    hits_done = True
                    if acc[q2]:
                        mass_acc += float(prob[e])
                else:
                    col.append(index[(s2, q2)])
                    pr.append(float(prob[e]))
            if presink_literal:
                mass_acc = 1.0 if presink[q] else 0.0
            row_action.append(a)
            to_done.append(hits_done)
            rc.append(-float(agent.cost[r]))
            rp.append(mass_acc)
            row_ptr.append(len(col))
        state_row.append(len(row_action))
    return Product(
        n_states=len(states), states=np.asarray(states, dtype=np.int64).reshape(-1, 2),
        state_row=np.asarray(state_row, dtype=np.int64),
        row_action=np.asarray(row_action, dtype=np.int64),
        row_ptr=np.asarray(row_ptr, dtype=np.int64), col=np.asarray(col, dtype=np.int64),
        prob=np.asarray(pr, dtype=np.float64), to_done=np.asarray(to_done, dtype=bool),
        rew_cost=np.asarray(rc, dtype=np.float64), rew_prob=np.asarray(rp, dtype=np.float64),
        init=index[start])


def build_all(workload, presink_literal: bool = False):
    """Products of every (agent, task) pair, model index m = i * |J| + j."""
    out = []
    for i, agent in enumerate(workload.agents):
        for j, task in enumerate(workload.tasks):
            out.append(build_product(agent, task, workload.letters[i][j], presink_literal))
    return out
