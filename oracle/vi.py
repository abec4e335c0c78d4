"""Scalarised value iteration, policy extraction and policy evaluation on one
product model, in FP64 (appendix A.5, Alg. 3 and Alg. 4).

Readings taken here:
  * Both loops of Alg. 3 / Alg. 4 are do-while loops (they start with the
    stability flag raised; the algorithm package's DoWhile form is meant).
  * Jacobi iteration with two buffers instead of the in-place update: sweep n
    computes y = T(x_{n-1}) from x_0 = 0 and stops at the first n with
    max_s |y - x_{n-1}| <= eps, returning that sweep's y.  The fixed point is
    the same; only where the iteration stops changes.
  * Stage retirement inside the iteration (``stage_retired_value_iteration``):
    a stage (height of its location group in the product's location DAG)
    stops being backed up in a column once every lower stage has stopped and
    its own largest change is <= eps; its values stay those of that sweep.
  * The policy is extracted from the final values, not along the trajectory
    (the trajectory rule of Alg. 3 is kept as ``policy_rule="paper"``, parity
    unpinned).
  * Tie rule: the eps-optimal action set A*(s) = {a : Q(s,a) >= max Q - tau}
    with Q in FP64 at the returned values.  Done states have rank 0; an
    unranked state gets rank l+1 when some a in A*(s) moves mass into the done
    set or into a state of rank <= l; its action is the one among those that
    moves the most probability into done or into states of rank <= l (masses
    within 1e-12 count as equal; then the lowest index wins).  Taking merely the
    lowest-index qualifying action is proper too, but may progress only through
    a rare slip and so take tens of thousands of steps on average.
    When the rounds stop with states left unranked (near-ties below the
    accuracy of eps-converged values can close cycles of strict argmax
    choices, e.g. where many actions reach the goal with probability ~1), the
    tolerance of the unranked states only is widened tenfold, 1e-9 -> 1e-3,
    and the rounds go on; ranked states keep their choice.  States still
    unranked make the policy improper (an error).  The chosen policy reaches
    done with probability 1 and is tau-greedy for the values.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .product import Product


class ImproperPolicy(RuntimeError):
    pass


def scalarised_rewards(prod: Product, wc, wp) -> np.ndarray:
    """Row rewards (w . rho)(s,q,a) = wc * rho_i + wp * rho_{j+|I|} for each
    column: ``wc`` / ``wp`` are scalars or [K] arrays.  Returns [R, K]."""
    wc = np.atleast_1d(np.asarray(wc, dtype=np.float64))
    wp = np.atleast_1d(np.asarray(wp, dtype=np.float64))
    return prod.rew_cost[:, None] * wc[None, :] + prod.rew_prob[:, None] * wp[None, :]


def _state_max(prod: Product, q: np.ndarray) -> np.ndarray:
    return np.maximum.reduceat(q, prod.state_row[:-1], axis=0)


def value_iteration(prod: Product, wc, wp, eps: float, max_sweeps: int = 1_000_000):
    """Alg. 3 for K weight columns at once, each column stopping on its own.

    Returns (y [S, K], sweeps [K]); column k of y is the values of the first
    sweep whose residual max_s |y - x| is <= eps."""
    r = scalarised_rewards(prod, wc, wp)
    K = r.shape[1]
    S = prod.n_states
    x = np.zeros((S, K))
    sweeps = np.zeros(K, dtype=np.int64)
    if S == 0:
        return x, sweeps
    P = prod.P()
    active = np.ones(K, dtype=bool)
    n = 0
    while active.any():
        n += 1
        if n > max_sweeps:
            raise RuntimeError("value iteration did not converge")
        cols = np.flatnonzero(active)
        y = _state_max(prod, r[:, cols] + P @ x[:, cols])
        res = np.abs(y - x[:, cols]).max(axis=0)
        x[:, cols] = y
        done = res <= eps
        sweeps[cols[done]] = n
        active[cols[done]] = False
    return x, sweeps


def location_stages(prod: Product) -> np.ndarray:
    """Stage of every live state for the stage-ordered iteration.

    The location graph has an edge q -> q' when a live transition leads from a
    state at location q to a state at q'.  Its strongly connected groups form
    a DAG; a group's stage is its height there (0 for a group with no other
    successor group, else one more than the highest successor group).  Every
    transition therefore leads to the same or a lower stage, and groups of one
    stage have no transitions between them.  Returns int64 [S]."""
    from scipy.sparse.csgraph import connected_components
    S = prod.n_states
    if S == 0:
        return np.zeros(0, dtype=np.int64)
    locs, loc_of = np.unique(prod.states[:, 1], return_inverse=True)
    L = len(locs)
    src = loc_of[np.repeat(prod.row_state(), np.diff(prod.row_ptr))]
    dst = loc_of[prod.col]
    g = sp.csr_matrix((np.ones(len(src)), (src, dst)), shape=(L, L))
    n_groups, group = connected_components(g, directed=True, connection="strong")
    succ = [set() for _ in range(n_groups)]
    for a, b in zip(group[src], group[dst]):
        if a != b:
            succ[a].add(b)
    height = [-1] * n_groups

    def h(u):
        if height[u] < 0:
            height[u] = 1 + max((h(v) for v in succ[u]), default=-1)
        return height[u]

    for u in range(n_groups):
        h(u)
    return np.asarray(height, dtype=np.int64)[group[loc_of]]


def stage_ordered_value_iteration(prod: Product, wc, wp, eps: float, max_sweeps: int = 1_000_000):
    """Value iteration stage by stage (the staged form of Alg. 3 that the
    acyclic stages of a reach-sequence automaton allow).

    Stages (``location_stages``) are solved in increasing order.  Stage g
    runs the Jacobi sweeps of ``value_iteration`` over its own states only,
    from 0, reading the values of lower stages as final, until its residual
    over its own states is <= eps (each column on its own).  The fixed point
    is the one of Alg. 3; the stopping points differ.

    Returns (y [S, K], sweeps [n_stages, K])."""
    r = scalarised_rewards(prod, wc, wp)
    K = r.shape[1]
    S = prod.n_states
    x = np.zeros((S, K))
    if S == 0:
        return x, np.zeros((0, K), dtype=np.int64)
    stage = location_stages(prod)
    n_stages = int(stage.max()) + 1
    sweeps = np.zeros((n_stages, K), dtype=np.int64)
    P = prod.P()
    for g in range(n_stages):
        sel = np.flatnonzero(stage == g)
        counts = np.diff(prod.state_row)[sel]
        assert (counts > 0).all()
        offsets = np.concatenate([[0], np.cumsum(counts)[:-1]])
        rows = np.repeat(prod.state_row[sel], counts) + (np.arange(counts.sum()) - np.repeat(offsets, counts))
        Pg, rg = P[rows], r[rows]
        active = np.ones(K, dtype=bool)
        n = 0
        while active.any():
            n += 1
            if n > max_sweeps:
                raise RuntimeError("value iteration did not converge")
            cols = np.flatnonzero(active)
            y = np.maximum.reduceat(rg[:, cols] + Pg @ x[:, cols], offsets, axis=0)
            res = np.abs(y - x[np.ix_(sel, cols)]).max(axis=0)
            x[np.ix_(sel, cols)] = y
            done = res <= eps
            sweeps[g, cols[done]] = n
            active[cols[done]] = False
    return x, sweeps


def stage_retired_value_iteration(prod: Product, wc, wp, eps: float, max_sweeps: int = 1_000_000):
    """Value iteration in which stages retire inside the Jacobi iteration
    (the staged form of Alg. 3 that keeps the plain sweep count).

    Every sweep backs up the states of the stages still active in a column
    (``location_stages``) from the previous sweep's values, exactly as
    ``value_iteration``; the states of a retired stage keep their values.
    After the sweep the stages of each column are taken in increasing order:
    a stage retires when every lower stage has retired (in an earlier sweep or
    in this one) and the largest change over its own states in this sweep is
    <= eps.  A column is done when all its stages have retired; with one
    stage this is ``value_iteration`` itself.  The fixed point is the one of
    Alg. 3; the stopping points differ.

    Returns (y [S, K], retired [n_stages, K] = the sweep in which each stage
    retired, backups = the rows backed up over all sweeps and columns)."""
    r = scalarised_rewards(prod, wc, wp)
    K = r.shape[1]
    S = prod.n_states
    x = np.zeros((S, K))
    if S == 0:
        return x, np.zeros((0, K), dtype=np.int64), 0
    stage = location_stages(prod)
    n_stages = int(stage.max()) + 1
    rows_of_stage = np.bincount(stage, weights=np.diff(prod.state_row), minlength=n_stages).astype(np.int64)
    retired = np.zeros((n_stages, K), dtype=np.int64)   # 0 = not yet
    P = prod.P()
    backups = 0
    n = 0
    while (retired == 0).any():
        n += 1
        if n > max_sweeps:
            raise RuntimeError("value iteration did not converge")
        live = retired == 0                       # [n_stages, K] stages swept now
        y = _state_max(prod, r + P @ x)
        swept = live[stage]                       # [S, K]
        y = np.where(swept, y, x)
        change = np.abs(y - x)
        backups += int((rows_of_stage[:, None] * live).sum())
        for k in range(K):
            lower_done = True
            for g in range(n_stages):
                if retired[g, k]:
                    continue
                res = change[stage == g, k].max()
                if lower_done and res <= eps:
                    retired[g, k] = n
                else:
                    lower_done = False
        x = y
    return x, retired, backups


def q_values(prod: Product, x: np.ndarray, wc, wp) -> np.ndarray:
    """Q(s,a) = (w . rho)(s,a) + sum_s' P(s,a,s') x(s') for every row, [R, K]."""
    x2 = x.reshape(prod.n_states, -1)
    return scalarised_rewards(prod, wc, wp) + prod.P() @ x2


TAU_STEPS = 6   # widenings of the tie tolerance: tau * 10**k, k <= 6


def extract_policy(prod: Product, x: np.ndarray, wc: float, wp: float,
                   tau: float = 1e-9, return_tau: bool = False):
    """Attractor tie rule on the eps-optimal action sets (module doc).

    ``x`` is one column of values.  Returns mu[S], the chosen row of each
    state counted from the state's first row (int64); with ``return_tau``
    also the tolerance each state's choice was made with (tau, or tau * 10^k
    after k widenings), as (mu, tau_used)."""
    S = prod.n_states
    if S == 0:
        z = np.zeros(0, dtype=np.int64)
        return (z, np.zeros(0)) if return_tau else z
    Q = q_values(prod, x, wc, wp)[:, 0]
    row_state = prod.row_state()
    qmax = _state_max(prod, Q[:, None])[:, 0]
    opt = Q >= qmax[row_state] - tau
    # structural successor matrix: B[r, s'] = 1 iff row r reaches live s'
    B = sp.csr_matrix((np.ones(prod.nnz), prod.col, prod.row_ptr),
                      shape=(prod.n_rows, S))
    rank = np.full(S, -1, dtype=np.int64)
    mu = np.full(S, -1, dtype=np.int64)
    tau_used = np.zeros(S)
    first_row = prod.state_row[:-1]
    level = 0
    widen = 0
    while True:
        ranked_before = (rank >= 0)
        # a row qualifies if it is eps-optimal and moves mass into done or
        # into a state ranked in an earlier round
        hits = opt & (prod.to_done | (B @ ranked_before.astype(np.float64) > 0))
        cand = hits & ~ranked_before[row_state]
        if not cand.any():
            if ranked_before.all() or widen == TAU_STEPS:
                break
            widen += 1
            loose = Q >= qmax[row_state] - tau * 10.0 ** widen
            opt = np.where(ranked_before[row_state], opt, loose)
            continue
        level += 1
        rows = np.flatnonzero(cand)
        # mass into done, then into earlier-ranked states, in entry order
        for s in np.unique(row_state[rows]):
            best_r, best_m = -1, -1.0
            for r in rows[row_state[rows] == s]:
                a, b = prod.row_ptr[r], prod.row_ptr[r + 1]
                m = 0.0
                if prod.to_done[r]:
                    live = 0.0
                    for e in range(a, b):
                        live += prod.prob[e]
                    m = 1.0 - live
                for e in range(a, b):
                    if ranked_before[prod.col[e]]:
                        m += prod.prob[e]
                if m > best_m + 1e-12:
                    best_r, best_m = r, m
            rank[s] = level
            mu[s] = best_r - first_row[s]
            tau_used[s] = tau * 10.0 ** widen
    if (rank < 0).any():
        raise ImproperPolicy(f"{int((rank < 0).sum())} states cannot reach done "
                             "through eps-optimal actions")
    return (mu, tau_used) if return_tau else mu


def extract_policy_paper(prod: Product, wc: float, wp: float, eps: float,
                         max_sweeps: int = 1_000_000) -> np.ndarray:
    """Alg. 3 as printed: Gauss-Seidel sweeps in state order, the maximising
    action (first one on ties) recorded only where |y - x| > eps, mu
    initialised to the first action.  The policy depends on the trajectory
    (where each state's value last moved by more than eps), so the device
    does not use it; it is pinned where the optimal action is unique (the
    corridor, the worked example, brute force on tiny products)."""
    S = prod.n_states
    r = scalarised_rewards(prod, wc, wp)[:, 0]
    x = np.zeros(S)
    mu = np.zeros(S, dtype=np.int64)
    for _ in range(max_sweeps):
        stable = True
        for s in range(S):
            best, arg = -np.inf, 0
            for rr in range(prod.state_row[s], prod.state_row[s + 1]):
                a, b = prod.row_ptr[rr], prod.row_ptr[rr + 1]
                v = r[rr] + float(np.dot(prod.prob[a:b], x[prod.col[a:b]]))
                if v > best:
                    best, arg = v, rr - prod.state_row[s]
            if abs(best - x[s]) > eps:
                stable = False
                mu[s] = arg
            x[s] = best
        if stable:
            return mu
    raise RuntimeError("value iteration did not converge")


def policy_rows(prod: Product, mu: np.ndarray) -> np.ndarray:
    return prod.state_row[:-1] + mu


def evaluate(prod: Product, mu: np.ndarray, eps: float, max_sweeps: int = 10_000_000):
    """Alg. 4 for both objectives of the model: Jacobi from 0 on the fixed
    policy, each objective stopping at its first sweep with residual <= eps.

    Returns ((cost value, probability value) at the initial state,
    (sweeps_cost, sweeps_prob), full value vectors [S, 2])."""
    S = prod.n_states
    if S == 0 or prod.init < 0:
        return (0.0, 0.0), (0, 0), np.zeros((S, 2))
    rows = policy_rows(prod, mu)
    P = prod.P()[rows]
    rho = np.stack([prod.rew_cost[rows], prod.rew_prob[rows]], axis=1)
    x = np.zeros((S, 2))
    sweeps = np.zeros(2, dtype=np.int64)
    active = np.ones(2, dtype=bool)
    n = 0
    while active.any():
        n += 1
        if n > max_sweeps:
            raise RuntimeError("policy evaluation did not converge")
        cols = np.flatnonzero(active)
        y = rho[:, cols] + P @ x[:, cols]
        res = np.abs(y - x[:, cols]).max(axis=0)
        x[:, cols] = y
        done = res <= eps
        sweeps[cols[done]] = n
        active[cols[done]] = False
    return (float(x[prod.init, 0]), float(x[prod.init, 1])), tuple(int(v) for v in sweeps), x


def evaluate_exact(prod: Product, mu: np.ndarray) -> np.ndarray:
    """Exact values of both objectives under mu: solve (I - P_mu) x = rho_mu.
    Returns x [S, 2]."""
    S = prod.n_states
    if S == 0:
        return np.zeros((0, 2))
    rows = policy_rows(prod, mu)
    A = sp.identity(S, format="csc") - prod.P()[rows].tocsc()
    rho = np.stack([prod.rew_cost[rows], prod.rew_prob[rows]], axis=1)
    return np.column_stack([spla.spsolve(A, rho[:, 0]), spla.spsolve(A, rho[:, 1])])


def optimal_exact(prod: Product, wc: float, wp: float, tau: float = 1e-9, max_iter: int = 100):
    """Exact optimal scalarised values by policy iteration, the ground truth
    for comparing chosen actions: value iteration (Alg. 3) to a tight
    tolerance gives a first proper policy (attractor tie rule), which is then
    evaluated exactly (a sparse linear solve) and improved greedily on its own
    exact values until no action beats the evaluated values by more than
    1e-12 max(1, |v|).  Returns (v[S], Q[R], err) where Q are the one-step
    values of every row at v and err = max_s |max_a Q(s, a) - v(s)|, the
    Bellman residual of the result."""
    S = prod.n_states
    if S == 0:
        return np.zeros(0), np.zeros(0), 0.0
    x, _ = value_iteration(prod, wc, wp, 1e-11)
    x = x[:, 0]
    w = np.array([wc, wp], dtype=np.float64)
    for _ in range(max_iter):
        mu = extract_policy(prod, x, wc, wp, tau)
        v = evaluate_exact(prod, mu) @ w
        Q = q_values(prod, v, wc, wp)[:, 0]
        qmax = _state_max(prod, Q[:, None])[:, 0]
        scale = max(1.0, float(np.abs(v).max()))
        if (qmax <= v + 1e-12 * scale).all():
            return v, Q, float(np.abs(qmax - v).max())
        x = v
    raise RuntimeError("policy iteration did not settle")


def q_gaps(prod: Product, Q: np.ndarray) -> tuple:
    """Per state: the best row (counted from the state's first row, lowest
    index among equal values) and the gap to the next best row's value (inf
    for a state with one row)."""
    S = prod.n_states
    best = np.zeros(S, dtype=np.int64)
    gap = np.full(S, np.inf)
    for s in range(S):
        q = Q[prod.state_row[s]:prod.state_row[s + 1]]
        order = np.argsort(-q, kind="stable")
        best[s] = order[0]
        if q.size > 1:
            gap[s] = q[order[0]] - q[order[1]]
    return best, gap
