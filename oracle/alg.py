"""Alg. 2 (supporting hyperplane for a weight vector) and Alg. 1
(point-oriented Pareto computation), Sec. 3.3, in FP64.

Readings taken here:
  * Objective order: d = |I| + |J| with the |I| agent costs first and then the
    |J| task probabilities (Alg. 1 input t = (c, p); Sec. 3.1).
  * More tasks than agents: an assignment is a bijection when |I| = |J|
    (Sec. 2, "Random Assignment"); agents are re-used for further tasks
    (Sec. 1), so with |J| > |I| each agent may take up to ceil(|J|/|I|) tasks:
    the assignment problem is solved on the matrix with every agent row
    repeated that many times (padded with zero-value dummy tasks when the rows
    outnumber the tasks).  An agent's cost objective is the sum of the costs of
    all tasks it receives; an agent with no task has cost 0.
  * Loop control: t_up is recomputed right after each new point is added and
    ||t_down - t_up||_M <= eps is tested at once (this never divides 0/0 in the
    weight update).  Each loop pass costs one call of Alg. 2.
  * Verdict: FEASIBLE iff t lies in down(Phi); INFEASIBLE iff some (w', r') in
    Lambda has w'.r' < w'.t (the outer approximation separates t); otherwise
    UNDECIDED (only possible for eps > 0).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
from scipy.optimize import linear_sum_assignment

from . import vi, geometry

FEASIBLE, INFEASIBLE, UNDECIDED = 1, 0, 2


def assign(c: np.ndarray) -> np.ndarray:
    """Assignment f maximising sum_j c[f(j), j] (Alg. 2, assignment step),
    with agent re-use when |J| > |I| (module doc).  c is [|I|, |J|]; returns
    f[|J|] (agent of each task)."""
    nI, nJ = c.shape
    cap = max(1, -(-nJ // nI))
    rows = np.repeat(np.arange(nI), cap)
    big = c[rows]
    if big.shape[0] > nJ:
        big = np.hstack([big, np.zeros((big.shape[0], big.shape[0] - nJ))])
    ri, cj = linear_sum_assignment(big, maximize=True)
    f = np.full(nJ, -1, dtype=np.int64)
    for r, j in zip(ri, cj):
        if j < nJ:
            f[j] = rows[r]
    return f


@dataclass
class SupportResult:
    r: np.ndarray            # [d]
    c: np.ndarray            # [|I|, |J|] scalarised optimum at each initial state
    f: np.ndarray            # [|J|]
    policies: list           # mu of each assigned model (task order)
    vi_sweeps: np.ndarray    # [|I|, |J|]
    values: list             # final VI values of every model (m = i*|J| + j)


def policy_for(prod, wi: float, wj: float, eps_vi: float, tau: float = 1e-9) -> np.ndarray:
    """The policy of one model under weights (wi, wj): value iteration on the
    two weights scaled to sum 1, then the tie rule.  Scaling leaves the
    optimal policies of the scalarised model unchanged (Alg. 3 maximises
    wi rho_i + wj rho_j); it keeps the absolute stop test and the tie
    tolerance meaningful when both weights are tiny."""
    sc = wi + wj
    if sc > 0:
        wi, wj = wi / sc, wj / sc
    x, _ = vi.value_iteration(prod, np.array([wi]), np.array([wj]), policy_eps(eps_vi, wi, wj))
    return vi.extract_policy(prod, x[:, 0], wi, wj, tau)


def policy_eps(eps_vi: float, wi: float, wj: float) -> float:
    """Stop of the values a policy is chosen from (weights scaled to sum 1):
    eps_vi, or eps_vi * 1e-4 (not below 1e-12, never above eps_vi) when the
    cost weight vanishes.  Every action that completes the task as surely as
    the best is then optimal, and values stopped at eps_vi differ between
    such actions by their own error, far above the tie tolerance: the greedy
    choice among them would be decided by that error and can progress only
    through a slip (hundreds of thousands of expected steps)."""
    if wi < 1e-6 and wj > 0:
        return min(eps_vi, max(eps_vi * 1e-4, 1e-12))
    return eps_vi


def support(products, nI: int, nJ: int, w: np.ndarray, eps_vi: float,
            eps_eval: Optional[float] = None, tau: float = 1e-9) -> SupportResult:
    """Alg. 2 for one weight vector w [d]."""
    eps_eval = eps_vi if eps_eval is None else eps_eval
    c = np.zeros((nI, nJ))
    sweeps = np.zeros((nI, nJ), dtype=np.int64)
    values = []
    for i in range(nI):
        for j in range(nJ):
            prod = products[i * nJ + j]
            y, n = vi.value_iteration(prod, w[i], w[nI + j], eps_vi)
            values.append(y[:, 0])
            sweeps[i, j] = n[0]
            c[i, j] = y[prod.init, 0] if prod.init >= 0 else 0.0
    f = assign(c)
    r = np.zeros(nI + nJ)
    policies = []
    for j in range(nJ):
        i = int(f[j])
        prod = products[i * nJ + j]
        mu = policy_for(prod, w[i], w[nI + j], eps_vi, tau)
        (vc, vp), _, _ = vi.evaluate(prod, mu, eps_eval)
        r[nI + j] = vp
        r[i] += vc
        policies.append(mu)
    return SupportResult(r=r, c=c, f=f, policies=policies, vi_sweeps=sweeps, values=values)


@dataclass
class QueryResult:
    verdict: int
    t_up: np.ndarray
    t_down: np.ndarray
    iterations: int
    Phi: List[np.ndarray] = field(default_factory=list)
    W: List[np.ndarray] = field(default_factory=list)
    lam: Optional[np.ndarray] = None
    trace: list = field(default_factory=list)   # (w, r, t_up, t_down) per pass


def query(products, nI: int, nJ: int, t: np.ndarray, eps: float, eps_vi: float,
          M: Optional[np.ndarray] = None, max_iter: int = 64, eps_eval=None,
          first_w: Optional[np.ndarray] = None, verification_only: bool = False,
          support_fn=None) -> QueryResult:
    """Alg. 1: decide whether t is feasible and find the closest Pareto point.

    ``first_w`` replaces the initial weight (1, 0, ..., 0).  With
    ``verification_only`` the loop stops as soon as the outer approximation
    separates t (Sec. 5, Experiment 2 setting)."""
    t = np.asarray(t, dtype=np.float64)
    d = nI + nJ
    sup = support_fn or (lambda w: support(products, nI, nJ, w, eps_vi, eps_eval).r)
    w = np.zeros(d)
    w[0] = 1.0
    if first_w is not None:
        w = np.asarray(first_w, dtype=np.float64)
    t_down = t.copy()
    t_up = np.full(d, -np.inf)
    Phi, Ws = [], []
    lam = None
    trace = []
    separated = False
    for it in range(1, max_iter + 1):
        r = sup(w)
        Phi.append(r)
        Ws.append(w.copy())
        if w @ r < w @ t_down:
            if verification_only:
                separated = True
            t_down = geometry.project_outer(np.array(Ws), np.array(Phi), t, M)
        t_up, lam = geometry.project_inner(np.array(Phi), t, M)
        trace.append((w.copy(), r.copy(), t_up.copy(), t_down.copy()))
        if separated or geometry.mnorm(t_down - t_up, M) <= eps:
            break
        w = geometry.weight_from(t, t_up, M)
        if w is None:          # t_up = t up to rounding
            break
    verdict = verdict_of(t, t_up, np.array(Ws), np.array(Phi), M)
    return QueryResult(verdict=verdict, t_up=t_up, t_down=t_down, iterations=len(Phi),
                       Phi=Phi, W=Ws, lam=lam, trace=trace)


@dataclass
class Synthesis:
    picked: np.ndarray       # passes with v > 0
    v: np.ndarray            # their weights, scaled to sum 1
    F: np.ndarray            # [m, |J|] assignment of each picked pass
    R: np.ndarray            # [m, d] its point
    matrix: np.ndarray       # [|I|, |J|] probability that agent i serves task j
    policies: list           # [m][|J|] scheduler of task j in pass m (model (F[m, j], j))


def synthesis(products, nI: int, nJ: int, Ws, v, eps_vi: float, eps_eval: Optional[float] = None,
              tau: float = 1e-9) -> Synthesis:
    """The answer extracted after Alg. 1 (Sec. 3.3, end): v is a convex
    weighting of the passes' points whose combination dominates t_up (the
    inner projection's weights); pass i's assignment f_i is drawn with
    probability v_i, and task j then runs the scheduler that pass computed for
    model (f_i(j), j).  The passes with v_i > 0 are replayed with Alg. 2 on
    their weight vectors; the convex combination of their assignments is the
    random assignment (each task served with probability 1)."""
    v = np.asarray(v, dtype=np.float64)
    picked = np.nonzero(v > 0)[0]
    vs = v[picked] / v[picked].sum()
    F, R, pol = [], [], []
    matrix = np.zeros((nI, nJ))
    for q, i in enumerate(picked):
        res = support(products, nI, nJ, np.asarray(Ws[i], dtype=np.float64), eps_vi, eps_eval, tau)
        F.append(res.f)
        R.append(res.r)
        pol.append(res.policies)
        for j in range(nJ):
            matrix[res.f[j], j] += vs[q]
    return Synthesis(picked=picked, v=vs, F=np.array(F), R=np.array(R), matrix=matrix, policies=pol)


def verdict_of(t, t_up, Ws, Rs, M=None, tol_in=1e-9, tol_sep=1e-12) -> int:
    if geometry.mnorm(t - t_up, M) <= tol_in:
        return FEASIBLE
    if (np.einsum("ij,ij->i", Ws, Rs) < Ws @ t - tol_sep).any():
        return INFEASIBLE
    return UNDECIDED
