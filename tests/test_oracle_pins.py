"""Pins of the FP64 oracle against what the paper and the mathematics fix:
printed values of the worked example, closed forms, brute force over
deterministic policies, the multi-objective LP, the centralised MDP, Dijkstra,
exact linear solves and textbook assignment.  CPU only."""
import itertools
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.optimize import linprog, linear_sum_assignment, minimize
from scipy.sparse.csgraph import dijkstra

from workloads import worked_example, tiny_workload, make_workload
from workloads.gridworld import Agent, Task, Workload, make_task_dfa, make_grid, make_agent
from oracle import product, vi, alg, geometry, centralised

HERE = os.path.dirname(__file__)
GOLD = json.load(open(os.path.join(HERE, "golden", "worked_example.json")))


# --------------------------------------------------------------------------
# worked example (Sec. 3.3 Example, Fig. 3)
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def example():
    wl = worked_example()
    return product.build_all(wl)


def test_example_product_structure(example):
    p = example[0]
    # live states (s0, q0) and (s2, q0); s1 is a trap, s3 accepts
    assert p.states.tolist() == [[0, 0], [2, 0]]
    assert p.state_row.tolist() == [0, 2, 3]
    assert p.row_ptr.tolist() == [0, 2, 2, 2]
    assert p.col.tolist() == [0, 1] and np.allclose(p.prob, [0.3, 0.5])
    assert np.allclose(p.rew_prob, [0.0, 0.1, 1.0])
    assert np.allclose(p.rew_cost, [-1, -1, -1]) and p.to_done.all() and p.init == 0


def test_example_policy_points(example):
    # policy b: one step, accept w.p. .1; policy a: cost 15/7, prob 5/7
    rb = alg.support(example, 1, 1, np.array([1.0, 0.0]), 1e-13).r
    ra = alg.support(example, 1, 1, np.array([0.0, 1.0]), 1e-13).r
    assert np.allclose(rb, [-1.0, 0.1], atol=1e-12)
    assert np.allclose(ra, [-15 / 7, 5 / 7], atol=1e-12)


def test_example_figure_polygon(example):
    # Fig. 3b is itself split between the two readings: its r1 vertex is the
    # literal pre-sink point, its r2 vertex the standard-reading point
    poly = np.array(GOLD["fig3b_polygon"])
    r1 = (3 * poly[2, 0], poly[2, 1])
    r2 = (3 * poly[3, 0], poly[3, 1])
    assert np.allclose(r1, GOLD["printed_r1"], atol=0.005)
    assert np.allclose(r2, [-15 / 7, 5 / 7], atol=0.005)


def test_example_literal_presink_reproduces_printed_r1():
    wl = worked_example()
    prods = product.build_all(wl, presink_literal=True)
    r1 = alg.support(prods, 1, 1, np.array([1.0, 0.0]), 1e-13).r
    assert np.allclose(r1, GOLD["printed_r1"], atol=1e-12)


def test_example_feasible_threshold(example):
    q = alg.query(example, 1, 1, np.array(GOLD["t_a"]), GOLD["eps"], 1e-13)
    assert q.verdict == alg.FEASIBLE and q.iterations == 2
    w1, r1, t_up1, t_down1 = q.trace[0]
    # after r1 the gap ||t_down - t_up|| is the printed 0.6
    assert geometry.mnorm(t_down1 - t_up1) == pytest.approx(GOLD["printed_gap_after_r1_for_t_a"], abs=1e-12)
    assert np.allclose(q.t_up, GOLD["t_a"]) and np.allclose(q.t_down, GOLD["t_a"])


def test_example_infeasible_threshold(example):
    q = alg.query(example, 1, 1, np.array(GOLD["t_u"]), GOLD["eps"], 1e-13)
    assert q.verdict == alg.INFEASIBLE
    assert q.iterations == 3
    assert geometry.mnorm(q.t_down - q.t_up) <= GOLD["eps"]
    # closest point on the segment between the two policy points
    A, B, t = np.array([-15 / 7, 5 / 7]), np.array([-1.0, 0.1]), np.array(GOLD["t_u"])
    n = np.array([-(B - A)[1], (B - A)[0]])
    n = n if n @ (t - A) > 0 else -n
    star = t - (n @ (t - A)) / (n @ n) * n
    assert np.allclose(q.t_down, star, atol=1e-9)


def test_example_printed_points_give_printed_closest_point():
    # the inner projection of t_u onto the printed points is the printed t_down
    Phi = np.array([GOLD["printed_r1"], [-15 / 7, 5 / 7]])
    x, lam = geometry.project_inner(Phi, np.array(GOLD["t_u"]))
    assert np.allclose(x, GOLD["printed_t_down_for_t_u"], atol=0.005)
    assert geometry.kkt_inner(Phi, np.array(GOLD["t_u"]), x, lam) < 1e-10


# --------------------------------------------------------------------------
# hand-worked closed forms
# --------------------------------------------------------------------------

def _agent(succ_rows, costs, init=0):
    """Agent from explicit rows: succ_rows[s][a] = [(s', p), ...]."""
    nA = max(len(r) for r in succ_rows)
    sa_ptr, succ, prob, cost = [0], [], [], []
    for s, rows in enumerate(succ_rows):
        for a in range(nA):
            if a < len(rows):
                for t, p in rows[a]:
                    succ.append(t)
                    prob.append(p)
            cost.append(costs[a] if a < len(rows) else 0.0)
            sa_ptr.append(len(succ))
    n = len(succ_rows)
    return Agent(width=n, height=1, cells=np.arange(n, dtype=np.int32), init=init, p_slip=0.0,
                 action_cost=np.asarray(costs, float), n_actions=nA,
                 sa_ptr=np.asarray(sa_ptr, np.int32), succ=np.asarray(succ, np.int32),
                 prob=np.asarray(prob, float), cost=np.asarray(cost, float))


def _task(kind, k):
    n, L, q0, delta, acc = make_task_dfa(kind, k)
    return Task(kind=kind, k=k, n_locs=n, n_letters=L, q0=q0, delta=delta, accepting=acc,
                waypoints_uv=np.zeros((k, 2, 2)), avoid_uv=None)


def _corridor(p, c):
    # cells 0,1,2; action 0 "right" succeeds w.p. p else stays; action 1 stays
    rows = [[[(1, p), (0, 1 - p)], [(0, 1.0)]],
            [[(2, p), (1, 1 - p)], [(1, 1.0)]],
            [[(2, 1.0)], [(2, 1.0)]]]
    a = _agent(rows, [c, c])
    letters = np.array([0, 0, 1], np.int32)
    return product.build_product(a, _task("reach", 1), letters)


@pytest.mark.parametrize("p,c", [(0.5, 1.0), (0.8, 2.5), (0.3, 1.7)])
def test_corridor_closed_form(p, c):
    prod = _corridor(p, c)
    y, _ = vi.value_iteration(prod, 1.0, 0.0, 1e-13)
    assert y[prod.init, 0] == pytest.approx(-2 * c / p, rel=1e-10)
    mu = vi.extract_policy(prod, y[:, 0], 1.0, 0.0)
    assert (mu == 0).all()
    (vc, vp), _, _ = vi.evaluate(prod, mu, 1e-13)
    assert vc == pytest.approx(-2 * c / p, rel=1e-10) and vp == pytest.approx(1.0, abs=1e-12)


@pytest.mark.parametrize("p,c", [(0.5, 1.0), (0.8, 2.5), (0.3, 1.7)])
def test_paper_policy_rule_on_the_corridor(p, c):
    # Alg. 3's own policy rule (trajectory form): "right" is the unique
    # optimal action of both live cells for the cost objective
    prod = _corridor(p, c)
    mu = vi.extract_policy_paper(prod, 1.0, 0.0, 1e-12)
    assert mu.tolist() == [0, 0]


def test_paper_policy_rule_on_the_worked_example(example):
    """Probability only: policy a (row 0 of (s0, q0), 5/7 against 0.1) in
    both rules.  Cost only, the optimum is policy b (row 1, one step) and the
    final-value rule finds it; the printed rule records row 0 at the first
    sweep (both rows give -1 from x = 0, the first wins the tie) and never
    again, because the value of (s0, q0) stays at -1 while the best row
    changes: the trajectory dependence that makes the build extract policies
    from the final values instead."""
    p = example[0]
    assert vi.extract_policy_paper(p, 0.0, 1.0, 1e-12).tolist() == [0, 0]
    assert vi.extract_policy_paper(p, 1.0, 0.0, 1e-12).tolist() == [0, 0]
    y, _ = vi.value_iteration(p, 1.0, 0.0, 1e-12)
    assert vi.extract_policy(p, y[:, 0], 1.0, 0.0).tolist() == [1, 0]
    # the printed rule's policy a costs 15/7 against b's 1
    assert vi.evaluate_exact(p, np.array([0, 0]))[p.init, 0] == pytest.approx(-15 / 7, abs=1e-12)


@pytest.mark.parametrize("seed,w,h,kind", [(11, 3, 2, "reach"), (12, 3, 3, "avoid"), (14, 3, 2, "avoid")])
def test_paper_policy_rule_is_optimal_on_tiny_products(seed, w, h, kind):
    # with both weights positive the optimum is unique by a margin here; the
    # trajectory rule's policy then attains the brute-force optimum exactly
    wl = tiny_workload(seed, 1, 1, width=w, height=h, kinds=(kind,), k=1)
    prod = product.build_all(wl)[0]
    pts, _ = _policy_points(prod)
    rng = np.random.default_rng(seed + 100)
    for _ in range(4):
        wv = rng.dirichlet([1.0, 1.0])
        vals = np.sort(pts @ wv)
        mu = vi.extract_policy_paper(prod, wv[0], wv[1], 1e-12)
        ex = vi.evaluate_exact(prod, mu)[prod.init] @ wv
        assert ex == pytest.approx(vals[-1], abs=1e-9)


def _widened_policy_loss(prod, wc, wp, noise, seed):
    """Optimal values V*, a policy extracted from values perturbed by
    `noise` (so the tie tolerance has to widen), and the bound on its loss."""
    vstar, _ = vi.value_iteration(prod, wc, wp, 1e-14)
    vstar = vstar[:, 0]
    x = vstar + np.random.default_rng(seed).uniform(-noise, noise, size=vstar.shape)
    mu, tau_used = vi.extract_policy(prod, x, wc, wp, tau=1e-9, return_tau=True)
    rows = vi.policy_rows(prod, mu)
    A = sp.identity(prod.n_states, format="csc") - prod.P()[rows].tocsc()
    vmu = vi.evaluate_exact(prod, mu) @ np.array([wc, wp])
    e = float(np.abs(x - vstar).max())
    # V* - V^mu <= (I - P_mu)^-1 (tau_used + 2 e): mu is tau_used-greedy for x,
    # and x is within e of V*
    bound = sp.linalg.spsolve(A, tau_used + 2 * e)
    return vstar, vmu, bound, tau_used


@pytest.mark.parametrize("noise", [1e-6, 1e-5, 3e-4])
def test_widened_tie_tolerance_loss_is_bounded(noise):
    """The tie rule's widening (tau up to 1e-3) picks actions up to tau below
    the best; the loss of the resulting policy is bounded by tau_used + 2 e
    per expected step.  Values perturbed by `noise` force widenings."""
    widened = 0
    for seed, (w, h, kind) in enumerate([(4, 4, "reach"), (5, 4, "avoid"), (6, 5, "reach")]):
        wl = tiny_workload(40 + seed, 1, 1, width=w, height=h, kinds=(kind,), k=2, p_slip=0.1)
        prod = product.build_all(wl)[0]
        for wc, wp in ((1.0, 0.0), (0.3, 0.7), (0.0, 1.0)):
            vstar, vmu, bound, tau_used = _widened_policy_loss(prod, wc, wp, noise, seed)
            widened += int((tau_used > 1e-9).sum())
            assert (vstar - vmu <= bound + 1e-9).all()
            # and the bound is what the values allow: at most 1e-3 + 2 noise per step
            assert (tau_used <= 1e-3 * (1 + 1e-12)).all()
    assert widened > 0   # the widening did happen


def test_widening_loss_pin_catches_a_non_greedy_choice(monkeypatch):
    # plant a mistake on the CPU: a tie rule that ignores the tolerance
    # (every action counts as optimal) breaks the loss bound
    wl = tiny_workload(40, 1, 1, width=4, height=4, kinds=("reach",), k=2, p_slip=0.1)
    prod = product.build_all(wl)[0]
    real_q = vi.q_values

    def flat_q(prod_, x, wc, wp):
        q = real_q(prod_, x, wc, wp)
        return np.zeros_like(q)

    monkeypatch.setattr(vi, "q_values", flat_q)
    vstar, vmu, bound, _ = _widened_policy_loss(prod, 1.0, 0.0, 1e-6, 0)
    assert (vstar - vmu > bound + 1e-3).any()


def test_corridor_probability_iterates_monotone():
    prod = _corridor(0.4, 1.0)
    P = prod.P()
    x = np.zeros(prod.n_states)
    for _ in range(60):
        y = np.maximum.reduceat(prod.rew_prob + P @ x, prod.state_row[:-1])
        assert (y >= x - 1e-15).all() and (y <= 1 + 1e-15).all()
        x = y


def _risky_safe(k, c, q):
    # state 0 decides; safe walks the chain 1..k-1 to the goal G (k steps);
    # risky reaches G w.p. q, else the avoid cell T
    G, T = k, k + 1
    rows = [[[(1 if k > 1 else G, 1.0)], [(G, q), (T, 1 - q)]]]
    for s in range(1, k):
        nxt = s + 1 if s + 1 < k else G
        rows.append([[(nxt, 1.0)], [(nxt, 1.0)]])
    rows.append([[(G, 1.0)], [(G, 1.0)]])
    rows.append([[(T, 1.0)], [(T, 1.0)]])
    a = _agent(rows, [c, c])
    letters = np.zeros(k + 2, np.int32)
    letters[G], letters[T] = 1, 2
    return product.build_product(a, _task("avoid", 1), letters)


def test_risky_safe_front_and_closest_point():
    k, c, q = 3, 1.0, 0.4
    prods = [_risky_safe(k, c, q)]
    rs = alg.support(prods, 1, 1, np.array([0.0, 1.0]), 1e-13).r
    rr = alg.support(prods, 1, 1, np.array([1.0, 0.0]), 1e-13).r
    assert np.allclose(rs, [-c * k, 1.0]) and np.allclose(rr, [-c, q])
    t = np.array([-1.5, 0.95])
    res = alg.query(prods, 1, 1, t, 1e-10, 1e-13)
    A, B = np.array([-c * k, 1.0]), np.array([-c, q])
    n = np.array([(B - A)[1] * -1, (B - A)[0]])
    n = n if n @ (t - A) > 0 else -n
    star = t - (n @ (t - A)) / (n @ n) * n
    assert res.verdict == alg.INFEASIBLE
    assert np.allclose(res.t_down, star, atol=1e-8) and np.allclose(res.t_up, star, atol=1e-8)
    # a threshold under the segment is feasible
    res2 = alg.query(prods, 1, 1, np.array([-2.5, 0.5]), 1e-10, 1e-13)
    assert res2.verdict == alg.FEASIBLE


# --------------------------------------------------------------------------
# brute force over deterministic policies
# --------------------------------------------------------------------------

def _policy_points(prod):
    """(cost, prob) at the initial state of every proper deterministic policy."""
    S = prod.n_states
    counts = np.diff(prod.state_row)
    pts, pols = [], []
    P = prod.P().toarray()
    for mu in itertools.product(*[range(n) for n in counts]):
        rows = prod.state_row[:-1] + np.array(mu)
        A = np.eye(S) - P[rows]
        # proper iff I - P_mu is invertible with a non-negative inverse
        try:
            inv = np.linalg.inv(A)
        except np.linalg.LinAlgError:
            continue
        if (inv < -1e-9).any() or np.abs(inv).max() > 1e9:
            continue
        x = inv @ np.stack([prod.rew_cost[rows], prod.rew_prob[rows]], axis=1)
        pts.append(x[prod.init])
        pols.append(np.array(mu))
    return np.array(pts), pols


@pytest.mark.parametrize("seed,w,h,kind", [(11, 3, 2, "reach"), (12, 3, 3, "avoid"), (13, 3, 3, "avoid")])
def test_scalarised_optimum_equals_brute_force(seed, w, h, kind):
    wl = tiny_workload(seed, 1, 1, width=w, height=h, kinds=(kind,), k=1)
    prod = product.build_all(wl)[0]
    pts, _ = _policy_points(prod)
    rng = np.random.default_rng(seed)
    for _ in range(5):
        wv = rng.dirichlet([1.0, 1.0])
        y, _ = vi.value_iteration(prod, wv[0], wv[1], 1e-13)
        best = (pts @ wv).max()
        assert y[prod.init, 0] == pytest.approx(best, abs=1e-9)
        mu = vi.extract_policy(prod, y[:, 0], wv[0], wv[1])
        ex = vi.evaluate_exact(prod, mu)[prod.init]
        assert ex @ wv == pytest.approx(best, abs=1e-9)


def _hull_top(points):
    """Points not dominated in every weighted direction (a superset of the
    vertices of down(conv) that matter): keep points optimal for some w."""
    keep = []
    for wv in np.linspace(0, 1, 201):
        wvec = np.array([wv, 1 - wv])
        keep.append(int(np.argmax(points @ wvec)))
    return points[sorted(set(keep))]


def _closest_brute(V, t):
    """min ||t - x|| over x <= V^T lam, lam in simplex, by SLSQP (independent
    of the least-distance route)."""
    m, d = V.shape
    fun = lambda z: float(np.sum(np.maximum(t - V.T @ z, 0.0) ** 2))
    cons = [{"type": "eq", "fun": lambda z: z.sum() - 1.0}]
    best = None
    for start in range(m):
        z0 = np.full(m, 0.1 / m)
        z0[start] += 0.9
        r = minimize(fun, z0, method="SLSQP", bounds=[(0, 1)] * m, constraints=cons,
                     options={"ftol": 1e-15, "maxiter": 500})
        if best is None or r.fun < best.fun:
            best = r
    return np.minimum(t, V.T @ best.x)


@pytest.mark.parametrize("seed", [21, 22])
def test_query_matches_brute_force_two_by_two(seed):
    wl = tiny_workload(seed, 2, 2, width=3, height=3, kinds=("avoid",), k=1, p_slip=0.3)
    prods = product.build_all(wl)
    tops = [_hull_top(_policy_points(p)[0]) for p in prods]
    # every point of C's generator set: per assignment, one top point per task
    V = []
    for f in [(0, 1), (1, 0)]:
        for a in tops[f[0] * 2 + 0]:
            for b in tops[f[1] * 2 + 1]:
                r = np.zeros(4)
                r[f[0]] += a[0]
                r[f[1]] += b[0]
                r[2], r[3] = a[1], b[1]
                V.append(r)
    V = np.array(V)
    rng = np.random.default_rng(seed)
    for _ in range(3):
        base = V[rng.integers(len(V))]
        t = base + np.array([0.3, 0.3, 0.05, 0.05]) * rng.uniform(-1, 2, 4)
        t[2:] = np.clip(t[2:], 0, 1)
        res = alg.query(prods, 2, 2, t, 1e-9, 1e-13, max_iter=200)
        # feasibility by LP over the generators
        lp = linprog(np.zeros(len(V)), A_ub=-V.T, b_ub=-t, A_eq=np.ones((1, len(V))), b_eq=[1],
                     bounds=[(0, None)] * len(V), method="highs")
        assert (res.verdict == alg.FEASIBLE) == (lp.status == 0)
        if res.verdict != alg.FEASIBLE:
            star = _closest_brute(V, t)
            assert np.allclose(res.t_down, star, atol=1e-5)


# --------------------------------------------------------------------------
# multi-objective LP (Fig. 2) and centralised MDP (Def. teamMDP)
# --------------------------------------------------------------------------

def _mo_lp(prods, nI, nJ):
    """Variables: x_{s,q,a} of every model, then x_ij.  Returns (A_eq, b_eq,
    objective rows [d, nvar])."""
    offs, n = [], 0
    for p in prods:
        offs.append(n)
        n += p.n_rows
    nx = n + nI * nJ
    Aeq, beq = [], []
    for m, p in enumerate(prods):
        i, j = divmod(m, nJ)
        rs = p.row_state()
        for s in range(p.n_states):
            row = np.zeros(nx)
            row[offs[m] + p.state_row[s]: offs[m] + p.state_row[s + 1]] += 1.0
            if s == p.init:
                row[n + i * nJ + j] -= 1.0
            for r in range(p.n_rows):
                for e in range(p.row_ptr[r], p.row_ptr[r + 1]):
                    if p.col[e] == s:
                        row[offs[m] + r] -= p.prob[e]
            Aeq.append(row)
            beq.append(0.0)
    for j in range(nJ):
        row = np.zeros(nx)
        row[n + np.arange(nI) * nJ + j] = 1
        Aeq.append(row)
        beq.append(1.0)
    for i in range(nI):
        row = np.zeros(nx)
        row[n + i * nJ + np.arange(nJ)] = 1
        Aeq.append(row)
        beq.append(1.0)
    obj = np.zeros((nI + nJ, nx))
    for m, p in enumerate(prods):
        i, j = divmod(m, nJ)
        obj[i, offs[m]:offs[m] + p.n_rows] += p.rew_cost
        obj[nI + j, offs[m]:offs[m] + p.n_rows] += p.rew_prob
    return np.array(Aeq), np.array(beq), obj


@pytest.mark.parametrize("seed", [31, 32])
def test_support_equals_lp_optimum(seed):
    wl = tiny_workload(seed, 2, 2, width=3, height=3, kinds=("avoid", "reach"), k=1, p_slip=0.2)
    prods = product.build_all(wl)
    Aeq, beq, obj = _mo_lp(prods, 2, 2)
    rng = np.random.default_rng(seed)
    for _ in range(3):
        w = rng.dirichlet(np.ones(4))
        s = alg.support(prods, 2, 2, w, 1e-13)
        lp = linprog(-(w @ obj), A_eq=Aeq, b_eq=beq, bounds=[(0, None)] * Aeq.shape[1], method="highs")
        assert lp.status == 0
        assert w @ s.r == pytest.approx(-lp.fun, abs=1e-8)
        # last equality of Lemma lem:face: w.r equals the assignment optimum
        assert w @ s.r == pytest.approx(sum(s.c[s.f[j], j] for j in range(2)), abs=1e-9)


@pytest.mark.parametrize("seed", [33])
def test_verdict_equals_lp_feasibility(seed):
    wl = tiny_workload(seed, 2, 2, width=3, height=3, kinds=("avoid",), k=1, p_slip=0.3)
    prods = product.build_all(wl)
    Aeq, beq, obj = _mo_lp(prods, 2, 2)
    pts = alg.support(prods, 2, 2, np.full(4, 0.25), 1e-13).r
    rng = np.random.default_rng(seed)
    for _ in range(6):
        t = pts + np.array([0.5, 0.5, 0.1, 0.1]) * rng.uniform(-1, 1, 4)
        t[2:] = np.clip(t[2:], 0, 1)
        lp = linprog(np.zeros(Aeq.shape[1]), A_ub=-obj, b_ub=-t, A_eq=Aeq, b_eq=beq,
                     bounds=[(0, None)] * Aeq.shape[1], method="highs")
        res = alg.query(prods, 2, 2, t, 1e-9, 1e-13, max_iter=200)
        slack = None
        if lp.status == 0 and res.verdict != alg.FEASIBLE:
            slack = geometry.mnorm(res.t_down - t)
        assert (res.verdict == alg.FEASIBLE) == (lp.status == 0) or (slack is not None and slack < 1e-6)


@pytest.mark.parametrize("n,seed", [(2, 41), (3, 42)])
def test_centralised_optimum_equals_decentralised_assignment(n, seed):
    """The team MDP of Def. teamMDP (n agents, n tasks) reaches, from its joint
    initial state, the value of the best assignment that Alg. 2 finds
    (Lemma lem:ct-mdp-prop)."""
    wl = tiny_workload(seed, n, n, width=3, height=2, kinds=("reach",), k=1, p_slip=0.25)
    prods = product.build_all(wl)
    team = centralised.build_team_mdp(wl)
    rng = np.random.default_rng(seed)
    for _ in range(2):
        w = rng.dirichlet(np.ones(2 * n))
        s = alg.support(prods, n, n, w, 1e-13)
        assert centralised.team_value(team, w) == pytest.approx(w @ s.r, abs=1e-8)


def test_team_optimum_at_a_zero_task_weight_corner_is_improper():
    """Where every task's weight and agent 1's cost weight are 0 (w = e_0),
    the team MDP lets agent 1 take the first task and never finish it: its
    optimum, 0, lies above the best assignment's (agent 0 must serve a task
    there) and no proper policy attains it.  The equality of Lemma
    lem:ct-mdp-prop is read for weights whose team optimum is proper."""
    from oracle.product import Product
    wl = tiny_workload(41, 2, 2, width=3, height=2, kinds=("reach",), k=1, p_slip=0.25)
    prods = product.build_all(wl)
    team = centralised.build_team_mdp(wl)
    w = np.eye(4)[0]
    assert centralised.team_value(team, w) == 0.0
    assert w @ alg.support(prods, 2, 2, w, 1e-13).r < -1e-3
    g = centralised.single_objective_model(team, w)
    S, R = len(g["state_row"]) - 1, len(g["row_ptr"]) - 1
    p = Product(n_states=S, states=np.zeros((S, 2), np.int64), state_row=g["state_row"].astype(np.int64),
                row_action=np.zeros(R, np.int64), row_ptr=g["row_ptr"].astype(np.int64),
                col=g["col"].astype(np.int64), prob=g["prob"], to_done=g["to_done"].astype(bool),
                rew_cost=g["rew"][:, 0].copy(), rew_prob=np.zeros(R), init=g["init"])
    x = vi.value_iteration(p, 1.0, 0.0, 1e-12)[0][:, 0]
    with pytest.raises(vi.ImproperPolicy):
        vi.extract_policy(p, x, 1.0, 0.0)
    # the optimum over proper policies is the assignment's
    assert centralised.team_value_proper(team, w) == pytest.approx(w @ alg.support(prods, 2, 2, w, 1e-13).r,
                                                                   abs=1e-8)


@pytest.mark.parametrize("n,seed", [(2, 41), (3, 42)])
def test_proper_team_optimum_equals_the_assignment_optimum(n, seed):
    """The proper optimum (least solution of the Bellman inequalities, a
    linear programme) equals the value iteration optimum at interior weights
    and the best assignment's everywhere, corners included (Lemma
    lem:ct-mdp-prop)."""
    wl = tiny_workload(seed, n, n, width=3, height=2, kinds=("reach",), k=1, p_slip=0.25)
    prods = product.build_all(wl)
    team = centralised.build_team_mdp(wl)
    rng = np.random.default_rng(seed + 3)
    d = 2 * n
    for w in [rng.dirichlet(np.ones(d)) for _ in range(2)] + [np.eye(d)[0], np.eye(d)[n], np.eye(d)[d - 1]]:
        best = w @ alg.support(prods, n, n, w, 1e-13).r
        assert centralised.team_value_proper(team, w) == pytest.approx(best, abs=1e-7)
        if w.min() > 0:
            assert centralised.team_value(team, w) == pytest.approx(best, abs=1e-8)


# --------------------------------------------------------------------------
# textbook reductions
# --------------------------------------------------------------------------

def test_assignment_equals_brute_force():
    rng = np.random.default_rng(5)
    for nI, nJ in [(3, 3), (4, 4), (2, 4), (3, 5), (5, 3)]:
        for _ in range(5):
            c = rng.normal(size=(nI, nJ))
            f = alg.assign(c)
            cap = max(1, -(-nJ // nI))
            best = -np.inf
            for g in itertools.product(range(nI), repeat=nJ):
                if max(np.bincount(g, minlength=nI)) <= cap:
                    best = max(best, sum(c[g[j], j] for j in range(nJ)))
            assert sum(c[f[j], j] for j in range(nJ)) == pytest.approx(best, abs=1e-12)
            assert max(np.bincount(f, minlength=nI)) <= cap


def test_deterministic_grid_cost_is_dijkstra():
    rng = np.random.default_rng(7)
    free = make_grid(rng, 7, 5, 0.2)
    cells = np.flatnonzero(free.ravel())
    agent = make_agent(rng, free, int(cells[0]), 0.0, rng.uniform(1, 3, 5))
    task = _task("reach", 2)
    letters = np.zeros(agent.n_states, np.int32)
    letters[[3, 4]] = 1
    letters[[len(cells) - 1, len(cells) - 2]] = 2
    prod = product.build_product(agent, task, letters)
    y, _ = vi.value_iteration(prod, 1.0, 0.0, 1e-12)
    S = prod.n_states
    src, dst, wt = [], [], []
    rs = prod.row_state()
    for r in range(prod.n_rows):
        a, b = prod.row_ptr[r], prod.row_ptr[r + 1]
        tgt = prod.col[a] if b > a else S
        src.append(rs[r])
        dst.append(tgt)
        wt.append(-prod.rew_cost[r])
    G = sp.csr_matrix((wt, (src, dst)), shape=(S + 1, S + 1))
    # csr_matrix sums duplicate edges; keep the cheapest parallel edge instead
    best = {}
    for u, v, c in zip(src, dst, wt):
        if u != v:
            best[(u, v)] = min(best.get((u, v), np.inf), c)
    G = sp.csr_matrix((list(best.values()), ([k[0] for k in best], [k[1] for k in best])),
                      shape=(S + 1, S + 1))
    dist = dijkstra(G, indices=prod.init)[S]
    assert y[prod.init, 0] == pytest.approx(-dist, abs=1e-9)


@pytest.mark.parametrize("cfg", [1])
def test_policy_evaluation_matches_exact_solve(cfg):
    wl = make_workload(cfg)
    prods = product.build_all(wl)
    rng = np.random.default_rng(3)
    for p in prods:
        wv = rng.dirichlet([1, 1])
        y, _ = vi.value_iteration(p, wv[0], wv[1], 1e-12)
        mu = vi.extract_policy(p, y[:, 0], wv[0], wv[1])
        (vc, vp), _, x = vi.evaluate(p, mu, 1e-12)
        ex = vi.evaluate_exact(p, mu)
        assert np.abs(x - ex).max() < 1e-8
        assert 0.0 <= vp <= 1.0 + 1e-12


# --------------------------------------------------------------------------
# invariants
# --------------------------------------------------------------------------

def test_probability_values_and_monotonicity():
    wl = make_workload(2, n_agents=2, n_tasks=3)
    for p in product.build_all(wl):
        P = p.P()
        xp = np.zeros(p.n_states)
        xc = np.zeros(p.n_states)
        for _ in range(40):
            yp = np.maximum.reduceat(p.rew_prob + P @ xp, p.state_row[:-1])
            yc = np.maximum.reduceat(p.rew_cost + P @ xc, p.state_row[:-1])
            assert (yp >= xp - 1e-15).all() and (yp <= 1 + 1e-12).all()
            assert (yc <= xc + 1e-12).all()
            xp, xc = yp, yc
        # one-step mass plus kept mass never exceeds 1
        rowsum = np.add.reduceat(p.prob, p.row_ptr[:-1]) if p.nnz else np.zeros(0)
        rowsum = np.where(np.diff(p.row_ptr) > 0, rowsum, 0.0)
        assert (rowsum + p.rew_prob <= 1 + 1e-12).all()


@pytest.mark.parametrize("seed", [51, 52, 53])
def test_alg1_invariants(seed):
    wl = tiny_workload(seed, 2, 2, width=3, height=3, kinds=("avoid", "reach"), k=1, p_slip=0.2)
    prods = product.build_all(wl)
    rng = np.random.default_rng(seed)
    base = alg.support(prods, 2, 2, np.full(4, 0.25), 1e-12).r
    t = base + np.array([1.0, 1.0, 0.2, 0.2]) * rng.uniform(-0.5, 1.0, 4)
    t[2:] = np.clip(t[2:], 0, 1)
    res = alg.query(prods, 2, 2, t, 1e-7, 1e-12, max_iter=100)
    prev_up, prev_down = np.inf, -np.inf
    Ws, Rs = [], []
    for w, r, t_up, t_down in res.trace:
        assert (w >= 0).all() and w.sum() == pytest.approx(1.0, abs=1e-12)      # lem:weight-vector
        for w2, r2 in zip(Ws, Rs):
            assert w2 @ r2 >= w2 @ r - 1e-7                                      # supporting hyperplanes
        Ws.append(w)
        Rs.append(r)
        d_up, d_down = geometry.mnorm(t - t_up), geometry.mnorm(t - t_down)
        assert d_down <= d_up + 1e-9                                             # thm:synthesis (iii)
        assert d_up <= prev_up + 1e-9 and d_down >= prev_down - 1e-9             # Phi, Lambda only grow
        prev_up, prev_down = d_up, d_down
        x, lam = geometry.project_inner(np.array(Rs), t)
        assert geometry.kkt_inner(np.array(Rs), t, x, lam) < 1e-8                # t_up in down(Phi)
    if res.verdict == alg.FEASIBLE:
        assert np.allclose(res.t_down, t)                                        # thm:synthesis (ii)


# --------------------------------------------------------------------------
# the projections themselves
# --------------------------------------------------------------------------

def test_inner_projection_single_point_and_diagonal_norm():
    r = np.array([[1.0, -2.0, 0.5]])
    t = np.array([2.0, -3.0, 0.7])
    x, lam = geometry.project_inner(r, t)
    assert np.allclose(x, np.minimum(t, r[0])) and np.allclose(lam, [1.0])
    M = np.diag([1.0, 4.0, 9.0])
    x2, _ = geometry.project_inner(r, t, M)
    assert np.allclose(x2, np.minimum(t, r[0]))


def test_outer_projection_single_halfspace_closed_form():
    rng = np.random.default_rng(9)
    for _ in range(10):
        d = 5
        w = rng.dirichlet(np.ones(d))
        rr = rng.normal(size=d)
        t = rr + rng.uniform(0.1, 1.0, d)
        A = rng.normal(size=(d, d))
        M = A @ A.T + d * np.eye(d)
        z = geometry.project_outer(w[None], rr[None], t, M)
        Mi_w = np.linalg.solve(M, w)
        star = t - (w @ t - w @ rr) / (w @ Mi_w) * Mi_w
        assert np.allclose(z, star, atol=1e-10)
        assert geometry.kkt_outer(w[None], rr[None], t, z, M) < 1e-10


def test_inner_projection_general_norm_against_slsqp():
    rng = np.random.default_rng(10)
    for _ in range(5):
        m, d = 4, 3
        Phi = rng.normal(size=(m, d))
        t = Phi.max(axis=0) + rng.uniform(0.1, 1.0, d)
        A = rng.normal(size=(d, d))
        M = A @ A.T + np.eye(d)
        x, lam = geometry.project_inner(Phi, t, M)
        assert geometry.kkt_inner(Phi, t, x, lam, M) < 1e-9
        # independent: minimise over (lam, slack) with SLSQP
        fun = lambda z: float((t - (Phi.T @ z[:m] - z[m:])) @ M @ (t - (Phi.T @ z[:m] - z[m:])))
        cons = [{"type": "eq", "fun": lambda z: z[:m].sum() - 1}]
        best = min((minimize(fun, np.r_[np.eye(m)[k], np.zeros(d)], method="SLSQP",
                             bounds=[(0, None)] * (m + d), constraints=cons,
                             options={"ftol": 1e-15, "maxiter": 1000}) for k in range(m)),
                   key=lambda r: r.fun)
        assert geometry.mnorm(t - x, M) ** 2 == pytest.approx(best.fun, abs=1e-7)


@pytest.mark.parametrize("seed", range(4))
def test_inner_projection_fixes_points_of_the_set(seed):
    # a threshold built as a convex combination of the points, lowered in
    # some coordinates, lies in down(Phi): its projection is itself, and the
    # returned weights dominate it
    rng = np.random.default_rng(1000 + seed)
    for _ in range(25):
        m, d = int(rng.integers(1, 30)), int(rng.integers(2, 60))
        Phi = rng.normal(size=(m, d)) * rng.uniform(0.1, 50, size=d)
        lam = rng.dirichlet(np.ones(m))
        t = Phi.T @ lam - rng.uniform(0, 1, d) * (rng.random(d) < 0.5)
        x, w = geometry.project_inner(Phi, t)
        assert np.array_equal(x, t)
        assert (Phi.T @ w >= t - 1e-9 * np.abs(t).max()).all()
        # raised above the best point in every coordinate it is outside
        t2 = Phi.max(0) + rng.uniform(0.1, 1.0, d)
        x2, w2 = geometry.project_inner(Phi, t2)
        assert geometry.kkt_inner(Phi, t2, x2, w2) <= 1e-8 * np.abs(t2).max()
        assert np.linalg.norm(t2 - x2) > 0


def test_nnls_against_textbook_cases():
    # exact solutions of small non-negative least-squares problems
    A = np.array([[1.0, 0.0], [0.0, 1.0], [1.0, 1.0]])
    x, r = geometry.nnls(A, np.array([1.0, -1.0, 0.5]))
    # unconstrained optimum has x2 < 0; with x2 = 0 the best x1 is 0.75
    assert np.allclose(x, [0.75, 0.0]) and r == pytest.approx(np.sqrt(0.0625 + 1 + 0.0625))
    x, r = geometry.nnls(np.eye(3), np.array([-1.0, 2.0, 3.0]))
    assert np.allclose(x, [0, 2, 3]) and r == pytest.approx(1.0)


def test_policy_from_tiny_weights_is_the_scaled_one():
    """With both weights of a model tiny, the unscaled value iteration meets
    the absolute stop test after one sweep and its greedy policy need not
    finish in reasonable time; the policy of Alg. 2 comes from the weights
    scaled to sum 1, i.e. here the cheapest way to finish (Dijkstra on a
    deterministic grid)."""
    from oracle import alg
    rng = np.random.default_rng(7)
    free = make_grid(rng, 7, 5, 0.2)
    cells = np.flatnonzero(free.ravel())
    agent = make_agent(rng, free, int(cells[0]), 0.0, rng.uniform(1, 3, 5))
    task = _task("reach", 2)
    letters = np.zeros(agent.n_states, np.int32)
    letters[[3, 4]] = 1
    letters[[len(cells) - 1, len(cells) - 2]] = 2
    prod = product.build_product(agent, task, letters)
    x, n = vi.value_iteration(prod, np.array([1e-9]), np.array([0.0]), 1e-6)
    assert n[0] == 1                                    # the unscaled stop test is met at once
    mu_tiny = alg.policy_for(prod, 1e-9, 0.0, 1e-6)
    mu_one = alg.policy_for(prod, 1.0, 0.0, 1e-6)
    assert mu_tiny.tolist() == mu_one.tolist()
    y, _ = vi.value_iteration(prod, 1.0, 0.0, 1e-12)
    cost = vi.evaluate_exact(prod, mu_tiny)[prod.init, 0]
    assert cost == pytest.approx(y[prod.init, 0], abs=1e-9)


# --------------------------------------------------------------------------
# synthesis after Alg. 1 (Sec. 3.3, end)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("cfg", ["cfg1", "rep"])
def test_synthesis_meets_feasible_thresholds(cfg):
    """On feasible thresholds the random assignment and its schedulers meet t
    in expectation (Def. MORAP), with every scheduler's values taken from an
    exact linear solve, not from the loop; the assignment matrix is doubly
    stochastic for |I| = |J| and has unit columns and rows of at most
    ceil(|J|/|I|) tasks with agent re-use."""
    if cfg == "cfg1":
        wl = make_workload(1)
    else:
        wl = tiny_workload(5, 2, 3, width=3, height=3, kinds=("reach", "avoid"), k=1, p_slip=0.2)
    prods = product.build_all(wl)
    nI, nJ = wl.n_agents, wl.n_tasks
    d = nI + nJ
    rng = np.random.default_rng(4)
    # thresholds below convex combinations of supporting points: feasible
    pts = [alg.support(prods, nI, nJ, rng.dirichlet(np.ones(d)), 1e-10).r for _ in range(4)]
    checked = 0
    for _ in range(3):
        lam = rng.dirichlet(np.ones(len(pts)))
        t = sum(l * p for l, p in zip(lam, pts)) - 0.02 * np.abs(sum(l * p for l, p in zip(lam, pts)))
        q = alg.query(prods, nI, nJ, t, 1e-9, 1e-10, max_iter=200)
        assert q.verdict == alg.FEASIBLE
        syn = alg.synthesis(prods, nI, nJ, q.W, q.lam, 1e-10)
        expect = np.zeros(d)
        for vq, f, pol in zip(syn.v, syn.F, syn.policies):
            r = np.zeros(d)
            for j in range(nJ):
                ex = vi.evaluate_exact(prods[f[j] * nJ + j], pol[j])
                init = prods[f[j] * nJ + j].init
                if init >= 0:
                    r[f[j]] += ex[init, 0]
                    r[nI + j] = ex[init, 1]
            expect += vq * r
        assert (expect >= t - 1e-7).all()
        assert np.allclose(syn.matrix.sum(axis=0), 1.0)
        cap = -(-nJ // nI)
        assert (syn.matrix.sum(axis=1) <= cap + 1e-12).all()
        if nI == nJ:
            assert np.allclose(syn.matrix.sum(axis=1), 1.0)
        checked += 1
    assert checked == 3


# --------------------------------------------------------------------------
# one agent, one task: the MOMDP special case (Sec. 5, verification
# experiment)
# --------------------------------------------------------------------------
def _projection_by_support(obj, Aeq, beq, t):
    """Euclidean projection of t (outside the set) onto the down-closure of
    the product's achievable (cost, probability) pairs, d = 2.  The distance
    is the maximum over unit weights w >= 0 of w.t - h(w), with h the
    occupation-measure LP's optimum; along the quarter circle that function is
    unimodal (its superlevel sets are convex and closed under scaling up), so
    a bounded scalar search finds it.  Returns (distance, projection)."""
    from scipy.optimize import minimize_scalar
    bounds = [(0, None)] * Aeq.shape[1]

    def gap(th):
        w = np.array([np.cos(th), np.sin(th)])
        lp = linprog(-(w @ obj), A_eq=Aeq, b_eq=beq, bounds=bounds, method="highs")
        assert lp.status == 0
        return w @ t + lp.fun

    best = minimize_scalar(lambda th: -gap(th), bounds=(0.0, np.pi / 2), method="bounded",
                           options={"xatol": 1e-12})
    # the search never evaluates the ends: a pure-cost or pure-probability
    # normal is taken from there
    dist, th = max((gap(x), x) for x in (best.x, 0.0, np.pi / 2))
    return dist, t - dist * np.array([np.cos(th), np.sin(th)])


@pytest.mark.parametrize("seed,kind", [(61, "reach"), (62, "avoid")])
def test_single_agent_single_task_is_the_momdp(seed, kind):
    """With one agent and one task the achievable set is the product MOMDP's
    own set of (cost, probability) pairs.  Verdicts equal the feasibility of
    its occupation-measure LP; outside the set, t_up lies within the bound the
    stop rule of Alg. 1 gives, sqrt(2 dist eps), of the exact projection."""
    wl = tiny_workload(seed, 1, 1, width=3, height=3, kinds=(kind,), k=2, p_slip=0.2)
    prods = product.build_all(wl)
    Aeq, beq, obj = _mo_lp(prods, 1, 1)
    mid = alg.support(prods, 1, 1, np.array([0.5, 0.5]), 1e-13).r
    rng = np.random.default_rng(seed)
    T = [mid - np.array([0.5, 0.05]), mid + np.array([0.5, 0.05])]
    for _ in range(4):
        T.append(mid + np.array([1.0, 0.2]) * rng.uniform(-1, 1, 2))
    eps = 1e-9
    seen = set()
    for t in T:
        lp = linprog(np.zeros(Aeq.shape[1]), A_ub=-obj, b_ub=-t, A_eq=Aeq, b_eq=beq,
                     bounds=[(0, None)] * Aeq.shape[1], method="highs")
        res = alg.query(prods, 1, 1, t, eps, 1e-13, max_iter=200)
        seen.add(res.verdict)
        if lp.status == 0:
            assert res.verdict == alg.FEASIBLE or geometry.mnorm(res.t_down - t) < 1e-6
            continue
        assert res.verdict != alg.FEASIBLE
        dist, p = _projection_by_support(obj, Aeq, beq, t)
        assert dist > 0
        assert np.linalg.norm(res.t_up - p) <= np.sqrt(2 * dist * eps) + 1e-7
        # inner and outer approximations bracket the distance (up to the LP
        # solver's own tolerance, ~1e-7)
        assert geometry.mnorm(t - res.t_down) <= dist + 1e-7
        assert dist <= geometry.mnorm(t - res.t_up) + 1e-7
    assert alg.FEASIBLE in seen and len(seen) > 1


# --------------------------------------------------------------------------
# stage-ordered value iteration (the staged form of Alg. 3)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("kind,k", [("reach", 4), ("avoid", 3)])
def test_location_stages_follow_the_sequence(kind, k):
    """reach-seq(k) / avoid-seq(k) automata are chains of waypoint locations
    (the trap and acceptance are done), so location q is stage k - 1 - q, and
    no transition climbs to a higher stage."""
    wl = tiny_workload(71, 1, 1, width=4, height=4, kinds=(kind,), k=k, p_slip=0.2)
    p = product.build_all(wl)[0]
    st = vi.location_stages(p)
    q = p.states[:, 1]
    assert set(q.tolist()) == set(range(k))
    assert np.array_equal(st, k - 1 - q)
    src = np.repeat(p.row_state(), np.diff(p.row_ptr))
    assert (st[p.col] <= st[src]).all()


def test_stage_ordered_vi_on_one_location_is_plain_vi():
    """With one live location there is one stage: the staged iteration is
    Alg. 3's iteration, bit for bit and sweep for sweep."""
    wl = tiny_workload(72, 1, 1, width=4, height=4, kinds=("avoid",), k=1, p_slip=0.2)
    p = product.build_all(wl)[0]
    assert len(np.unique(p.states[:, 1])) == 1
    W = np.random.default_rng(72).dirichlet(np.ones(2), size=4)
    xs, ss = vi.stage_ordered_value_iteration(p, W[:, 0], W[:, 1], 1e-9)
    xp, sp_ = vi.value_iteration(p, W[:, 0], W[:, 1], 1e-9)
    assert np.array_equal(xs, xp) and np.array_equal(ss[0], sp_)


@pytest.mark.parametrize("seed", [73, 74])
def test_stage_ordered_vi_reaches_the_lp_optimum(seed):
    """Four stages solved lowest first reach the scalarised optimum that the
    occupation-measure LP gives at the initial state, and plain VI's values
    everywhere (a stage solved in the wrong order, or against the wrong rows,
    misses both)."""
    wl = tiny_workload(seed, 1, 1, width=3, height=3, kinds=("reach",), k=4, p_slip=0.2)
    prods = product.build_all(wl)
    p = prods[0]
    Aeq, beq, obj = _mo_lp(prods, 1, 1)
    W = np.random.default_rng(seed).dirichlet(np.ones(2), size=3)
    xs, ss = vi.stage_ordered_value_iteration(p, W[:, 0], W[:, 1], 1e-12)
    assert ss.shape[0] == 4 and (ss > 0).all()
    xp, _ = vi.value_iteration(p, W[:, 0], W[:, 1], 1e-12)
    assert np.abs(xs - xp).max() <= 1e-9 * max(1.0, np.abs(xp).max())
    for col, w in enumerate(W):
        lp = linprog(-(w @ obj), A_eq=Aeq, b_eq=beq, bounds=[(0, None)] * Aeq.shape[1], method="highs")
        assert lp.status == 0
        assert xs[p.init, col] == pytest.approx(-lp.fun, abs=1e-7)


def test_stage_ordered_vi_trades_updates_for_sweeps():
    """On a reach-seq(7) product (seven stages of equal size) the staged
    iteration updates fewer states than plain VI, but the stages run one after
    another while plain VI's converge together: more sweeps in sequence.  Both
    stop within eps of each other's fixed point."""
    wl = make_workload(2, n_agents=1, n_tasks=20)
    j = next(b for b, t in enumerate(wl.tasks) if t.kind == "reach" and t.n_locs == 8)
    p = product.build_product(wl.agents[0], wl.tasks[j], wl.letters[0][j])
    W = np.array([[0.3, 0.7], [0.05, 0.95]])
    xs, ss = vi.stage_ordered_value_iteration(p, W[:, 0], W[:, 1], 1e-6)
    xp, sp_ = vi.value_iteration(p, W[:, 0], W[:, 1], 1e-6)
    sizes = np.bincount(vi.location_stages(p))
    assert len(sizes) == 7
    updates = (sizes[:, None] * ss).sum(axis=0)
    assert (updates < p.n_states * sp_).all()
    assert (ss.sum(axis=0) > sp_).all()
    assert (ss.max(axis=0) <= sp_ + 1).all()
    assert np.abs(xs - xp).max() <= 1e-4


def test_stage_retired_vi_on_one_location_is_plain_vi():
    """With one stage the in-iteration retirement is Alg. 3's iteration, bit
    for bit and sweep for sweep, and backs up every row in every sweep."""
    wl = tiny_workload(72, 1, 1, width=4, height=4, kinds=("avoid",), k=1, p_slip=0.2)
    p = product.build_all(wl)[0]
    W = np.random.default_rng(72).dirichlet(np.ones(2), size=4)
    xr, ret, backups = vi.stage_retired_value_iteration(p, W[:, 0], W[:, 1], 1e-9)
    xp, sp_ = vi.value_iteration(p, W[:, 0], W[:, 1], 1e-9)
    assert ret.shape == (1, 4)
    assert np.array_equal(xr, xp) and np.array_equal(ret[0], sp_)
    assert backups == p.n_rows * sp_.max() * 4 - p.n_rows * (sp_.max() - sp_).sum()


@pytest.mark.parametrize("seed", [73, 74])
def test_stage_retired_vi_reaches_the_lp_optimum(seed):
    """Four stages retiring inside the iteration reach the occupation-measure
    LP's optimum at the initial state and plain VI's values everywhere; the
    stages retire lowest first."""
    wl = tiny_workload(seed, 1, 1, width=3, height=3, kinds=("reach",), k=4, p_slip=0.2)
    prods = product.build_all(wl)
    p = prods[0]
    Aeq, beq, obj = _mo_lp(prods, 1, 1)
    W = np.vstack([np.random.default_rng(seed).dirichlet(np.ones(2), size=3), [[0.0, 1.0]]])
    xr, ret, _ = vi.stage_retired_value_iteration(p, W[:, 0], W[:, 1], 1e-12)
    assert ret.shape[0] == 4 and (ret > 0).all()
    assert (np.diff(ret, axis=0) >= 0).all()
    xp, _ = vi.value_iteration(p, W[:, 0], W[:, 1], 1e-12)
    assert np.abs(xr - xp).max() <= 1e-9 * max(1.0, np.abs(xp).max())
    for col, w in enumerate(W):
        lp = linprog(-(w @ obj), A_eq=Aeq, b_eq=beq, bounds=[(0, None)] * Aeq.shape[1], method="highs")
        assert lp.status == 0
        assert xr[p.init, col] == pytest.approx(-lp.fun, abs=1e-7)


def test_stage_retired_vi_keeps_the_sweep_count_and_saves_updates():
    """On the reach-seq(7) product the lower stages retire early while the
    sweep count stays plain VI's (within a sweep or two), so fewer rows are
    backed up; the values stay within eps-scale of plain VI's."""
    wl = make_workload(2, n_agents=1, n_tasks=20)
    j = next(b for b, t in enumerate(wl.tasks) if t.kind == "reach" and t.n_locs == 8)
    p = product.build_product(wl.agents[0], wl.tasks[j], wl.letters[0][j])
    W = np.array([[0.3, 0.7], [0.05, 0.95]])
    xr, ret, backups = vi.stage_retired_value_iteration(p, W[:, 0], W[:, 1], 1e-6)
    xp, sp_ = vi.value_iteration(p, W[:, 0], W[:, 1], 1e-6)
    assert ret.shape[0] == 7
    assert (ret.max(axis=0) <= sp_ + 2).all()
    assert (ret[0] < ret[-1]).all()
    assert backups < p.n_rows * sp_.sum()
    assert np.abs(xr - xp).max() <= 1e-4


# --------------------------------------------------------------------------
# the pins have teeth: a plausible mistake planted in the oracle (on the CPU,
# through monkeypatch) makes the independent check disagree far beyond its
# tolerance
# --------------------------------------------------------------------------
def _lp_gap(prods, w):
    Aeq, beq, obj = _mo_lp(prods, 2, 2)
    lp = linprog(-(w @ obj), A_eq=Aeq, b_eq=beq, bounds=[(0, None)] * Aeq.shape[1], method="highs")
    assert lp.status == 0
    return abs(w @ alg.support(prods, 2, 2, w, 1e-13).r - (-lp.fun))


def test_mutation_dropped_probability_term_fails_the_lp_pin(monkeypatch):
    wl = tiny_workload(31, 2, 2, width=3, height=3, kinds=("avoid", "reach"), k=1, p_slip=0.2)
    prods = product.build_all(wl)
    w = np.array([0.1, 0.1, 0.4, 0.4])
    assert _lp_gap(prods, w) <= 1e-8
    real = vi.scalarised_rewards
    monkeypatch.setattr(vi, "scalarised_rewards", lambda p, wc, wp: real(p, wc, 0.0 * np.atleast_1d(wp)))
    assert _lp_gap(prods, w) > 1e-3


def test_mutation_cost_sign_fails_the_lp_pin(monkeypatch):
    wl = tiny_workload(32, 2, 2, width=3, height=3, kinds=("avoid", "reach"), k=1, p_slip=0.2)
    prods = product.build_all(wl)
    w = np.array([0.3, 0.3, 0.2, 0.2])
    assert _lp_gap(prods, w) <= 1e-8
    real = vi.scalarised_rewards
    monkeypatch.setattr(vi, "scalarised_rewards", lambda p, wc, wp: real(p, -np.atleast_1d(wc), wp))
    real_vi = vi.value_iteration      # a diverging iteration is reported after 20k sweeps, not 1M
    monkeypatch.setattr(vi, "value_iteration",
                        lambda p, wc, wp, eps, max_sweeps=20_000: real_vi(p, wc, wp, eps, min(max_sweeps, 20_000)))
    try:
        failed = _lp_gap(prods, w) > 1e-3
    except (RuntimeError, vi.ImproperPolicy):
        failed = True          # rewarding cost makes the iteration diverge
    assert failed


def test_mutation_minimising_assignment_fails_brute_force(monkeypatch):
    rng = np.random.default_rng(33)
    c = rng.normal(size=(3, 5))
    cap = 2
    best = max(sum(c[f[j], j] for j in range(5)) for f in itertools.product(range(3), repeat=5)
               if np.bincount(f, minlength=3).max() <= cap)
    f = alg.assign(c)
    assert sum(c[f[j], j] for j in range(5)) == pytest.approx(best, abs=1e-12)
    real = alg.assign
    monkeypatch.setattr(alg, "assign", lambda m: real(-m))
    f = alg.assign(c)
    assert sum(c[f[j], j] for j in range(5)) < best - 1e-3


def test_mutation_reversed_stage_order_fails_the_plain_vi_pin(monkeypatch):
    wl = tiny_workload(73, 1, 1, width=3, height=3, kinds=("reach",), k=4, p_slip=0.2)
    p = product.build_all(wl)[0]
    W = np.array([[0.4, 0.6]])
    xp, _ = vi.value_iteration(p, W[:, 0], W[:, 1], 1e-12)
    xs, _ = vi.stage_ordered_value_iteration(p, W[:, 0], W[:, 1], 1e-12)
    assert np.abs(xs - xp).max() <= 1e-9 * max(1.0, np.abs(xp).max())
    real = vi.location_stages
    monkeypatch.setattr(vi, "location_stages", lambda q: real(q).max() - real(q))
    xs, _ = vi.stage_ordered_value_iteration(p, W[:, 0], W[:, 1], 1e-12)
    assert np.abs(xs - xp).max() > 1e-3


def test_mutation_reversed_retirement_order_fails_the_plain_vi_pin(monkeypatch):
    """Retiring the stage of the initial state first (stage order reversed)
    freezes it at 0 under probability-only weights: its states see no reward
    until the lower stages' values arrive."""
    wl = tiny_workload(73, 1, 1, width=3, height=3, kinds=("reach",), k=4, p_slip=0.2)
    p = product.build_all(wl)[0]
    W = np.array([[0.0, 1.0]])
    xp, _ = vi.value_iteration(p, W[:, 0], W[:, 1], 1e-12)
    xr, _, _ = vi.stage_retired_value_iteration(p, W[:, 0], W[:, 1], 1e-12)
    assert np.abs(xr - xp).max() <= 1e-9
    real = vi.location_stages
    monkeypatch.setattr(vi, "location_stages", lambda q: real(q).max() - real(q))
    xr, _, _ = vi.stage_retired_value_iteration(p, W[:, 0], W[:, 1], 1e-12)
    assert np.abs(xr - xp).max() > 1e-3


def test_mutation_frozen_weight_update_fails_the_projection_pin(monkeypatch):
    wl = tiny_workload(62, 1, 1, width=3, height=3, kinds=("avoid",), k=2, p_slip=0.2)
    prods = product.build_all(wl)
    Aeq, beq, obj = _mo_lp(prods, 1, 1)
    r1 = alg.support(prods, 1, 1, np.array([1.0, 0.0]), 1e-13).r
    r2 = alg.support(prods, 1, 1, np.array([0.0, 1.0]), 1e-13).r
    t = 0.2 * r1 + 0.8 * r2 + np.array([0.5, 0.1])
    dist, p = _projection_by_support(obj, Aeq, beq, t)
    bound = np.sqrt(2 * dist * 1e-9) + 1e-7
    assert np.linalg.norm(alg.query(prods, 1, 1, t, 1e-9, 1e-13, max_iter=200).t_up - p) <= bound
    monkeypatch.setattr(geometry, "weight_from", lambda t, t_up, M=None: np.full(len(t), 1.0 / len(t)))
    assert np.linalg.norm(alg.query(prods, 1, 1, t, 1e-9, 1e-13, max_iter=40).t_up - p) > 1e-3


@pytest.mark.parametrize("seed,w,h,kind", [(11, 3, 2, "reach"), (12, 3, 3, "avoid"), (13, 3, 3, "avoid")])
def test_exact_policy_iteration_equals_brute_force(seed, w, h, kind):
    """The oracle's exact optimum (policy iteration) is the best deterministic
    policy's value at the initial state, and its Q-gaps name that policy's
    action wherever they are clear."""
    wl = tiny_workload(seed, 1, 1, width=w, height=h, kinds=(kind,), k=1)
    prod = product.build_all(wl)[0]
    pts, pols = _policy_points(prod)
    rng = np.random.default_rng(seed + 7)
    for _ in range(4):
        wv = rng.dirichlet([1.0, 1.0])
        v, Q, err = vi.optimal_exact(prod, wv[0], wv[1])
        vals = pts @ wv
        assert v[prod.init] == pytest.approx(vals.max(), abs=1e-11)
        assert err <= 1e-11
        best, gap = vi.q_gaps(prod, Q)
        # every optimal deterministic policy takes the unique best action
        # wherever the gap is clear (states reachable or not: all of them are
        # optimal from their own start in an optimal stationary policy)
        opt = [pols[i] for i in np.flatnonzero(vals >= vals.max() - 1e-11)]
        clear = gap > 1e-9
        assert any((mu[clear] == best[clear]).all() for mu in opt)


@pytest.mark.parametrize("seed", [73, 74])
def test_exact_policy_iteration_equals_the_lp_optimum(seed):
    wl = tiny_workload(seed, 1, 1, width=3, height=3, kinds=("reach",), k=3, p_slip=0.2)
    prods = product.build_all(wl)
    p = prods[0]
    Aeq, beq, obj = _mo_lp(prods, 1, 1)
    for w in np.random.default_rng(seed).dirichlet(np.ones(2), size=3):
        v, _, _ = vi.optimal_exact(p, w[0], w[1])
        lp = linprog(-(w @ obj), A_eq=Aeq, b_eq=beq, bounds=[(0, None)] * Aeq.shape[1], method="highs")
        assert lp.status == 0
        assert v[p.init] == pytest.approx(-lp.fun, abs=1e-7)


def test_exact_policy_iteration_pin_catches_a_minimising_improvement(monkeypatch):
    # plant a mistake on the CPU: an improvement step that keeps the worst
    # action instead of the best one misses the brute-force optimum
    wl = tiny_workload(12, 1, 1, width=3, height=3, kinds=("avoid",), k=1)
    prod = product.build_all(wl)[0]
    pts, _ = _policy_points(prod)
    real = vi.q_values
    monkeypatch.setattr(vi, "q_values", lambda p, x, wc, wp: -real(p, x, wc, wp))
    wv = np.array([0.4, 0.6])
    try:
        v, _, _ = vi.optimal_exact(prod, wv[0], wv[1])
        assert abs(v[prod.init] - (pts @ wv).max()) > 1e-3
    except (RuntimeError, vi.ImproperPolicy):
        pass   # or it fails outright: either way the planted mistake is caught


# --------------------------------------------------------------------------
# the values a policy is chosen from when the cost weight vanishes
# --------------------------------------------------------------------------
def test_policy_values_for_a_vanishing_cost_weight_give_a_fast_optimal_policy():
    """Probability-only weights on a 48 x 48 agent with an avoid task: from
    values stopped at 1e-6 the tie rule picks, among actions that all keep
    the completion probability at 1, one decided by the values' own error
    (394,543 expected steps at the worst state, beyond any evaluation); from
    the tighter values of policy_eps the policy is as sure (probability 1
    everywhere, the exact optimum) and finishes in ~10^2 expected steps."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    wl = make_workload(3)
    i, j = 46, 61
    p = product.build_product(wl.agents[i], wl.tasks[j], wl.letters[i][j])

    def steps(mu):
        rows = vi.policy_rows(p, mu)
        A = sp.identity(p.n_states, format="csc") - p.P()[rows].tocsc()
        return spla.spsolve(A, np.ones(p.n_states))

    x, _ = vi.value_iteration(p, 0.0, 1.0, 1e-6)
    slow = vi.extract_policy(p, x[:, 0], 0.0, 1.0)
    assert steps(slow).max() > 1e5
    assert alg.policy_eps(1e-6, 0.0, 1.0) == pytest.approx(1e-10)
    assert alg.policy_eps(1e-6, 0.5, 0.5) == 1e-6 and alg.policy_eps(1e-13, 0.0, 1.0) == 1e-13
    fast = alg.policy_for(p, 0.0, 0.7, 1e-6)
    assert steps(fast).max() < 1e3
    ex = vi.evaluate_exact(p, fast)
    v_opt, _, _ = vi.optimal_exact(p, 0.0, 1.0)
    assert np.abs(ex[:, 1] - v_opt).max() <= 1e-9
