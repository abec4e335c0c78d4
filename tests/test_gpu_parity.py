"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars:
  * product construction, assignment and policies: bit-exact (integer work);
  * FP64 value iteration mirrors the oracle's arithmetic up to summation
    order, so values agree to rounding when both stop at the same sweep; the
    bound used is 4 eps + 1e-10 |v| (a stop one sweep apart moves a value by at
    most one residual, <= eps);
  * per-objective evaluation (Alg. 4) is FP64 in both: 1e-9 |v| + 4 eps_eval;
  * FP32 sweeps: the reported scalarised values carry the FP32 stopping error
    (the test states and checks the bound of each result).
"""
import numpy as np
import pytest

from workloads import make_workload, worked_example, tiny_workload, dirichlet_weights
from oracle import product, vi, alg, centralised
from parity_g12 import check_support

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def morap():
    from paper_2305_04397_amd import morap as m
    return m


@pytest.fixture(scope="module")
def ctx(morap):
    c = morap.Context(0)
    yield c
    c.close()


def _load(ctx, wl):
    ctx.build_products(wl)
    return product.build_all(wl)


def _same_product(g, o):
    assert g["state_row"].tolist() == o.state_row.tolist()
    assert g["row_ptr"].tolist() == o.row_ptr.tolist()
    assert g["col"].tolist() == o.col.tolist()
    assert np.array_equal(g["prob"], o.prob)
    assert np.array_equal(g["rew"][:, 0], o.rew_cost) and np.array_equal(g["rew"][:, 1], o.rew_prob)
    assert g["to_done"].astype(bool).tolist() == o.to_done.tolist()
    assert g["init"] == o.init
    assert g["states"].tolist() == o.states.tolist()


@pytest.mark.parametrize("name", ["example", "cfg1", "cfg2_sub", "tiny"])
def test_products_bit_exact(ctx, name):
    wl = {"example": worked_example, "cfg1": lambda: make_workload(1),
          "cfg2_sub": lambda: make_workload(2, n_agents=3, n_tasks=5),
          "tiny": lambda: tiny_workload(5, 2, 3, width=3, height=3, kinds=("avoid", "reach"))}[name]()
    prods = _load(ctx, wl)
    for m, p in enumerate(prods):
        _same_product(ctx.get_model(m), p)


def _oracle_c(prods, nI, nJ, W, eps):
    K = W.shape[0]
    c = np.zeros((K, nI, nJ))
    sw = np.zeros((K, nI, nJ), dtype=np.int64)
    vals = {}
    for i in range(nI):
        for j in range(nJ):
            p = prods[i * nJ + j]
            y, n = vi.value_iteration(p, W[:, i], W[:, nI + j], eps)
            vals[i * nJ + j] = y
            if p.init >= 0:
                c[:, i, j] = y[p.init]
            sw[:, i, j] = n
    return c, sw, vals


def _oracle_policy(p, wi, wj, eps):
    """The oracle's policy of one model: value iteration on the two weights
    scaled to sum 1, then the tie rule."""
    sc = wi + wj
    if sc > 0:
        wi, wj = wi / sc, wj / sc
    x, _ = vi.value_iteration(p, np.array([wi]), np.array([wj]), eps)
    return vi.extract_policy(p, x[:, 0], wi, wj)


@pytest.mark.parametrize("K", [1, 3, 16, 70])
def test_solve_f64_matches_oracle(ctx, morap, K):
    wl = make_workload(1)
    prods = _load(ctx, wl)
    nI, nJ = wl.n_agents, wl.n_tasks
    W = dirichlet_weights(np.random.default_rng(K), K, nI + nJ)
    W[0] = np.eye(nI + nJ)[0]          # the initial weight of Alg. 1
    eps = 1e-8
    c, st = ctx.solve(W, morap.Options(eps_vi=eps, precision="f64"))
    co, sw, vals = _oracle_c(prods, nI, nJ, W, eps)
    assert np.abs(c - co).max() <= 4 * eps + 1e-10 * np.abs(co).max()
    assert st["max_pair_sweeps"] in (sw.max(), sw.max() + 1, sw.max() - 1)
    for m in range(len(prods)):
        for k in (0, K - 1):
            x = ctx.get_values(k, m)
            assert np.abs(x - vals[m][:, k]).max() <= 4 * eps + 1e-10 * np.abs(vals[m]).max()


SHAPES = [(1, 1), (1, 2), (2, 1), (1, 4), (2, 2), (4, 1), (1, 8), (2, 4), (4, 2), (1, 16), (2, 8),
          (4, 4), (1, 32), (2, 16), (4, 8), (1, 64), (2, 32), (4, 16)]


def test_every_variant_gives_identical_f64_values(ctx, morap):
    """Variants 1-18 (CSR tiles) share one summation order, so their values are
    bit-identical, eager or graph-replayed; so are variants 19-38 (neighbourhood
    blocks) among themselves.  The two families add the same products in a
    different order: they agree to rounding."""
    wl = make_workload(2, n_agents=2, n_tasks=3)
    _load(ctx, wl)
    W = dirichlet_weights(np.random.default_rng(0), 16, 5)
    ref = {}
    for v in range(1, 39):
        cpl, lps = SHAPES[(v - 1) % 18] if v <= 36 else (1, 64)
        if 16 % (cpl * lps):
            continue
        fam = v > 18
        for graph in (False, True):
            c, st = ctx.solve(W, morap.Options(eps_vi=1e-7, precision="f64", schedule=v, use_graph=graph))
            assert st["variant"] == v
            if fam not in ref:
                ref[fam] = c
            assert np.array_equal(c, ref[fam]), (v, graph)
    assert np.abs(ref[True] - ref[False]).max() <= 1e-12 * np.abs(ref[False]).max()


def test_graph_is_not_replayed_after_a_new_upload(ctx, morap):
    """A captured chunk of sweeps holds the model buffers, the zero row and
    the block pattern.  After a larger load has sized every buffer, model set
    A is solved with graph replay; model set B has A's tile count (one tile
    per product) but more states, so its zero row moves while no buffer is
    reallocated.  B's replayed solve must equal its eager solve bit for bit."""
    W = dirichlet_weights(np.random.default_rng(3), 64, 4)
    big = make_workload(2, n_agents=2, n_tasks=2)
    a = tiny_workload(21, 2, 2, width=3, height=2)
    b = tiny_workload(22, 2, 2, width=5, height=4)
    pa, pb = product.build_all(a), product.build_all(b)
    n_tiles = lambda ps: sum((p.n_states + 127) // 128 for p in ps)
    assert n_tiles(pa) == n_tiles(pb) == 4
    assert sum(p.n_states for p in pb) > sum(p.n_states for p in pa)
    for prec in ("f64", "f32"):
        opts = dict(eps_vi=1e-7, precision=prec, schedule=37)
        ctx.build_products(big)
        ctx.solve(W, morap.Options(**opts, use_graph=True))
        ctx.build_products(a)
        ctx.solve(W, morap.Options(**opts, use_graph=True))
        ctx.build_products(b)
        cg, _ = ctx.solve(W, morap.Options(**opts, use_graph=True))
        ce, _ = ctx.solve(W, morap.Options(**opts, use_graph=False))
        assert np.array_equal(cg, ce), prec
        co, _, _ = _oracle_c(pb, 2, 2, W, 1e-7)
        assert np.abs(ce - co).max() <= (4e-7 + 1e-10 * np.abs(co).max() if prec == "f64"
                                         else 1e-4 * max(1.0, np.abs(co).max())), prec


@pytest.mark.parametrize("v", [28, 31, 34, 36])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_block_sweep_matches_oracle_cfg2(ctx, morap, v, prec):
    """The neighbourhood-block sweep against the oracle's value iteration, on
    products of uneven size (obstacles, reach and avoid automata), K = 64."""
    wl = make_workload(2, n_agents=3, n_tasks=6)
    prods = _load(ctx, wl)
    nI, nJ = wl.n_agents, wl.n_tasks
    W = dirichlet_weights(np.random.default_rng(5), 64, nI + nJ)
    eps = 1e-8 if prec == "f64" else 1e-6
    c, st = ctx.solve(W, morap.Options(eps_vi=eps, precision=prec, schedule=v))
    assert st["variant"] == v
    co, _, _ = _oracle_c(prods, nI, nJ, W, eps)
    if prec == "f64":
        assert np.abs(c - co).max() <= 4 * eps + 1e-10 * np.abs(co).max()
    else:
        assert (np.abs(c - co) <= 2e-4 * np.maximum(1.0, np.abs(co))).all()


def test_block_sweep_self_loop_changing_location(ctx, morap):
    """Staying on a waypoint cell advances a counting automaton (visit the cell
    set three times), so a state's own successor is another product state: the
    sweep must then read the state's old value separately."""
    from workloads.gridworld import Task
    wl = tiny_workload(3, 2, 1, width=4, height=3, kinds=("reach",), k=1)
    delta = np.array([[0, 1], [1, 2], [2, 3], [3, 3]], dtype=np.int32)
    wl.tasks[0] = Task(kind="count", k=3, n_locs=4, n_letters=2, q0=0, delta=delta,
                       accepting=np.array([0, 0, 0, 1], dtype=np.uint8), waypoints_uv=np.zeros((0, 2, 2)),
                       avoid_uv=None)
    for i in range(wl.n_agents):
        lab = np.zeros(wl.agents[i].n_states, dtype=np.int32)
        lab[[1, 5]] = 1
        lab[wl.agents[i].init] = 0
        wl.letters[i][0] = lab
    prods = _load(ctx, wl)
    W = dirichlet_weights(np.random.default_rng(1), 64, 3)
    eps = 1e-10
    for v in (28, 34):
        c, _ = ctx.solve(W, morap.Options(eps_vi=eps, precision="f64", schedule=v))
        co, _, _ = _oracle_c(prods, 2, 1, W, eps)
        assert np.abs(c - co).max() <= 4 * eps + 1e-10 * np.abs(co).max()


def test_support_f64_cfg1_matches_oracle(ctx, morap):
    wl = make_workload(1)
    prods = _load(ctx, wl)
    nI, nJ = wl.n_agents, wl.n_tasks
    W = np.vstack([np.eye(4), dirichlet_weights(np.random.default_rng(7), 4, 4)])
    eps = 1e-8
    r, A, c, st = ctx.support(W, morap.Options(eps_vi=eps, precision="f64"))
    for k in range(W.shape[0]):
        so = alg.support(prods, nI, nJ, W[k], eps)
        assert np.abs(c[k] - so.c).max() <= 4 * eps + 1e-10 * np.abs(so.c).max()
        # w.r equals the assignment optimum (Lemma lem:face)
        assert W[k] @ r[k] == pytest.approx(sum(c[k][A[k][j], j] for j in range(nJ)), abs=1e-6)
        assert W[k] @ r[k] == pytest.approx(W[k] @ so.r, abs=1e-6)
        if np.array_equal(A[k], so.f):
            for j in range(nJ):
                p = prods[A[k][j] * nJ + j]
                mu = ctx.get_policy(k, j, p.n_states)
                assert mu.tolist() == so.policies[j].tolist()
            assert np.abs(r[k] - so.r).max() <= 1e-9 * np.abs(so.r).max() + 4 * eps


def test_example_queries(ctx, morap):
    wl = worked_example()
    _load(ctx, wl)
    o = morap.Options(eps_vi=1e-12, precision="f64")
    qa = ctx.query([-2.5, 0.7], eps=1e-3, opts=o, trace=True)
    assert qa["verdict"] == morap.FEASIBLE and qa["iterations"] == 2
    assert np.allclose(qa["R"], [[-1.0, 0.1], [-15 / 7, 5 / 7]], atol=1e-10)
    qu = ctx.query([-1.8, 0.9], eps=1e-3, opts=o, trace=True)
    assert qu["verdict"] == morap.INFEASIBLE and qu["iterations"] == 3
    A, B, t = np.array([-15 / 7, 5 / 7]), np.array([-1.0, 0.1]), np.array([-1.8, 0.9])
    n = np.array([-(B - A)[1], (B - A)[0]])
    n = n if n @ (t - A) > 0 else -n
    assert np.allclose(qu["t_down"], t - (n @ (t - A)) / (n @ n) * n, atol=1e-7)


def test_query_cfg1_matches_oracle(ctx, morap):
    wl = make_workload(1)
    prods = _load(ctx, wl)
    o = morap.Options(eps_vi=1e-8, precision="f64")
    rng = np.random.default_rng(11)
    base = alg.support(prods, 2, 2, np.full(4, 0.25), 1e-8).r
    T = [np.array([-40.0, -40.0, 0.8, 0.8])]
    for _ in range(4):
        T.append(base + np.array([5.0, 5.0, 0.0, 0.0]) * rng.uniform(-1, 1, 4))
    for t in T:
        g = ctx.query(t, eps=1e-6, opts=o, trace=True)
        q = alg.query(prods, 2, 2, t, 1e-6, 1e-8)
        # free running: the same answer
        assert g["verdict"] == q.verdict
        assert np.abs(g["t_down"] - q.t_down).max() <= 1e-6
        assert np.abs(g["t_up"] - q.t_up).max() <= 1e-6
        # replay: each weight vector of the device's loop gives the oracle's point
        for w, r in zip(g["W"], g["R"]):
            ro = alg.support(prods, 2, 2, w, 1e-8).r
            assert np.abs(r - ro).max() <= 1e-9 * max(1.0, np.abs(ro).max())
        # while both loops see the same weights they take the same path
        same = all(np.abs(a - b).max() <= 1e-9 for a, b in zip(g["W"], q.W))
        if same:
            assert g["iterations"] == q.iterations


def test_f32_solve_and_support_cfg2(ctx, morap):
    """FP32 solve, FP64 re-solve of the assigned pairs from the FP32 values,
    policies and evaluation: every column against the oracle under the
    contract of parity_g12 (assignment within the FP32 errors of the oracle's
    optimum, actions equal to the exact optimum's off ties, r and w.r)."""
    wl = make_workload(2, n_agents=3, n_tasks=6)
    prods = _load(ctx, wl)
    nI, nJ = wl.n_agents, wl.n_tasks
    W = dirichlet_weights(np.random.default_rng(3), 16, nI + nJ)
    W[0] = np.eye(nI + nJ)[0]
    W[1] = np.eye(nI + nJ)[nI]             # probability only: many near-ties
    eps = 1e-6
    r, A, c, st = ctx.support(W, morap.Options(eps_vi=eps, precision="f32"))
    co, _, vals = _oracle_c(prods, nI, nJ, W, eps)
    # FP32 stopping error: the FP32 sweep stops once its residual is below
    # max(eps, 8 u32 |y|); the values stay within 2e-4 relative of the oracle's
    err = np.abs(c - co)
    assert (err <= 2e-4 * np.maximum(1.0, np.abs(co))).all(), err.max()
    rep = check_support(ctx, prods, nI, nJ, W, r, A, c, co, eps)
    print("\nparity f32 cfg2:", dict(rep))
    # most excluded states are exact ties (probability-only columns tie every
    # action of states that reach acceptance surely); few are excluded only
    # because the gap is below what eps-accurate values resolve
    assert rep["excluded_states"] - rep["excluded_exact_ties"] <= 0.02 * rep["states"]


def test_edge_cases(ctx, morap):
    wl = make_workload(1)
    _load(ctx, wl)
    o = morap.Options(eps_vi=1e-8, precision="f64")
    with pytest.raises(morap.MorapError) as e:
        ctx.solve(np.full((1, 4), 0.3), o)                # row does not sum to 1
    assert e.value.code == morap.E_INVALID
    with pytest.raises(morap.MorapError) as e:
        ctx.solve(np.eye(4)[:1], morap.Options(eps_vi=1e-8, precision="f64", max_sweeps=4, check_every=2))
    assert e.value.code == morap.E_NOT_CONVERGED
    with pytest.raises(morap.MorapError) as e:
        ctx.evaluate(np.zeros((2, 2), np.int32), o)       # K differs from the last solve (1)
    assert e.value.code in (morap.E_INVALID, morap.E_STATE)
    # a task whose initial location is already accepting: empty models
    wl2 = worked_example()
    wl2.tasks[0].q0 = 1
    ctx.build_products(wl2)
    assert ctx.model_info(0)["n_states"] == 0
    r, A, c, _ = ctx.support(np.array([[0.5, 0.5]]), o)
    assert np.allclose(r, 0) and np.allclose(c, 0)
    # caller-built CSR products have no neighbourhood-block form
    prods = product.build_all(make_workload(1))
    ctx.load_models([{"state_row": p.state_row, "row_ptr": p.row_ptr, "col": p.col, "prob": p.prob,
                      "rew": np.stack([p.rew_cost, p.rew_prob], 1), "to_done": p.to_done, "init": p.init}
                     for p in prods], 2, 2)
    with pytest.raises(morap.MorapError) as e:
        ctx.solve(np.eye(4)[:1], morap.Options(eps_vi=1e-8, precision="f64", schedule=19))
    assert e.value.code == morap.E_UNSUPPORTED
    c, st = ctx.solve(np.eye(4)[:1], morap.Options(eps_vi=1e-8, precision="f64"))
    assert st["variant"] <= 18


def _cfg1_thresholds(prods):
    rng = np.random.default_rng(21)
    base = alg.support(prods, 2, 2, np.full(4, 0.25), 1e-8).r
    T = [np.array([-40.0, -40.0, 0.8, 0.8]), base - np.array([3.0, 3.0, 0.0, 0.0])]
    for _ in range(3):
        T.append(base + np.array([5.0, 5.0, 0.0, 0.0]) * rng.uniform(-1, 1, 4))
    return np.array(T)


def test_query_batch_equals_single_queries(ctx, morap):
    """Lockstep queries (one weight column each per pass) give what the
    same queries give one at a time."""
    wl = make_workload(1)
    prods = _load(ctx, wl)
    o = morap.Options(eps_vi=1e-8, precision="f64")
    T = _cfg1_thresholds(prods)
    batch = ctx.query_batch(T, eps=1e-6, opts=o)
    for t, b in zip(T, batch):
        s = ctx.query(t, eps=1e-6, opts=o)
        assert b["verdict"] == s["verdict"] and b["iterations"] == s["iterations"]
        assert np.abs(b["t_down"] - s["t_down"]).max() <= 1e-9
        assert np.abs(b["t_up"] - s["t_up"]).max() <= 1e-9


def test_warm_started_passes_agree_with_cold_ones(ctx, morap):
    """Alg. 1 passes whose FP32 solves start from the previous pass's values
    (pairs with a positive cost weight) against passes solved from 0: the same
    verdicts, and final inner points within the stop rule's reach of each
    other (each lies within sqrt(2 dist eps) of the exact projection, dist =
    ||t - t_up||), on the 10 x 20 family (d = 30)."""
    wl = make_workload(2)
    ctx.build_products(wl)
    nI, d = wl.n_agents, wl.n_agents + wl.n_tasks
    rng = np.random.default_rng(12)
    opts = morap.Options(eps_vi=1e-6, precision="f32")
    front, _, _, _ = ctx.support(dirichlet_weights(rng, 8, d), opts)
    T = []
    for k in range(16):
        u = front[k % 8]
        hi = 0.0 if k % 2 else 0.3          # odd: inside (below a front point), even: mixed
        t = u + rng.uniform(-0.3, hi, d) * np.abs(u)
        t[nI:] = np.clip(t[nI:], 0.0, 1.0)
        T.append(t)
    T = np.array(T)
    eps = 0.01
    warm = ctx.query_batch(T, eps=eps, max_iter=200, opts=opts, warm_start=True)
    cold = ctx.query_batch(T, eps=eps, max_iter=200, opts=opts, warm_start=False)
    decided = 0
    for t, a, b in zip(T, warm, cold):
        assert a["verdict"] == b["verdict"]
        decided += int(a["verdict"] != morap.UNDECIDED)
        if a["gap"] <= eps and b["gap"] <= eps:
            dist = max(np.linalg.norm(t - a["t_up"]), np.linalg.norm(t - b["t_up"]))
            assert np.linalg.norm(a["t_up"] - b["t_up"]) <= 2 * np.sqrt(2 * dist * eps) + 1e-6
    # thresholds within the loop's tolerance of the front may stay undecided
    # (in both runs alike, checked above)
    assert decided >= len(T) - 4


def test_query_with_norm_matrix_matches_oracle(ctx, morap):
    """Alg. 1 with a diagonal SPD norm matrix M (the M-norm projections)."""
    wl = make_workload(1)
    prods = _load(ctx, wl)
    o = morap.Options(eps_vi=1e-8, precision="f64")
    M = np.diag([1.0, 2.0, 30.0, 40.0])
    for t in _cfg1_thresholds(prods)[:3]:
        g = ctx.query(t, M=M, eps=1e-6, opts=o, trace=True)
        q = alg.query(prods, 2, 2, t, 1e-6, 1e-8, M=M)
        assert g["verdict"] == q.verdict
        assert np.abs(g["t_down"] - q.t_down).max() <= 1e-6
        assert np.abs(g["t_up"] - q.t_up).max() <= 1e-6


def test_verification_only_stops_at_the_first_separation(ctx, morap):
    """Verification mode (Sec. 5, second experiment): stop once a hyperplane
    separates t from the achievable set."""
    wl = make_workload(1)
    prods = _load(ctx, wl)
    o = morap.Options(eps_vi=1e-8, precision="f64")
    t = _cfg1_thresholds(prods)[1] + np.array([0.0, 0.0, 0.5, 0.5])   # beyond every probability
    g = ctx.query(t, eps=1e-6, opts=o, verification_only=True, trace=True)
    q = alg.query(prods, 2, 2, t, 1e-6, 1e-8, verification_only=True)
    full = ctx.query(t, eps=1e-6, opts=o)
    assert g["verdict"] == q.verdict == morap.INFEASIBLE
    assert g["iterations"] == q.iterations <= full["iterations"]
    w, r = g["W"][-1], g["R"][-1]
    assert w @ r < w @ t


def test_single_agent_single_task_query(ctx, morap):
    """One agent and one task, a plain MOMDP with d = 2 (the setting of the
    paper's verification experiment), on a product of several tiles with a
    ragged last one: the device loop gives the oracle's verdicts and points,
    in the full and in the verification-only mode."""
    wl = make_workload(2, n_agents=1, n_tasks=1)
    prods = _load(ctx, wl)
    assert prods[0].n_states > 512 and prods[0].n_states % 128
    o = morap.Options(eps_vi=1e-8, precision="f64")
    r1 = alg.support(prods, 1, 1, np.array([1.0, 0.0]), 1e-8).r     # cost only
    r2 = alg.support(prods, 1, 1, np.array([0.0, 1.0]), 1e-8).r     # probability only
    T = [r2 + np.array([0.0, 0.05]),                                # beyond probability 1
         0.75 * r1 + 0.25 * r2 + np.array([60.0, 0.2])]             # projects to the cost corner
    for a in (0.25, 0.5):
        base = a * r1 + (1 - a) * r2
        T += [base - np.array([0.5, 0.02]), base + np.array([20.0, 0.1])]
    verdicts = set()
    for t in T:
        tol = 1e-6 * max(1.0, np.abs(t).max())
        g = ctx.query(t, eps=1e-6, opts=o, trace=True)
        q = alg.query(prods, 1, 1, t, 1e-6, 1e-8)
        verdicts.add(q.verdict)
        assert g["verdict"] == q.verdict, t
        assert np.abs(g["t_down"] - q.t_down).max() <= tol
        assert np.abs(g["t_up"] - q.t_up).max() <= tol
        for w, r in zip(g["W"], g["R"]):
            ro = alg.support(prods, 1, 1, w, 1e-8).r
            assert np.abs(r - ro).max() <= 1e-9 * max(1.0, np.abs(ro).max())
        if all(np.abs(x - y).max() <= 1e-9 for x, y in zip(g["W"], q.W)):
            assert g["iterations"] == q.iterations
        gv = ctx.query(t, eps=1e-6, opts=o, verification_only=True)
        qv = alg.query(prods, 1, 1, t, 1e-6, 1e-8, verification_only=True)
        assert gv["verdict"] == qv.verdict
        assert gv["iterations"] <= g["iterations"]
    assert verdicts == {alg.FEASIBLE, alg.INFEASIBLE}


def test_timed_solves_match_untimed(ctx, morap):
    """Sampled launch timing (``time_kernels``, which the benchmark uses)
    changes no value: a timed solve enqueues the same launches directly
    instead of replaying graphs.  Its events go back to the context's pool
    also when a solve fails part-way, and a timed solve after a failed one
    still works."""
    wl = make_workload(2, n_agents=3, n_tasks=6)
    _load(ctx, wl)
    W = dirichlet_weights(np.random.default_rng(9), 64, 9)
    c0, _ = ctx.solve(W, morap.Options(eps_vi=1e-6, precision="f32"))
    with pytest.raises(morap.MorapError) as e:
        ctx.solve(W, morap.Options(eps_vi=1e-6, precision="f32", time_kernels=True, max_sweeps=4, check_every=2))
    assert e.value.code == morap.E_NOT_CONVERGED
    c1, s1 = ctx.solve(W, morap.Options(eps_vi=1e-6, precision="f32", time_kernels=True))
    assert np.array_equal(c0, c1)
    assert s1["sweep_launches"] > 0 and s1["ms_sweep_kernel"] > 0
    r0, a0, _, _ = ctx.support(W[:4], morap.Options(eps_vi=1e-6, precision="f32"))
    r1, a1, _, s2 = ctx.support(W[:4], morap.Options(eps_vi=1e-6, precision="f32", time_kernels=True))
    assert np.array_equal(a0, a1) and np.array_equal(r0, r1)
    assert s2["sweep_launches_refine"] > 0 and s2["ms_sweep_kernel_refine"] > 0


@pytest.mark.parametrize("n,seed", [(2, 41), (3, 42)])
def test_team_mdp_on_the_device(ctx, morap, n, seed):
    """The team MDP of Def. teamMDP (the centralised model), built by the
    library's own builder scalarised for one weight vector and loaded as a
    caller-built model, solved by the device's CSR sweep: its value at the
    joint initial state is the oracle's, and the best assignment's that the
    device's own Alg. 2 finds on the decentralised products (Lemma
    lem:ct-mdp-prop; interior weights, where the optimum is proper)."""
    wl = tiny_workload(seed, n, n, width=3, height=2, kinds=("reach",), k=1, p_slip=0.25)
    team = centralised.build_team_mdp(wl)
    o = morap.Options(eps_vi=1e-12, precision="f64")
    rng = np.random.default_rng(seed)
    for _ in range(2):
        w = rng.dirichlet(np.ones(2 * n))
        ctx.build_products(wl)
        r, _, _, _ = ctx.support(w[None, :], o)
        ctx.load_models([morap.team_model_host(wl, w)], 1, 1)
        cv, st = ctx.solve(np.array([[1.0, 0.0]]), o)
        assert st["variant"] <= 18
        assert cv[0, 0, 0] == pytest.approx(centralised.team_value(team, w), abs=1e-9)
        assert cv[0, 0, 0] == pytest.approx(w @ r[0], abs=1e-8)


@pytest.mark.parametrize("cfg", ["cfg1", "rep"])
def test_synthesis_matches_oracle(ctx, morap, cfg):
    """morap_synthesize on traced queries: the picked passes reproduce the
    query's points and assignments, every returned scheduler attains its
    point under an exact linear solve of the oracle, the assignment matrix is
    the v-weighted sum of the picked assignments with unit columns, and on a
    feasible threshold the random assignment meets t in expectation."""
    if cfg == "cfg1":
        wl = make_workload(1)
    else:
        wl = tiny_workload(5, 2, 3, width=3, height=3, kinds=("reach", "avoid"), k=1, p_slip=0.2)
    prods = _load(ctx, wl)
    nI, nJ = wl.n_agents, wl.n_tasks
    d = nI + nJ
    o = morap.Options(eps_vi=1e-10, precision="f64")
    rng = np.random.default_rng(4)
    pts = [alg.support(prods, nI, nJ, rng.dirichlet(np.ones(d)), 1e-10).r for _ in range(4)]
    mix = sum(l * p for l, p in zip(rng.dirichlet(np.ones(4)), pts))
    feasible_t = mix - 0.02 * np.abs(mix)
    infeasible_t = mix + 0.05 * np.abs(mix)
    infeasible_t[nI:] = np.minimum(infeasible_t[nI:], 1.0)
    for t, feasible in ((feasible_t, True), (infeasible_t, False)):
        # cold passes: the synthesis re-solves and re-evaluates from 0, so the
        # points are reproduced to rounding (warm-started passes stop their
        # evaluations elsewhere, within eps_eval)
        g = ctx.query(t, eps=1e-6, max_iter=200, opts=o, trace=True, warm_start=False)
        syn = ctx.synthesize(g, o)
        picked = syn["picked"]
        assert len(picked) >= 1 and (g["lam"][picked] > 0).all()
        assert (g["lam"][np.setdiff1d(np.arange(g["iterations"]), picked)] == 0).all()
        assert np.array_equal(syn["F"], g["F"][picked])
        assert np.abs(syn["R"] - g["R"][picked]).max() <= 1e-12 * max(1.0, np.abs(g["R"]).max())
        mat = np.zeros((nI, nJ))
        v = syn["v"] / syn["v"].sum()
        for vq, f in zip(v, syn["F"]):
            mat[f, np.arange(nJ)] += vq
        assert np.abs(syn["matrix"] - mat).max() <= 1e-12
        assert np.allclose(syn["matrix"].sum(axis=0), 1.0)
        expect = np.zeros(d)
        for vq, f, r, sch in zip(v, syn["F"], syn["R"], syn["schedulers"]):
            rx = np.zeros(d)
            for j in range(nJ):
                p = prods[f[j] * nJ + j]
                ex = vi.evaluate_exact(p, sch[j])
                if p.init >= 0:
                    rx[f[j]] += ex[p.init, 0]
                    rx[nI + j] = ex[p.init, 1]
            assert np.abs(rx - r).max() <= 1e-6 * max(1.0, np.abs(r).max())
            expect += vq * rx
        assert (expect >= g["t_up"] - 1e-6 * np.maximum(1.0, np.abs(g["t_up"]))).all()
        if feasible:
            assert g["verdict"] == morap.FEASIBLE
            assert (expect >= t - 1e-6 * np.maximum(1.0, np.abs(t))).all()


def test_synthesis_rejects_bad_inputs(ctx, morap):
    """morap_synthesize: no pass with v > 0, a negative v and an agent index out
    of range are INVALID; a valid call after them still works."""
    wl = make_workload(1)
    _load(ctx, wl)
    o = morap.Options(eps_vi=1e-8, precision="f64")
    g = ctx.query(np.array([-40.0, -40.0, 0.8, 0.8]), eps=1e-6, max_iter=64, opts=o, trace=True)
    for bad in ({**g, "lam": np.zeros_like(g["lam"])},
                {**g, "lam": np.where(np.arange(len(g["lam"])) == 0, -1.0, g["lam"])},
                {**g, "F": np.full_like(g["F"], 7)}):
        with pytest.raises(morap.MorapError) as e:
            ctx.synthesize(bad, o)
        assert e.value.code == morap.E_INVALID
    syn = ctx.synthesize(g, o)
    assert np.allclose(syn["matrix"].sum(axis=0), 1.0)


def test_readme_example(ctx, morap):
    """The usage example of the README runs as written and returns a
    consistent answer: the threshold lies below an achievable point, so it is
    never INFEASIBLE (with eps = 0.01 the loop may stop UNDECIDED within eps of
    it), and the synthesised random assignment serves every task."""
    wl = make_workload(2)
    ctx.build_products(wl)
    opts = morap.Options(eps_vi=1e-6, precision="f32")
    r, assign, c, stats = ctx.support(np.full((1, 30), 1 / 30), opts)
    q = ctx.query(r[0] - 0.05 * np.abs(r[0]), eps=0.01, opts=opts, trace=True)
    syn = ctx.synthesize(q, opts)
    assert q["verdict"] in (morap.FEASIBLE, morap.UNDECIDED)
    t = r[0] - 0.05 * np.abs(r[0])
    assert q["verdict"] == morap.FEASIBLE or np.linalg.norm(t - q["t_up"]) <= 0.01 + 1e-9
    assert np.allclose(syn["matrix"].sum(axis=0), 1.0)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_support_on_caller_loaded_csr_products(ctx, morap, prec):
    """Products handed over as CSR (morap_load_models, no neighbourhood-block
    form): the CSR sweep, the masked batched FP64 re-solve of the assigned
    pairs and the CSR evaluation kernel.  Same bar as the block path: c within
    the FP32 stopping error (or 4 eps in FP64), identical policies and r to
    rounding wherever the assignment is the oracle's."""
    wl = make_workload(2, n_agents=3, n_tasks=6)
    prods = product.build_all(wl)
    nI, nJ = wl.n_agents, wl.n_tasks
    ctx.load_models([{"state_row": p.state_row, "row_ptr": p.row_ptr, "col": p.col, "prob": p.prob,
                      "rew": np.stack([p.rew_cost, p.rew_prob], 1), "to_done": p.to_done, "init": p.init}
                     for p in prods], nI, nJ)
    W = dirichlet_weights(np.random.default_rng(8), 8, nI + nJ)
    W[1] = np.eye(nI + nJ)[nI]
    eps = 1e-6 if prec == "f32" else 1e-8
    r, A, c, st = ctx.support(W, morap.Options(eps_vi=eps, precision=prec))
    assert st["variant"] <= 18                      # the CSR sweep served the solve
    co, _, _ = _oracle_c(prods, nI, nJ, W, eps)
    tol = 2e-4 * np.maximum(1.0, np.abs(co)) if prec == "f32" else 4 * eps + 1e-10 * np.abs(co).max()
    assert (np.abs(c - co) <= tol).all()
    rep = check_support(ctx, prods, nI, nJ, W, r, A, c, co, eps)
    print(f"\nparity {prec} caller-loaded CSR:", dict(rep))


@pytest.mark.parametrize("K", [65, 128, 130])
def test_f32_solve_more_than_64_columns(ctx, morap, K):
    """K > 64 pads to multiples of 64 and sweeps two or three column tiles per
    launch (FP32, neighbourhood blocks): every column against the oracle."""
    wl = make_workload(2, n_agents=2, n_tasks=4)
    prods = _load(ctx, wl)
    nI, nJ = wl.n_agents, wl.n_tasks
    W = dirichlet_weights(np.random.default_rng(K), K, nI + nJ)
    eps = 1e-6
    c, st = ctx.solve(W, morap.Options(eps_vi=eps, precision="f32"))
    assert st["variant"] > 18
    co, _, _ = _oracle_c(prods, nI, nJ, W, eps)
    assert (np.abs(c - co) <= 2e-4 * np.maximum(1.0, np.abs(co))).all()


def test_assignment_check_after_fp32_solves(ctx, morap):
    """After an FP32 solve the support step checks its assignment on FP64
    values: pairs whose slack lies within twice the column's FP32 error are
    re-solved in FP64 and the column reassigned if that raises its value.
    With agent 1 a copy of agent 0, every task ties between the two: the tied
    pairs are re-solved (refine_pairs > 0) and no column changes (the values
    stay equal); on every column the assignment is optimal for the FP64
    values of a full FP64 solve to rounding, and the evaluated point is the
    one morap_evaluate gives for that assignment."""
    import dataclasses
    base = make_workload(1)
    agents = [base.agents[0], base.agents[0]]
    letters = [base.letters[0], base.letters[0]]
    wl = dataclasses.replace(base, agents=agents, letters=letters)
    ctx.build_products(wl)
    nI, nJ = wl.n_agents, wl.n_tasks
    W = dirichlet_weights(np.random.default_rng(8), 16, nI + nJ)
    W[:, 1] = W[:, 0]           # the two agents' costs weigh the same: exact ties
    W /= W.sum(axis=1, keepdims=True)
    o = morap.Options(eps_vi=1e-6, eps_eval=1e-10, precision="f32")
    r, A, c, st = ctx.support(W, o)
    assert st["refine_pairs"] > 0 and st["refine_columns"] == 0
    c64, _ = ctx.solve(W, morap.Options(eps_vi=1e-12, precision="f64"))
    for k in range(len(W)):
        opt = max(sum(c64[k][f[j], j] for j in range(nJ)) for f in ([0, 1], [1, 0], [0, 0], [1, 1])
                  if max(np.bincount(f, minlength=nI)) <= 1)
        val = sum(c64[k][A[k][j], j] for j in range(nJ))
        assert val >= opt - 1e-9 * max(1.0, abs(opt)), k
    ctx.solve(W, o)
    r2, _ = ctx.evaluate(A, o)
    assert np.abs(r2 - r).max() <= 1e-9 * max(1.0, np.abs(r).max())


def test_assignment_check_keeps_parity_on_cfg2(ctx, morap):
    """The 10 x 20 family in FP32: every column's assignment is optimal for
    the values of a full FP64 solve within the FP64 solve's accuracy."""
    wl = make_workload(2)
    ctx.build_products(wl)
    nI, nJ = wl.n_agents, wl.n_tasks
    W = dirichlet_weights(np.random.default_rng(9), 32, nI + nJ)
    r, A, c, st = ctx.support(W, morap.Options(eps_vi=1e-6, precision="f32"))
    c64, _ = ctx.solve(W, morap.Options(eps_vi=1e-12, precision="f64"))
    A64 = ctx.assign(c64)
    for k in range(len(W)):
        opt = sum(c64[k][A64[k][j], j] for j in range(nJ))
        val = sum(c64[k][A[k][j], j] for j in range(nJ))
        assert val >= opt - 1e-9 * max(1.0, abs(opt)), (k, val, opt)
    assert st["refine_pairs"] >= 0 and st["refine_columns"] >= 0
