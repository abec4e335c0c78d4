"""Parity at the full 50 x 100 size (5,000 product MDPs, 1.3e7 states), in
the launch configuration bench.py times: K = 64 Dirichlet columns, FP32
batched solve with the autotuned persistent sweep replayed from hipGraphs,
then the support step (assignment, FP64 re-solve of the assigned pairs,
policies, evaluation).  The oracle cannot solve the whole workload, so it
recomputes sampled outputs one by one (models of 32 x 32 agents, where its
FP64 value iteration takes about a second), and properties that hold at any
size are checked on everything."""
import numpy as np
import pytest

from workloads import make_workload, dirichlet_weights
from oracle import product, vi, alg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def full():
    from paper_2305_04397_amd import morap
    wl = make_workload(3)
    ctx = morap.Context(0)
    ctx.build_products(wl)
    yield morap, ctx, wl
    ctx.close()


def _small_models(wl, rng, n):
    nI, nJ = wl.n_agents, wl.n_tasks
    cand = [(i, j) for i in range(nI) for j in range(nJ)
            if wl.agents[i].width == 32 and wl.tasks[j].n_locs <= 4]
    pick = rng.choice(len(cand), size=n, replace=False)
    return [cand[p] for p in pick]


def test_full_size_solve_sampled(full):
    morap, ctx, wl = full
    nI, nJ = wl.n_agents, wl.n_tasks
    rng = np.random.default_rng(0)
    W = dirichlet_weights(rng, 64, nI + nJ)
    eps = 1e-6
    c, st = ctx.solve(W, morap.Options(eps_vi=eps, precision="f32"))
    assert st["variant"] > 18                       # the neighbourhood-block sweep served the solve
    # costs are negative and a task's probability is at most 1: c[k, i, j] <= w_j
    assert np.isfinite(c).all()
    assert (c <= W[:, None, nI:] + 1e-6).all()
    for i, j in _small_models(wl, rng, 6):
        p = product.build_product(wl.agents[i], wl.tasks[j], wl.letters[i][j])
        ks = rng.choice(64, size=3, replace=False)
        y, _ = vi.value_iteration(p, W[ks, i], W[ks, nI + j], eps)
        for col, k in enumerate(ks):
            ref = y[p.init, col] if p.init >= 0 else 0.0
            # FP32 sweeps stop at max(eps, 8 u32 |y|): 2e-4 relative covers it
            assert abs(c[k, i, j] - ref) <= 2e-4 * max(1.0, abs(ref)), (i, j, k, c[k, i, j], ref)


def test_tail_kernel_switch_keeps_the_values(full):
    """An autotuned solve whose kernel is the wave-per-state gather sweep
    runs its last sweeps (under 20 % of the tiles active) with the LDS-staged
    kernel; the values, the stop sweeps, the backups, the bytes and the floor
    stops are those of the same solve with the gather sweep throughout (a
    fixed schedule never switches), bit for bit."""
    morap, ctx, wl = full
    nI, nJ = wl.n_agents, wl.n_tasks
    W = dirichlet_weights(np.random.default_rng(5), 64, nI + nJ)
    c1, st1 = ctx.solve(W, morap.Options(eps_vi=1e-6, precision="f32"))
    if st1["variant"] not in (34, 37, 38):
        pytest.skip(f"the autotuner chose variant {st1['variant']}, not a wave-per-state gather sweep")
    assert st1["variant_tail"] == 39 and 0 < st1["sweeps_tail"] < st1["sweeps"]
    big = [m for m in range(nI * nJ) if ctx.model_info(m)["n_states"] > 100_000][:2]
    v1 = {(k, m): ctx.get_values(k, m) for m in big for k in (0, 63)}
    c2, st2 = ctx.solve(W, morap.Options(eps_vi=1e-6, precision="f32", schedule=st1["variant"]))
    assert st2["sweeps_tail"] == 0 and st2["variant_tail"] == 0
    assert np.array_equal(c1, c2)
    assert st1["sweeps"] == st2["sweeps"] and st1["backups"] == st2["backups"]
    assert st1["bytes"] + st1["bytes_tail"] == pytest.approx(st2["bytes"], rel=1e-12)
    assert st1["floor_stops"] == st2["floor_stops"] and st1["max_pair_sweeps"] == st2["max_pair_sweeps"]
    for (k, m), x in v1.items():
        assert np.array_equal(x, ctx.get_values(k, m)), (k, m)


@pytest.mark.parametrize("kind", ["avoid", "reach"])
def test_full_size_largest_product_sampled(full, kind):
    """The products of maximum size class: the 128 x 128 agent with a
    12-location task (1.3-1.4e5 live states, about a thousand tiles each), the
    oracle's FP64 value iteration on two columns against the batched FP32
    solve.  The reach-seq(11) product is the one that converges last (over
    2,200 sweeps), where the FP32 stop rule's error is largest."""
    morap, ctx, wl = full
    nI, nJ = wl.n_agents, wl.n_tasks
    i = max(range(nI), key=lambda a: wl.agents[a].width)
    j = max((b for b in range(nJ) if wl.tasks[b].kind == kind), key=lambda b: wl.tasks[b].n_locs)
    assert wl.agents[i].width == 128 and wl.tasks[j].n_locs == 12
    W = dirichlet_weights(np.random.default_rng(0), 64, nI + nJ)
    eps = 1e-6
    c, st = ctx.solve(W, morap.Options(eps_vi=eps, precision="f32"))
    p = product.build_product(wl.agents[i], wl.tasks[j], wl.letters[i][j])
    assert p.n_states > 100_000
    ks = [0, 63]
    y, _ = vi.value_iteration(p, W[ks, i], W[ks, nI + j], eps)
    for col, k in enumerate(ks):
        ref = y[p.init, col]
        # the FP32 stop rule max(eps, 8 u32 |y|) leaves an error of that
        # residual times 1/(1 - rho): rho ~ 0.96 (avoid) and ~0.992 (reach)
        # give ~1e-5 and ~6e-5 relative
        assert abs(c[k, i, j] - ref) <= 2e-4 * max(1.0, abs(ref)), (k, c[k, i, j], ref)


def test_full_size_support_sampled(full):
    """The support step at full size.  On every column: Lemma lem:face (w.r
    equals the assignment's sum of scalarised values, within the FP32 errors
    of those values, each below the per-pair bound 2e-4 max(1, |c|) that the
    sampled solve tests check against the oracle), the capacity of the
    replicated agents and probabilities in [0, 1].  On sampled 32 x 32 agents
    of sampled columns: the agent's cost objective r[i] (the sum over both of
    its tasks) and the probabilities of those tasks against the oracle's Alg. 4
    evaluation of the device's policies, and the policies against the exact
    optimum off ties (tau_cmp of parity_g12, excluded states counted)."""
    morap, ctx, wl = full
    nI, nJ = wl.n_agents, wl.n_tasks
    rng = np.random.default_rng(1)
    W = dirichlet_weights(rng, 4, nI + nJ)
    eps = 1e-6
    r, A, c, st = ctx.support(W, morap.Options(eps_vi=eps, precision="f32"))
    worst = 0.0
    for k in range(W.shape[0]):
        terms = np.array([c[k][A[k][j], j] for j in range(nJ)])
        bound = (2e-4 * np.maximum(1.0, np.abs(terms))).sum()
        dev = abs(W[k] @ r[k] - terms.sum())
        assert dev <= bound, (k, dev, bound)
        worst = max(worst, dev / max(1.0, abs(terms.sum())))
        loads = np.bincount(A[k], minlength=nI)
        assert loads.max() <= 2 and (r[k][nI:] >= -1e-12).all() and (r[k][nI:] <= 1 + 1e-9).all()
    excluded = states = agents = 0
    tau_max = 0.0
    for k in range(W.shape[0]):
        small = [i for i in range(nI) if wl.agents[i].width == 32 and
                 all(wl.tasks[j].n_locs <= 4 for j in np.flatnonzero(A[k] == i))]
        for i in rng.choice(small, size=2, replace=False):
            ri = 0.0
            for j in np.flatnonzero(A[k] == i):
                p = product.build_product(wl.agents[i], wl.tasks[j], wl.letters[i][j])
                mu = ctx.get_policy(k, int(j), p.n_states).astype(np.int64)
                sc = W[k, i] + W[k, nI + j]
                a, b = W[k, i] / sc, W[k, nI + j] / sc
                v, Q, err = vi.optimal_exact(p, a, b)
                y, _ = vi.value_iteration(p, a, b, eps)
                tau = max(1e-9, 2 * err, 4 * float(np.abs(y[:, 0] - v).max()))
                best, gap = vi.q_gaps(p, Q)
                clear = gap > tau
                assert not (clear & (mu != best)).any(), (k, i, j)
                excluded += int((~clear & (gap > 1e-9)).sum())
                states += p.n_states
                tau_max = max(tau_max, tau)
                (vc, vp), _, _ = vi.evaluate(p, mu, eps)
                assert r[k][nI + j] == pytest.approx(vp, rel=1e-9, abs=4 * eps)
                ri += vc
            # the agent's cost objective sums its (up to two) tasks' costs
            assert r[k][i] == pytest.approx(ri, rel=1e-9, abs=8 * eps), (k, i)
            agents += 1
    print(f"\nparity f32 50x100: w.r vs sum c max rel {worst:.2e}; {agents} agents; "
          f"{excluded} of {states} states with a Q-gap in (1e-9, tau_cmp] (max {tau_max:.1e}) excluded")
    assert agents == 8 and excluded <= 0.02 * states


def test_full_size_query_geometry_replay(full):
    """Alg. 1 at full size (d = 150, lockstep queries inside and outside the
    achievable set): the oracle's projections, run on the device's own trace
    of weight vectors and points, reproduce every pass's next weight vector,
    the final t_up and t_down and the verdict.  The points themselves are
    the support step's, whose sampled parity is checked above."""
    from oracle import geometry
    morap, ctx, wl = full
    nI, nJ = wl.n_agents, wl.n_tasks
    d = nI + nJ
    rng = np.random.default_rng(2)
    opts = morap.Options(eps_vi=1e-6, precision="f32")
    front, _, _, _ = ctx.support(dirichlet_weights(rng, 4, d), opts)
    T = []
    for k in range(8):
        # above the front in every objective (separated, outer projections)
        # or below it (inside, inner projections only)
        u = front[k % 4]
        t = u + rng.uniform(0.0, 0.3, d) * np.abs(u) * (1 if k % 2 else -1)
        t[nI:] = np.clip(t[nI:], 0.0, 1.0)
        T.append(t)
    res = ctx.query_batch(np.array(T), eps=0.01, max_iter=6, opts=opts, trace=True)
    separated = 0
    for t, q in zip(T, res):
        n = q["iterations"]
        W, R = q["W"], q["R"]
        scale = max(1.0, np.abs(t).max())
        t_down = t.copy()
        for i in range(n):
            if W[i] @ R[i] < W[i] @ t_down:
                t_down = geometry.project_outer(W[:i + 1], R[:i + 1], t)
            t_up, _ = geometry.project_inner(R[:i + 1], t)
            if i + 1 < n:
                w = geometry.weight_from(t, t_up)
                assert w is not None
                assert np.abs(w - W[i + 1]).max() <= 1e-6, (i, np.abs(w - W[i + 1]).max())
        assert np.abs(t_up - q["t_up"]).max() <= 1e-6 * scale
        assert np.abs(t_down - q["t_down"]).max() <= 1e-6 * scale
        assert q["verdict"] == alg.verdict_of(t, t_up, W, R)
        separated += int(np.any(np.einsum("ij,ij->i", W, R) < W @ t))
    assert separated >= 2
