"""What the trained proposer gains over the plain loop (Alg. 1 from e_1).

On a seeded instance of the 10 x 20 family (reduced to 4 agents x 8 tasks so
the test stays short), the plain method's support steps give (t, target
weight) pairs: thresholds drawn around the point r(w) of a Dirichlet weight
vector w, with target w; the proposer is trained on them and then starts
unseen queries (half of them below front points, hence achievable).  Both loops must reach the same verdicts and closest points
(the plain update and the exact value iteration still decide every answer);
the learned start must need fewer Alg. 2 passes on average.
"""
import numpy as np
import pytest

from workloads import make_workload

pytestmark = pytest.mark.gpu


def test_learned_start_needs_fewer_passes():
    from paper_2305_04397_amd import morap, proposer_data as pdata
    wl = make_workload(2, variant=1, n_agents=4, n_tasks=8)
    nI, d = wl.n_agents, wl.n_agents + wl.n_tasks
    ctx = morap.Context(0)
    try:
        ctx.build_products(wl)
        opts = morap.Options(eps_vi=1e-6, precision="f32")
        rng = np.random.default_rng(0)
        phi = pdata.features(ctx, wl, opts)
        front = pdata.front_points(ctx, wl, 256, rng, opts)
        T_test = pdata.thresholds(rng, front, 96, nI, inside_half=True)
        X, Wt = pdata.generate_from_support(ctx, wl, 4096, 2, phi, rng, opts)
        ctx.proposer_init(X.shape[1], d, seed=1)
        ctx.proposer_set_input_norm(X.mean(0), X.std(0) + 1e-3)
        losses = ctx.proposer_train(X, Wt, batch=128, epochs=60, lr=1e-3, seed=2)
        assert losses[-1] < losses[0]
        ctx.set_features(phi)
        plain = ctx.query_batch(T_test, eps=0.01, opts=opts)
        learned = ctx.query_batch(T_test, eps=0.01, opts=opts, use_proposer=True)
        assert all(q["fallback"] == 0 for q in learned)
        eps = 0.01
        for t, p, q in zip(T_test, plain, learned):
            # feasibility and infeasibility are both certificates: never in conflict
            decided = {p["verdict"], q["verdict"]} - {morap.UNDECIDED}
            assert len(decided) <= 1
            # each loop brackets the closest point t* between t_up and t_down
            # with ||t_down - t_up|| <= eps, so ||t_down - t*||^2 <= 2 R eps
            # with R = ||t - t_up|| (projections on nested convex sets)
            R = max(np.linalg.norm(t - p["t_up"]), np.linalg.norm(t - q["t_up"]))
            assert np.linalg.norm(p["t_down"] - q["t_down"]) <= 2 * np.sqrt(2 * R * eps) + 2 * eps
        n_plain = np.mean([q["iterations"] for q in plain])
        n_learned = np.mean([q["iterations"] for q in learned])
        print(f"passes per query: plain {n_plain:.2f}, learned {n_learned:.2f}")
        assert n_learned < n_plain
    finally:
        ctx.close()
