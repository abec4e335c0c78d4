"""Seeded generator: determinism and the structural guarantees the oracle
and the library rely on (stochastic rows, unlabelled start cells, disjoint
task cells, configuration sizes).  CPU only."""
import numpy as np
import pytest

from workloads import make_workload, tiny_workload, dirichlet_weights
from oracle import product


def _same(a, b):
    for x, y in zip(a.agents, b.agents):
        assert np.array_equal(x.succ, y.succ) and np.array_equal(x.prob, y.prob)
        assert np.array_equal(x.cost, y.cost) and x.init == y.init
    for la, lb in zip(a.letters, b.letters):
        for x, y in zip(la, lb):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("cfg", [1, 2])
def test_deterministic_per_seed(cfg):
    _same(make_workload(cfg), make_workload(cfg))
    other = make_workload(cfg, variant=1)
    assert any(not np.array_equal(x.cost, y.cost) for x, y in zip(make_workload(cfg).agents, other.agents))


@pytest.mark.parametrize("cfg", [1, 2])
def test_structure(cfg):
    wl = make_workload(cfg)
    for i, a in enumerate(wl.agents):
        sums = np.add.reduceat(a.prob, a.sa_ptr[:-1])
        assert np.allclose(sums, 1.0, atol=1e-15)
        assert ((a.succ >= 0) & (a.succ < a.n_states)).all()
        for j, t in enumerate(wl.tasks):
            let = wl.letters[i][j]
            assert let[a.init] == 0                       # start cell unlabelled
            assert let.max() < t.n_letters
            for l in range(1, t.k + 1):
                assert (let == l).sum() == 2              # waypoint sets of 2 cells
            if t.kind == "avoid":
                assert (let == t.k + 1).sum() == 3


def test_config_sizes():
    wl = make_workload(1)
    prods = product.build_all(wl)
    assert len(prods) == 4 and all(p.n_states <= 72 for p in prods)
    assert wl.n_agents + wl.n_tasks == 4
    wl2 = make_workload(2)
    assert (wl2.n_agents, wl2.n_tasks) == (10, 20)
    assert all(3 <= t.n_locs <= 8 for t in wl2.tasks)


def test_dirichlet_rows():
    W = dirichlet_weights(np.random.default_rng(0), 16, 30)
    assert (W >= 0).all() and np.allclose(W.sum(1), 1.0, atol=1e-15)
