"""The LDS-staged sweep over halo tiles (variants 39 and 40) against the
wave-per-state block sweep (variant 37) and the FP64 oracle.

Both kernels add the same terms in the same order (cost reward, probability
reward, then the successor slots in slot order), so their FP32 values are
bit-identical; the oracle bounds them by the FP32 stopping rule."""
import numpy as np
import pytest

from workloads import make_workload, tiny_workload, dirichlet_weights
from oracle import product, vi

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


def _solve(ctx, morap, W, v, eps=1e-6):
    c, st = ctx.solve(W, morap.Options(eps_vi=eps, precision="f32", schedule=v))
    assert st["variant"] == v
    return c, st


def _same_values(ctx, a, b, models, K):
    for m in models:
        for k in sorted({0, K // 2, K - 1}):
            assert np.array_equal(a[(k, m)], b[(k, m)]), (k, m)


@pytest.mark.parametrize("K", [64, 100, 128])
def test_halo_sweep_equals_block_sweep_cfg2(ctx, morap, K):
    wl = make_workload(2)
    ctx.build_products(wl)
    nI, nJ = wl.n_agents, wl.n_tasks
    W = dirichlet_weights(np.random.default_rng(K), K, nI + nJ)
    W[0] = np.eye(nI + nJ)[0]     # models of agents != 0 are all zero: they stop after one sweep
    models = [0, 7, 55, 120, 199]
    ref, vals = None, {}
    for v in (37, 39, 40):
        c, st = _solve(ctx, morap, W, v)
        vals[v] = {(k, m): ctx.get_values(k, m) for m in models for k in {0, K // 2, K - 1}}
        if ref is None:
            ref, ref_st = c, st
        assert np.array_equal(c, ref), v
        assert st["sweeps"] == ref_st["sweeps"] and st["backups"] == ref_st["backups"], v
    _same_values(ctx, vals[37], vals[39], models, K)
    _same_values(ctx, vals[37], vals[40], models, K)
    # against the oracle, within the FP32 stopping rule's reach
    prods = product.build_all(wl)
    for m in models:
        i, j = divmod(m, nJ)
        p = prods[m]
        if p.init < 0:
            continue
        y, _ = vi.value_iteration(p, W[:, i], W[:, nI + j], 1e-9)
        assert (np.abs(ref[:, i, j] - y[p.init]) <= 2e-4 * np.maximum(1.0, np.abs(y[p.init]))).all()


def test_halo_sweep_self_loop_changing_location(ctx, morap):
    """A state whose own successor is another product state (a counting
    automaton that advances while the agent stays on a waypoint)."""
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
    ctx.build_products(wl)
    W = dirichlet_weights(np.random.default_rng(1), 64, 3)
    c37, _ = _solve(ctx, morap, W, 37, eps=1e-7)
    c39, _ = _solve(ctx, morap, W, 39, eps=1e-7)
    assert np.array_equal(c37, c39)
    prods = product.build_all(wl)
    for m, p in enumerate(prods):
        y, _ = vi.value_iteration(p, W[:, m], W[:, 2], 1e-10)
        assert (np.abs(c39[:, m, 0] - y[p.init]) <= 2e-4 * np.maximum(1.0, np.abs(y[p.init]))).all()


def test_halo_sweep_on_many_small_products(ctx, morap):
    """Products of a few states each (tiles of one to a few states, most
    waves of a workgroup without a state)."""
    wl = tiny_workload(9, 3, 4, width=3, height=2, kinds=("avoid", "reach"))
    ctx.build_products(wl)
    W = dirichlet_weights(np.random.default_rng(2), 64, 7)
    c37, _ = _solve(ctx, morap, W, 37, eps=1e-7)
    c40, _ = _solve(ctx, morap, W, 40, eps=1e-7)
    assert np.array_equal(c37, c40)


def test_halo_variant_refuses_fp64(ctx, morap):
    wl = make_workload(1)
    ctx.build_products(wl)
    W = dirichlet_weights(np.random.default_rng(0), 64, 4)
    with pytest.raises(morap.MorapError):
        ctx.solve(W, morap.Options(eps_vi=1e-8, precision="f64", schedule=39))
