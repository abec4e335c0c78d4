"""The C-ABI library loads and exports every entry point include/morap.h
declares, and its host-only projections (Alg. 1 geometry) agree with the
oracle.  CPU only: no call here touches a GPU."""
import os
import re

import numpy as np
import scipy.sparse as sp
import pytest

from oracle import geometry

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "morap.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(morap_[a-z_0-9]+)\s*\(", src)))


def test_header_symbols_exported():
    from paper_2305_04397_amd import morap
    names = _declared()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(morap.lib, n)]
    assert not missing, missing


def test_library_is_gfx950():
    # the offload bundle of the library built here names its target
    lib = os.path.join(ROOT, "paper_2305_04397_amd", "libmorap.so")
    assert b"amdgcn-amd-amdhsa--gfx950" in open(lib, "rb").read()


@pytest.mark.parametrize("seed", range(6))
def test_inner_projection_matches_oracle(seed):
    from paper_2305_04397_amd import morap
    rng = np.random.default_rng(seed)
    m, d = rng.integers(1, 12), rng.integers(2, 40)
    Phi = rng.normal(size=(m, d)) * rng.uniform(0.1, 100, size=d)
    t = Phi.mean(0) + rng.normal(size=d) * np.abs(Phi).mean(0)
    x, lam = morap.project_inner(Phi, t)
    xo, lo = geometry.project_inner(Phi, t)
    scale = max(1.0, np.abs(t).max())
    assert np.abs(x - xo).max() <= 1e-8 * scale
    assert geometry.kkt_inner(Phi, t, x, lam) <= 1e-7 * scale
    # diagonal and full norm matrices
    D = np.diag(rng.uniform(0.5, 3.0, d))
    x2, _ = morap.project_inner(Phi, t, D)
    assert np.abs(x2 - geometry.project_inner(Phi, t, D)[0]).max() <= 1e-7 * scale
    A = rng.normal(size=(d, d))
    Mf = A @ A.T / d + np.eye(d)
    x3, _ = morap.project_inner(Phi, t, Mf)
    assert np.abs(x3 - geometry.project_inner(Phi, t, Mf)[0]).max() <= 1e-6 * scale


@pytest.mark.parametrize("seed", range(6))
def test_outer_projection_matches_oracle(seed):
    from paper_2305_04397_amd import morap
    rng = np.random.default_rng(100 + seed)
    n, d = rng.integers(1, 10), rng.integers(2, 30)
    W = rng.dirichlet(np.ones(d), size=n)
    R = rng.normal(size=(n, d))
    t = R.max(0) + rng.uniform(0, 2, d)
    z = morap.project_outer(W, R, t)
    zo = geometry.project_outer(W, R, t)
    assert np.abs(z - zo).max() <= 1e-8 * max(1.0, np.abs(t).max())
    A = rng.normal(size=(d, d))
    Mf = A @ A.T / d + np.eye(d)
    z2 = morap.project_outer(W, R, t, Mf)
    assert np.abs(z2 - geometry.project_outer(W, R, t, Mf)).max() <= 1e-7 * max(1.0, np.abs(t).max())


def test_projection_rejects_bad_norm_matrix():
    from paper_2305_04397_amd import morap
    with pytest.raises(morap.MorapError) as e:
        morap.project_inner(np.ones((2, 2)), np.zeros(2), np.array([[1.0, 2.0], [2.0, 1.0]]))
    assert e.value.code == morap.E_INVALID


@pytest.mark.parametrize("mode", range(4))
def test_projections_stress_against_oracle(mode):
    from paper_2305_04397_amd import morap
    rng = np.random.default_rng(42 + mode)
    for _ in range(40):
        m, d = int(rng.integers(1, 30)), int(rng.integers(2, 60))
        Phi = rng.normal(size=(m, d)) * rng.uniform(0.1, 50, size=d)
        lam = rng.dirichlet(np.ones(m))
        t = [Phi.mean(0) + rng.normal(size=d) * np.abs(Phi).mean(0), Phi.max(0) + rng.uniform(0, 1, d),
             Phi.T @ lam, Phi.T @ lam - rng.uniform(0, 1, d) * (rng.random(d) < 0.5)][mode]
        x, w = morap.project_inner(Phi, t)
        xo, _ = geometry.project_inner(Phi, t)
        sc = max(1.0, np.abs(t).max())
        assert np.abs(x - xo).max() <= 1e-9 * sc
        assert geometry.kkt_inner(Phi, t, x, w) <= 1e-9 * sc
        W = rng.dirichlet(np.ones(d), size=m)
        R = rng.normal(size=(m, d))
        t2 = R.max(0) + rng.uniform(-1, 2, d)
        assert np.abs(morap.project_outer(W, R, t2) - geometry.project_outer(W, R, t2)).max() <= 1e-9 * max(
            1.0, np.abs(t2).max())


# --------------------------------------------------------------------------
# Alg. 2's assignment step on the host (the library's Hungarian method)
# --------------------------------------------------------------------------
def _value(c, f):
    return sum(c[f[j], j] for j in range(c.shape[1]))


def _valid(f, nI, nJ):
    cap = max(1, -(-nJ // nI))
    return f.shape == (nJ,) and (f >= 0).all() and (f < nI).all() and np.bincount(f, minlength=nI).max() <= cap


@pytest.mark.parametrize("nI,nJ", [(1, 1), (3, 3), (2, 5), (3, 7), (4, 2), (4, 7)])
def test_assignment_equals_brute_force(nI, nJ):
    """Every assignment with at most ceil(|J|/|I|) tasks per agent is
    enumerated; the library's optimum reaches the best value."""
    import itertools
    from paper_2305_04397_amd import morap
    rng = np.random.default_rng(nI * 10 + nJ)
    cap = max(1, -(-nJ // nI))
    C = rng.normal(size=(5, nI, nJ)) * rng.uniform(0.1, 10)
    F = morap.assign_host(C)
    for k in range(C.shape[0]):
        best = max(_value(C[k], f) for f in itertools.product(range(nI), repeat=nJ)
                   if np.bincount(f, minlength=nI).max() <= cap)
        assert _valid(F[k], nI, nJ)
        assert _value(C[k], F[k]) == pytest.approx(best, abs=1e-9)


@pytest.mark.parametrize("nI,nJ,K", [(50, 100, 64), (10, 20, 200), (30, 30, 3)])
def test_assignment_matches_oracle_at_workload_sizes(nI, nJ, K):
    """At the workloads' sizes (and with enough columns for the threaded
    path), the optimum equals the oracle's (scipy's Hungarian on the
    replicated matrix)."""
    from paper_2305_04397_amd import morap
    from oracle import alg
    rng = np.random.default_rng(nI + nJ + K)
    C = -rng.uniform(0, 200, size=(K, nI, nJ)) + rng.uniform(0, 1, size=(K, 1, nJ))
    F = morap.assign_host(C)
    for k in range(K):
        assert _valid(F[k], nI, nJ)
        fo = alg.assign(C[k])
        assert _value(C[k], F[k]) == pytest.approx(_value(C[k], fo), rel=1e-12, abs=1e-9)


def test_assignment_rejects_bad_input():
    from paper_2305_04397_amd import morap
    C = np.zeros((2, 3, 3))
    C[1, 2, 0] = np.nan
    with pytest.raises(morap.MorapError) as e:
        morap.assign_host(C)
    assert e.value.code == morap.E_INVALID
    out = np.zeros(3, np.int32)
    assert morap.lib.morap_assign_host(None, 3, 3, 1, out.ctypes.data) == morap.E_INVALID
    assert morap.lib.morap_assign_host(np.zeros(9).ctypes.data, 0, 3, 1, out.ctypes.data) == morap.E_INVALID
    assert morap.lib.morap_assign_host(np.zeros(9).ctypes.data, 3, 3, 0, out.ctypes.data) == morap.E_INVALID


# --------------------------------------------------------------------------
# product construction on the host (Sec. 2 "Product MDP", Sec. 3.1)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("name", ["example", "cfg1", "cfg2_sub", "tiny", "q0_accepting"])
def test_host_products_bit_exact(name):
    """The library's product builder, called without a context, gives the
    oracle's product bit for bit: states in (q, s) order, rows, successors,
    probabilities, both reward columns, the to-done flags and the initial
    state (-1 and no states when q0 is already accepting)."""
    from paper_2305_04397_amd import morap
    from workloads import worked_example, make_workload, tiny_workload
    from oracle import product
    if name == "q0_accepting":
        wl = worked_example()
        wl.tasks[0].q0 = 1
    else:
        wl = {"example": worked_example, "cfg1": lambda: make_workload(1),
              "cfg2_sub": lambda: make_workload(2, n_agents=3, n_tasks=5),
              "tiny": lambda: tiny_workload(5, 2, 3, width=3, height=3, kinds=("avoid", "reach"))}[name]()
    for i, ag in enumerate(wl.agents):
        for j, tk in enumerate(wl.tasks):
            g = morap.product_host(ag, tk, wl.letters[i][j])
            o = product.build_product(ag, tk, wl.letters[i][j])
            assert g["init"] == o.init
            assert g["state_row"].tolist() == o.state_row.tolist()
            assert g["row_ptr"].tolist() == o.row_ptr.tolist()
            assert g["col"].tolist() == o.col.tolist()
            assert np.array_equal(g["prob"], o.prob)
            assert np.array_equal(g["rew"][:, 0], o.rew_cost) and np.array_equal(g["rew"][:, 1], o.rew_prob)
            assert g["to_done"].astype(bool).tolist() == o.to_done.tolist()
            assert g["states"].tolist() == o.states.tolist()
    if name == "q0_accepting":
        assert g["init"] == -1 and len(g["state_row"]) == 1


def test_host_product_rejects_bad_letters():
    from paper_2305_04397_amd import morap
    from workloads import worked_example
    wl = worked_example()
    bad = np.array(wl.letters[0][0]).copy()
    bad[0] = wl.tasks[0].n_letters
    with pytest.raises(morap.MorapError) as e:
        morap.product_host(wl.agents[0], wl.tasks[0], bad)
    assert e.value.code == morap.E_INVALID


@pytest.mark.parametrize("case", ["duplicates", "collinear", "one_dim", "repeated_halfspaces"])
def test_projections_on_degenerate_sets(case):
    """Inputs Alg. 1 really produces: the same support point twice (two passes
    that return one point), points on a line, a single objective, and the same
    hyperplane recorded twice.  The library's projections agree with the
    oracle's and satisfy the optimality conditions."""
    from paper_2305_04397_amd import morap
    rng = np.random.default_rng(len(case))
    d = 1 if case == "one_dim" else 5
    base = rng.normal(size=(3, d)) * 10
    if case == "duplicates":
        Phi = np.vstack([base, base[:2]])
    elif case == "collinear":
        a, b = base[0], base[1]
        Phi = np.array([a + s * (b - a) for s in (0.0, 0.25, 0.5, 1.0)])
    else:
        Phi = base
    for t in (Phi.max(0) + 1.0, Phi.mean(0), Phi.min(0) - 1.0, Phi.max(0) + rng.uniform(-2, 2, d)):
        x, lam = morap.project_inner(Phi, t)
        xo, _ = geometry.project_inner(Phi, t)
        sc = max(1.0, np.abs(t).max())
        assert np.abs(x - xo).max() <= 1e-9 * sc
        assert geometry.kkt_inner(Phi, t, x, lam) <= 1e-9 * sc
        W = rng.dirichlet(np.ones(d), size=len(Phi))
        if case == "repeated_halfspaces":
            W = np.vstack([W, W[:2]])
            R = np.vstack([Phi, Phi[:2]])
        else:
            R = Phi
        z = morap.project_outer(W, R, t)
        assert np.abs(z - geometry.project_outer(W, R, t)).max() <= 1e-9 * sc
        assert (W @ z <= np.einsum("ij,ij->i", W, R) + 1e-9 * sc).all()


@pytest.mark.parametrize("nI,nJ", [(3, 3), (2, 5), (4, 2)])
def test_assignment_under_ties_is_valid(nI, nJ):
    """All-equal values and values equal per task (every assignment optimal):
    the result is still a valid assignment within each agent's capacity."""
    from paper_2305_04397_amd import morap
    C = np.stack([np.zeros((nI, nJ)), np.tile(np.arange(nJ, dtype=float), (nI, 1))])
    F = morap.assign_host(C)
    for k in range(2):
        assert _valid(F[k], nI, nJ)
        assert _value(C[k], F[k]) == pytest.approx(C[k].max(axis=0).sum(), abs=1e-12)


def test_binding_fails_loudly_without_the_library(tmp_path):
    """The binding has no fallback: a copy of it beside no built library
    refuses to import, naming the missing file."""
    import importlib.util
    import shutil
    src = os.path.join(ROOT, "paper_2305_04397_amd", "morap.py")
    dst = tmp_path / "morap_copy.py"
    shutil.copy(src, dst)
    spec = importlib.util.spec_from_file_location("morap_copy", dst)
    mod = importlib.util.module_from_spec(spec)
    with pytest.raises(ImportError, match="libmorap.so is missing"):
        spec.loader.exec_module(mod)


# --------------------------------------------------------------------------
# the team MDP (Def. teamMDP) built by the library on the host
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n,seed", [(2, 41), (3, 42), (2, 43)])
def test_host_team_model_equals_the_oracle(n, seed):
    """The library's team-MDP builder (written separately from the oracle's)
    gives the oracle's single-objective layout: states, rows, successors,
    probabilities, to-done flags and the initial state exactly, rewards to
    one rounding (the oracle's dot product may fuse its multiply-adds).  Its
    value from the initial state is the oracle's team value."""
    from paper_2305_04397_amd import morap
    from workloads import tiny_workload
    from oracle import centralised
    kinds = ("reach",) if seed != 43 else ("avoid", "reach")
    wl = tiny_workload(seed, n, n, width=3, height=2, kinds=kinds, k=1, p_slip=0.25)
    team = centralised.build_team_mdp(wl)
    rng = np.random.default_rng(seed)
    for _ in range(2):
        w = rng.dirichlet(np.ones(2 * n))
        g = morap.team_model_host(wl, w)
        o = centralised.single_objective_model(team, w)
        for k in ("state_row", "row_ptr", "col", "to_done"):
            assert g[k].tolist() == o[k].tolist(), k
        assert np.array_equal(g["prob"], o["prob"]) and g["init"] == o["init"]
        assert np.abs(g["rew"] - o["rew"]).max() <= 4e-16 * max(1.0, np.abs(o["rew"]).max())
        # plain VI on the library's model
        S, R = len(g["state_row"]) - 1, len(g["row_ptr"]) - 1
        P = sp.csr_matrix((g["prob"], g["col"], g["row_ptr"]), shape=(R, S))
        x = np.zeros(S)
        for _ in range(100_000):
            y = np.maximum.reduceat(g["rew"][:, 0] + P @ x, g["state_row"][:-1])
            if np.abs(y - x).max() <= 1e-13:
                break
            x = y
        assert y[g["init"]] == pytest.approx(centralised.team_value(team, w), abs=1e-10)


@pytest.mark.parametrize("n,seed", [(2, 41), (3, 42), (2, 43)])
def test_host_team_mo_model_equals_the_oracle(n, seed):
    """The team MDP with its d = 2n objectives (one reward pair and its two
    objective indices per row): the same states, rows, successors and
    probabilities as the scalarised layout, and each row's objective vector,
    spread out from (rew, obj), is the oracle's exactly (states without rows
    get one empty row with the zero vector)."""
    from paper_2305_04397_amd import morap
    from workloads import tiny_workload
    from oracle import centralised
    kinds = ("reach",) if seed != 43 else ("avoid", "reach")
    wl = tiny_workload(seed, n, n, width=3, height=2, kinds=kinds, k=1, p_slip=0.25)
    team = centralised.build_team_mdp(wl)
    d = 2 * n
    g = morap.team_model_mo_host(wl)
    o = centralised.single_objective_model(team, np.full(d, 1.0 / d))
    for k in ("state_row", "row_ptr", "col", "to_done"):
        assert g[k].tolist() == o[k].tolist(), k
    assert np.array_equal(g["prob"], o["prob"]) and g["init"] == o["init"]
    R = len(g["row_ptr"]) - 1
    assert g["obj"].shape == (R, 2) and g["obj"].min() >= 0 and g["obj"].max() < d
    spread = np.zeros((R, d))
    np.add.at(spread, (np.arange(R), g["obj"][:, 0]), g["rew"][:, 0])
    np.add.at(spread, (np.arange(R), g["obj"][:, 1]), g["rew"][:, 1])
    want = []
    for s in range(team.n_states):
        lo, hi = team.state_row[s], team.state_row[s + 1]
        want.extend(team.rew[lo:hi] if hi > lo else [np.zeros(d)])
    assert np.array_equal(spread, np.array(want))


def test_host_team_model_rejects_unequal_counts():
    from paper_2305_04397_amd import morap
    from workloads import tiny_workload
    wl = tiny_workload(44, 2, 3, width=3, height=2, kinds=("reach",), k=1)
    with pytest.raises(morap.MorapError) as e:
        morap.team_model_host(wl, np.full(5, 0.2))
    assert e.value.code == morap.E_INVALID


def test_proposer_target_on_the_host():
    """The proposer's training target (host only): the face normal
    M (t - t_down) at the closest point for a threshold outside, the last
    weight vector for one inside; clipped at 0, normalised to sum 1."""
    from paper_2305_04397_amd import morap
    t = np.array([-1.0, -2.0, 0.9])
    t_down = np.array([-1.5, -2.0, 0.5])
    w = morap.proposer_target(t, t_down, np.array([0.2, 0.3, 0.5]))
    assert np.allclose(w, [0.5 / 0.9, 0.0, 0.4 / 0.9], atol=1e-15)
    # negative parts of the normal are rounding noise and become 0
    w = morap.proposer_target(t, t_down + np.array([0.0, 1e-3, 0.0]), np.ones(3) / 3)
    assert w[1] == 0.0 and w.sum() == pytest.approx(1.0, abs=1e-15)
    # inside: the last weight vector, normalised
    w = morap.proposer_target(t, t, np.array([1.0, 1.0, 2.0]))
    assert np.allclose(w, [0.25, 0.25, 0.5])
    # a diagonal norm matrix scales the normal
    w = morap.proposer_target(t, t_down, np.zeros(3), M=np.diag([2.0, 1.0, 1.0]))
    assert np.allclose(w, [1.0 / 1.4, 0.0, 0.4 / 1.4])
    with pytest.raises(morap.MorapError):
        morap.proposer_target(np.array([np.nan, 0.0, 0.0]), t_down, np.ones(3))
