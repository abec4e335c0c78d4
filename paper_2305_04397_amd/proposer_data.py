"""Training data and features for the learned weight proposer.

Everything here runs through the library (the plain Alg. 1 loop on the
device); nothing is learned from the oracle.

* ``features``: the instance summary phi the proposer sees beside the threshold
  point: the ideal point (the optimum of every single objective, one batched
  solve with the d unit weight vectors), the mean slip probability of the
  agents and log10 of the number of product states.
* ``around`` / ``thresholds``: threshold points t = u + delta |u| around front
  points u (delta ~ U[-0.3, 0.3] per coordinate, or U[-0.3, 0] for every
  second one when half of them should be achievable; probabilities clipped to
  [0, 1]).
* ``target_weight``: the weight vector a query should have started from: for
  a threshold outside the achievable set, the normal M (t - t_down) of the
  face holding the closest point; otherwise the last weight vector the plain
  loop used.  Both normalised to sum 1.
* ``generate``: plain-loop queries in lockstep batches, returning the network
  inputs [t; phi], the targets and the query results.
* ``generate_from_support``: tuples from the plain method's own support steps
  (Alg. 2): for weight vectors w drawn from Dirichlet(1_d), the point r(w) the
  support step returns lies on the front and w is the normal of a face
  holding it, so thresholds drawn around r(w) (as above) get w as target.  One
  support call gives 64 such points, so 200k tuples cost a few thousand
  passes instead of 200k full queries.
"""
from __future__ import annotations

import numpy as np


def features(ctx, wl, opts) -> np.ndarray:
    nI, nJ = wl.n_agents, wl.n_tasks
    d = nI + nJ
    r, _, _, _ = ctx.support(np.eye(d), opts)
    ideal = np.array([r[k, k] for k in range(d)])
    states = sum(ctx.model_info(m)["n_states"] for m in range(nI * nJ))
    slip = float(np.mean([a.p_slip for a in wl.agents]))
    return np.concatenate([ideal, [slip, np.log10(max(states, 1))]])


def front_points(ctx, wl, n, rng, opts) -> np.ndarray:
    d = wl.n_agents + wl.n_tasks
    out = []
    for b in range(0, n, 64):
        k = min(64, n - b)
        r, _, _, _ = ctx.support(rng.dirichlet(np.ones(d), size=k), opts)
        out.append(r)
    return np.vstack(out)


def around(rng, u: np.ndarray, nI: int, inside_half: bool = False) -> np.ndarray:
    """One threshold per row of u: u + delta |u|, delta ~ U[-0.3, 0.3] per
    coordinate (every second row U[-0.3, 0], below its point and hence
    achievable, with inside_half); probabilities clipped to [0, 1]."""
    hi = np.full((u.shape[0], 1), 0.3)
    if inside_half:
        hi[1::2] = 0.0
    t = u + (rng.uniform(0.0, 1.0, size=u.shape) * (hi + 0.3) - 0.3) * np.abs(u)
    t[:, nI:] = np.clip(t[:, nI:], 0.0, 1.0)
    return t


def thresholds(rng, front: np.ndarray, n: int, nI: int, inside_half: bool = False) -> np.ndarray:
    """n thresholds around rows of front drawn at random (see ``around``)."""
    return around(rng, front[rng.integers(front.shape[0], size=n)], nI, inside_half)


def target_weight(t: np.ndarray, res: dict, M=None) -> np.ndarray:
    from paper_2305_04397_amd.morap import proposer_target
    return proposer_target(t, res["t_down"], res["W"][-1], M)


def generate(ctx, wl, T: np.ndarray, phi: np.ndarray, opts, eps: float = 0.01, max_iter: int = 64,
             batch: int = 64, errors: list | None = None):
    """Plain-loop queries for every row of T; returns (X, Wt, results).  A
    batch the library rejects is skipped; its message goes to ``errors`` when
    a list is given, otherwise the error is raised."""
    from paper_2305_04397_amd.morap import MorapError
    X, Wt, results = [], [], []
    for b in range(0, T.shape[0], batch):
        try:
            res = ctx.query_batch(T[b:b + batch], eps=eps, max_iter=max_iter, opts=opts, trace=True)
        except MorapError as e:
            if errors is None:
                raise
            errors.append(str(e))
            continue
        for t, q in zip(T[b:b + batch], res):
            X.append(np.concatenate([t, phi]))
            Wt.append(target_weight(t, q))
            results.append(q)
    return np.asarray(X, np.float32), np.asarray(Wt, np.float32), results


def generate_from_support(ctx, wl, n_points: int, per_point: int, phi: np.ndarray, rng, opts,
                          inside_half: bool = True):
    """(X, Wt): n_points support points, per_point thresholds around each
    (with inside_half, every second threshold lies below its point), network
    inputs [t; phi] and the generating weight vectors as targets."""
    nI, d = wl.n_agents, wl.n_agents + wl.n_tasks
    X, Wt = [], []
    for b in range(0, n_points, 64):
        k = min(64, n_points - b)
        W = rng.dirichlet(np.ones(d), size=k)
        W /= W.sum(axis=1, keepdims=True)
        r, _, _, _ = ctx.support(W, opts)
        u = np.repeat(r, per_point, axis=0)
        t = around(rng, u, nI, inside_half)
        X.append(np.hstack([t, np.broadcast_to(phi, (t.shape[0], phi.size))]))
        Wt.append(np.repeat(W, per_point, axis=0))
    return np.vstack(X).astype(np.float32), np.vstack(Wt).astype(np.float32)

