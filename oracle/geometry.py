"""Geometry of Alg. 1 (Sec. 3.3): M-norm, the projection of t onto the inner
approximation down(Phi) and onto the outer approximation given by Lambda, and
the weight update.

Both projections are least-distance problems after the change of variables
y = L^T (x - t) with M = L L^T (so ||x - t||_M = ||y||_2):
  * outer (find z minimising ||t - z|| s.t. w'.z <= w'.r' for all (w', r')):
    min ||y|| s.t. -(L^{-1} w')^T y >= w'.(t - r');
  * inner (find x in down(Phi) minimising ||t - x||): the minimum-norm point of
    conv{L^T (r_i - t)} + cone{-L^T e_k}.  A point y* of that set is the
    minimum-norm point iff y*.g >= ||y*||^2 for every point generator g and
    y*.g >= 0 for every ray; hence y* = z*/||z*||^2 where z* solves
    min ||z|| s.t. v_i.z >= 1, g_k.z >= 0, and the problem has no solution iff
    t already lies in down(Phi).
Each least-distance problem min ||z|| s.t. G z >= h is solved exactly by the
classical reduction to non-negative least squares (Lawson and Hanson, "Solving
Least Squares Problems", ch. 23): with u >= 0 minimising
|| [G^T; h^T] u - e_{n+1} ||, r = [G^T; h^T] u - e_{n+1}; the problem is
infeasible iff r = 0, else z = -r[:n] / r[n].  The NNLS step is Lawson and
Hanson's active-set algorithm (ch. 23, algorithm NNLS) written out below with
dense least-squares solves; every projection is then checked against its
optimality conditions.

Readings: ||v|| is sqrt(v^T M v) (the text's "||v| = <v, v>" is garbled;
squaring does not move a minimiser).  M defaults to the identity.
"""
from __future__ import annotations

import numpy as np

def nnls(A: np.ndarray, b: np.ndarray, maxiter: int | None = None):
    """min ||A x - b||_2 subject to x >= 0 (Lawson and Hanson's NNLS).
    Returns (x, ||A x - b||)."""
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    m, n = A.shape
    maxiter = 3 * n + 30 if maxiter is None else maxiter
    x = np.zeros(n)
    passive = np.zeros(n, dtype=bool)
    tol = 10 * np.finfo(float).eps * max(1.0, np.abs(A).max()) * max(m, n)
    w = A.T @ (b - A @ x)
    for _ in range(maxiter):
        cand = ~passive & (w > tol)
        if not cand.any():
            break
        j = int(np.argmax(np.where(cand, w, -np.inf)))
        passive[j] = True
        while True:
            s = np.zeros(n)
            idx = np.flatnonzero(passive)
            s[idx] = np.linalg.lstsq(A[:, idx], b, rcond=None)[0]
            if (s[idx] > 0).all():
                break
            neg = idx[s[idx] <= 0]
            alpha = np.min(x[neg] / (x[neg] - s[neg]))
            x = x + alpha * (s - x)
            passive &= x > tol
            x[~passive] = 0.0
        x = s
        w = A.T @ (b - A @ x)
    else:
        raise RuntimeError("NNLS did not converge")
    return x, float(np.linalg.norm(A @ x - b))



# Every projection is certified by its optimality conditions: the largest
# violation (kkt_inner / kkt_outer) must be at most KKT_TOL * max(1, ||t||_inf).
KKT_TOL = 1e-10


def mnorm(v: np.ndarray, M: np.ndarray | None = None) -> float:
    v = np.asarray(v, dtype=np.float64)
    if M is None:
        return float(np.sqrt(v @ v))
    return float(np.sqrt(max(v @ M @ v, 0.0)))


def _chol(M, d):
    if M is None:
        return np.eye(d)
    return np.linalg.cholesky(np.asarray(M, dtype=np.float64))


def ldp(G: np.ndarray, h: np.ndarray):
    """min ||z||_2 s.t. G z >= h.  Returns (z, u) or (None, u) if infeasible;
    u >= 0 are the non-negative least-squares coefficients (multipliers up to
    scale)."""
    m, n = G.shape
    E = np.vstack([G.T, h[None, :]])
    f = np.zeros(n + 1)
    f[n] = 1.0
    u, _ = nnls(E, f)
    r = E @ u - f
    scale = max(1.0, float(np.abs(E).max()))
    if np.linalg.norm(r) <= 1e-13 * scale or r[n] >= 0.0:
        return None, u
    return -r[:n] / r[n], u


def project_inner(Phi: np.ndarray, t: np.ndarray, M: np.ndarray | None = None):
    """x in down(conv Phi) minimising ||t - x||_M (Alg. 1, inner problem).

    Returns (x, lam) with x <= Phi^T lam, lam >= 0, sum lam = 1; x == t when
    t lies in down(Phi)."""
    Phi = np.atleast_2d(np.asarray(Phi, dtype=np.float64))
    t = np.asarray(t, dtype=np.float64)
    m, d = Phi.shape
    L = _chol(M, d)
    V = (Phi - t[None, :]) @ L            # rows: L^T (r_i - t)
    Gr = -L                              # rows: -L^T e_k  (row k of -L)
    G = np.vstack([V, Gr])
    h = np.concatenate([np.ones(m), np.zeros(d)])
    z, u = ldp(G, h)
    if z is None:
        # t is inside down(Phi): find a witness lam with Phi^T lam >= t
        lam = _witness(Phi, t)
        return t.copy(), lam
    y = z / float(z @ z)
    x = t + np.linalg.solve(L.T, y)
    s = u[:m].sum()
    lam = u[:m] / s if s > 0 else np.full(m, 1.0 / m)
    if M is None:
        x, lam = _polish_inner(Phi, t, x, lam)
    viol = kkt_inner(Phi, t, x, lam, M)
    if viol > KKT_TOL * max(1.0, float(np.abs(t).max())):
        raise RuntimeError(f"inner projection failed its optimality check ({viol:.3g})")
    return x, lam


def _polish_inner(Phi, t, x, lam):
    """Active-set refinement of an inner projection (M = I).  On the face the
    solution identifies (the points with lam > 0, the components k where
    x_k binds at (Phi^T lam)_k < t_k), the projection is the equality-
    constrained least-squares problem  min sum_{k in K} (t_k - (Phi_S^T lam)_k)^2
    subject to sum lam = 1,  with x_k = t_k off K; solved exactly through its
    KKT system.  The least-distance reduction above loses accuracy when t is
    far from down(Phi) (its answer is then a small vector divided by a small
    number); the refined point is kept only if it satisfies the optimality
    conditions at least as well."""
    w = t - x
    K = np.flatnonzero(w > 1e-9 * max(1.0, float(np.abs(w).max())))
    S = np.flatnonzero(lam > 1e-12)
    if K.size == 0 or S.size == 0:
        return x, lam
    A = Phi[S][:, K].T                       # |K| x |S|
    b = t[K]
    n = S.size
    kkt = np.zeros((n + 1, n + 1))
    kkt[:n, :n] = A.T @ A
    kkt[:n, n] = 1.0
    kkt[n, :n] = 1.0
    rhs = np.concatenate([A.T @ b, [1.0]])
    try:
        sol = np.linalg.lstsq(kkt, rhs, rcond=None)[0]
    except np.linalg.LinAlgError:
        return x, lam
    ls = sol[:n]
    if (ls < -1e-12).any():
        return x, lam
    lam2 = np.zeros_like(lam)
    lam2[S] = np.maximum(ls, 0.0)
    lam2 /= lam2.sum()
    x2 = np.minimum(t, Phi.T @ lam2)
    if kkt_inner(Phi, t, x2, lam2) <= kkt_inner(Phi, t, x, lam):
        return x2, lam2
    return x, lam


def _witness(Phi: np.ndarray, t: np.ndarray) -> np.ndarray:
    """A convex combination lam with Phi^T lam >= t (feasibility witness), by
    a linear program."""
    from scipy.optimize import linprog
    m, d = Phi.shape
    # maximise s subject to Phi^T lam - s >= t, sum lam = 1, lam >= 0
    c = np.zeros(m + 1)
    c[-1] = -1.0
    A_ub = np.hstack([-Phi.T, np.ones((d, 1))])
    b_ub = -t
    A_eq = np.concatenate([np.ones(m), [0.0]])[None, :]
    res = linprog(c, A_ub=A_ub, b_ub=b_ub, A_eq=A_eq, b_eq=[1.0],
                  bounds=[(0, None)] * m + [(None, None)], method="highs")
    return res.x[:m] if res.status == 0 else np.full(m, 1.0 / m)


def project_outer(Ws: np.ndarray, Rs: np.ndarray, t: np.ndarray,
                  M: np.ndarray | None = None) -> np.ndarray:
    """z minimising ||t - z||_M s.t. w'.z <= w'.r' for every (w', r') in
    Lambda (Alg. 1, outer problem)."""
    Ws = np.atleast_2d(np.asarray(Ws, dtype=np.float64))
    Rs = np.atleast_2d(np.asarray(Rs, dtype=np.float64))
    t = np.asarray(t, dtype=np.float64)
    d = t.shape[0]
    L = _chol(M, d)
    # w'^T L^{-T} y <= w'.(r' - t)  <=>  -(L^{-1} w')^T y >= w'.(t - r')
    G = -np.linalg.solve(L, Ws.T).T
    h = np.einsum("ij,ij->i", Ws, t[None, :] - Rs)
    if (h <= 0).all():
        return t.copy()
    z, _ = ldp(G, h)
    if z is None:
        raise RuntimeError("outer approximation is empty")
    out = t + np.linalg.solve(L.T, z)
    viol = kkt_outer(Ws, Rs, t, out, M)
    if viol > KKT_TOL * max(1.0, float(np.abs(t).max())):
        raise RuntimeError(f"outer projection failed its optimality check ({viol:.3g})")
    return out


NOISE = 1e-12   # relative size of the projection's rounding noise


def weight_from(t: np.ndarray, t_up: np.ndarray, M: np.ndarray | None = None) -> np.ndarray | None:
    """w = M (t - t_up) / ||M (t - t_up)||_1 (Alg. 1, weight update).  The
    direction is non-negative in exact arithmetic (Lemma lem:weight-vector).
    Components at or below NOISE * max(1, ||t||_inf) are rounding noise of the
    projection t_up and are set to 0, like negative ones (a positive noise
    component would otherwise become the whole objective of the models it
    touches).  Returns None when nothing is left (t_up = t to rounding)."""
    t = np.asarray(t, dtype=np.float64)
    v = t - np.asarray(t_up, dtype=np.float64)
    wv = v if M is None else np.asarray(M, dtype=np.float64) @ v
    floor = NOISE * max(1.0, float(np.abs(t).max()))
    wv = np.where(wv > floor, wv, 0.0)
    s = wv.sum()
    return wv / s if s > 0 else None


def kkt_inner(Phi, t, x, lam, M=None) -> float:
    """Largest violation of the optimality conditions of the inner projection:
    x <= Phi^T lam, lam in the simplex, w = M(t - x) >= 0, w.r_i <= w.x for
    every point, and w_k = 0 wherever x_k < (Phi^T lam)_k."""
    Phi = np.atleast_2d(Phi)
    t, x, lam = map(np.asarray, (t, x, lam))
    w = (t - x) if M is None else np.asarray(M) @ (t - x)
    v = Phi.T @ lam
    viol = [max(0.0, float((x - v).max())), max(0.0, float(-lam.min())),
            abs(float(lam.sum()) - 1.0), max(0.0, float(-w.min())),
            max(0.0, float((Phi @ w - w @ x).max())),
            float(np.abs(w * (v - x)).max())]
    return max(viol)


def kkt_outer(Ws, Rs, t, z, M=None, tol=1e-9) -> float:
    """Largest violation of the optimality conditions of the outer projection
    (feasibility, and M(t - z) a non-negative combination of the constraint
    normals that are active at z)."""
    Ws, Rs = np.atleast_2d(Ws), np.atleast_2d(Rs)
    t, z = np.asarray(t), np.asarray(z)
    b = np.einsum("ij,ij->i", Ws, Rs)
    slack = b - Ws @ z
    g = (t - z) if M is None else np.asarray(M) @ (t - z)
    act = slack <= tol * max(1.0, float(np.abs(b).max()))
    if not act.any():
        return max(max(0.0, float(-slack.min())), float(np.abs(g).max()))
    mu, res = nnls(Ws[act].T, g)
    return max(max(0.0, float(-slack.min())), float(res))
