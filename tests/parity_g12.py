"""Parity contract of a support step (Alg. 2) against the oracle, per column
(reading G12 of the design notes):

  * assignment: the device's assignment is optimal for its own values c, so
    on the oracle's values it is within the FP32 errors of the pairs involved
    of the oracle's optimum: sum_j c°[f(j), j] >= opt° - sum_j (|c - c°|[f(j), j]
    + |c - c°|[f°(j), j]); when it is not the oracle's assignment it is checked
    by that bound, never skipped;
  * actions: identical to the exact optimum's (policy iteration) wherever the
    exact Q-gap exceeds tau_cmp = max(1e-9, 2 err_exact, 4 err_vi), err_vi the
    distance of an eps-stopped value iteration from the exact values (the
    accuracy the device's values have); states under that gap are counted as
    excluded, not compared, and so are, apart, the exact ties among them;
  * r: the oracle's Alg. 4 evaluation of the device's own policies, to 1e-9
    relative (plus 4 eps_eval);
  * w.r: the oracle's sum_j c°[f(j), j] to 1e-6 relative (Lemma lem:face).

Returns a report with the per-result errors the step showed."""
import numpy as np

from oracle import vi, alg


def _scaled(wi, wj):
    sc = wi + wj
    return (wi / sc, wj / sc) if sc > 0 else (wi, wj)


class Report(dict):
    def add(self, key, v, op=max):
        self[key] = op(self.get(key, v), v)


def check_support(ctx, prods, nI, nJ, W, r, A, c, co, eps, report=None, columns=None):
    report = Report() if report is None else report
    cache = {}
    for k in (range(W.shape[0]) if columns is None else columns):
        w = W[k]
        f = np.asarray(A[k])
        fo = alg.assign(co[k])
        val = sum(co[k][f[j], j] for j in range(nJ))
        opt = sum(co[k][fo[j], j] for j in range(nJ))
        e = np.abs(c[k] - co[k])
        bound = sum(e[f[j], j] + e[fo[j], j] for j in range(nJ)) + 1e-12 * max(1.0, abs(opt))
        assert val >= opt - bound, (k, val, opt, bound)
        report.add("c_err_rel", float((e / np.maximum(1.0, np.abs(co[k]))).max()))
        report.add("assign_gap", float(opt - val))
        report.add("columns_not_oracle_assignment", int(not np.array_equal(f, fo)), op=lambda a, b: a + b)
        ro = np.zeros(nI + nJ)
        for j in range(nJ):
            i = int(f[j])
            p = prods[i * nJ + j]
            if p.n_states == 0 or p.init < 0:
                continue
            mu = ctx.get_policy(k, j, p.n_states).astype(np.int64)
            a, b = _scaled(w[i], w[nI + j])
            key = (i * nJ + j, a, b)
            if key not in cache:
                v, Q, err = vi.optimal_exact(p, a, b)
                y, _ = vi.value_iteration(p, a, b, eps)
                cache[key] = (Q, max(1e-9, 2 * err, 4 * float(np.abs(y[:, 0] - v).max())))
            Q, tau = cache[key]
            best, gap = vi.q_gaps(p, Q)
            clear = gap > tau
            wrong = np.flatnonzero(clear & (mu != best))
            assert wrong.size == 0, (k, j, wrong[:5], gap[wrong[:5]], tau)
            report.add("states", int(p.n_states), op=lambda x, y: x + y)
            report.add("excluded_states", int((~clear).sum()), op=lambda x, y: x + y)
            # of which exact ties (several actions equally good to 1e-9)
            report.add("excluded_exact_ties", int((gap <= 1e-9).sum()), op=lambda x, y: x + y)
            report.add("tau_cmp_max", tau)
            (vc, vp), _, _ = vi.evaluate(p, mu, eps)
            ro[nI + j] = vp
            ro[i] += vc
        rerr = float(np.abs(r[k] - ro).max())
        assert rerr <= 1e-9 * max(1.0, np.abs(ro).max()) + 4 * eps, (k, rerr)
        report.add("r_err", rerr)
        wr = float(w @ r[k])
        assert abs(wr - val) <= 1e-6 * max(1.0, abs(val)), (k, wr, val)
        report.add("wr_err_rel", abs(wr - val) / max(1.0, abs(val)))
    return report
