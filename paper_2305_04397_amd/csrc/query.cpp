// Alg. 1 (point-oriented Pareto computation, Sec. 3.3) on the host, with the
// supporting-hyperplane step (Alg. 2) on the device.  Several queries advance
// in lockstep: each pass solves the current weight vectors of all unfinished
// queries as the columns of one batched value iteration.
//
// Loop control (a reading of the loop test): t_up is recomputed right after
// each new point is added and ||t_down - t_up||_M <= eps is tested at once;
// this never divides 0/0 in the weight update.  Verdict: FEASIBLE iff t lies
// in down(Phi), INFEASIBLE iff some (w', r') has w'.r' < w'.t, otherwise
// UNDECIDED.
#include "common.h"

#include <cstdio>
#include <cstdlib>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <exception>
#include <mutex>
#include <thread>

namespace morap {

void proposer_infer_host(morap_ctx* c, const float* X, int n, float* out);   // mlp.hip
bool proposer_ready(const morap_ctx* c, int n_in, int d);

namespace {

double mnorm(const std::vector<double>& v, const double* M) {
    const int d = (int)v.size();
    double s = 0;
    if (!M) {
        for (double x : v) s += x * x;
    } else {
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j) s += v[i] * M[(size_t)i * d + j] * v[j];
    }
    return std::sqrt(std::max(s, 0.0));
}

struct QState {
    std::vector<double> t, t_up, t_down, w, lam;
    std::vector<std::vector<double>> Phi, Ws;
    std::vector<std::vector<int32_t>> Fs;   // assignment of every pass
    bool done = false, separated = false;
    int fallback = 0;
    int learned_passes = 0;      // passes whose weight vector the proposer gave
    double gap_before = -1.0;    // the gap when the last learned weight was set
    double latency_ms = -1.0;   // set when the query stops
    double gap = 0;
    int64_t backups = 0;
    double ms = 0;
};

// f(i) for i < n on up to 16 host threads; the first exception is rethrown.
template <class F>
void parallel_for(int n, F f) {
    const int nt = std::max(1, std::min<int>(n, (int)std::min(16u, std::thread::hardware_concurrency())));
    if (nt == 1) {
        for (int i = 0; i < n; ++i) f(i);
        return;
    }
    std::atomic<int> next{0};
    std::exception_ptr err;
    std::mutex mu;
    auto worker = [&] {
        for (int i; (i = next++) < n;) {
            try {
                f(i);
            } catch (...) {
                std::lock_guard<std::mutex> g(mu);
                if (!err) err = std::current_exception();
            }
        }
    };
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t) th.emplace_back(worker);
    for (auto& t : th) t.join();
    if (err) std::rethrow_exception(err);
}

// The proposer's weight vectors after the first pass (morap_query_opts,
// proposer_passes): input [t_down; phi]; a proposal replaces Alg. 1's update
// only while it is valid, new to the query, and the previous learned pass
// shrank the gap by 1 %, else the query keeps the update from then on.
void propose_later(morap_ctx* c, std::vector<QState>& qs, const std::vector<int>& act, int d, int passes) {
    std::vector<int> ask;
    for (int q : act) {
        const QState& s = qs[q];
        if (!s.done && s.fallback == 0 && s.learned_passes > 0 && s.learned_passes < passes) ask.push_back(q);
    }
    if (ask.empty()) return;
    const int nfeat = (int)c->features.size();
    std::vector<float> X(ask.size() * (size_t)(d + nfeat)), out(ask.size() * (size_t)d);
    for (size_t a = 0; a < ask.size(); ++a) {
        const QState& s = qs[ask[a]];
        for (int k = 0; k < d; ++k) X[a * (d + nfeat) + k] = (float)s.t_down[k];
        for (int k = 0; k < nfeat; ++k) X[a * (d + nfeat) + d + k] = (float)c->features[k];
    }
    proposer_infer_host(c, X.data(), (int)ask.size(), out.data());
    for (size_t a = 0; a < ask.size(); ++a) {
        QState& s = qs[ask[a]];
        std::vector<double> w(d);
        double sum = 0;
        bool ok = !(s.gap >= 0.99 * s.gap_before);
        for (int k = 0; k < d; ++k) {
            const double v = out[a * d + k];
            ok &= std::isfinite(v) && v >= 0;
            w[k] = v;
            sum += v;
        }
        ok &= std::fabs(sum - 1.0) <= 1e-3 && sum > 0;
        if (ok) {
            for (auto& v : w) v /= sum;
            for (const auto& prev : s.Ws) {
                double diff = 0;
                for (int k = 0; k < d; ++k) diff = std::max(diff, std::fabs(prev[k] - w[k]));
                ok &= diff > 1e-6;
            }
        }
        if (ok) {
            s.gap_before = s.gap;
            s.w = w;
            ++s.learned_passes;
        } else {
            s.fallback = 2;
        }
    }
}

}  // namespace

void query_batch(morap_ctx* c, const double* T, const double* W0, int Q, const double* M,
                 const morap_query_opts& o, morap_query_result* res) {
    MORAP_CHECK(c->loaded, MORAP_E_STATE, "no models loaded");
    MORAP_CHECK(T && res && Q >= 1, MORAP_E_INVALID, "bad query arguments");
    MORAP_CHECK(o.eps >= 0 && o.max_iter >= 1, MORAP_E_INVALID, "need eps >= 0 and max_iter >= 1");
    const int nI = n_agents_of(c), nJ = n_tasks_of(c), d = nI + nJ;
    for (int64_t i = 0; i < (int64_t)Q * d; ++i) MORAP_CHECK(std::isfinite(T[i]), MORAP_E_INVALID, "t must be finite");
    std::vector<QState> qs(Q);
    const auto t_start = std::chrono::steady_clock::now();
    // initial weight vectors: e_1, or the learned proposer's output
    std::vector<float> prop;
    const int nfeat = (int)c->features.size();
    const bool learned = o.use_proposer && proposer_ready(c, d + nfeat, d);
    if (learned) {
        std::vector<float> X((size_t)Q * (d + nfeat));
        for (int q = 0; q < Q; ++q) {
            for (int k = 0; k < d; ++k) X[(size_t)q * (d + nfeat) + k] = (float)T[(size_t)q * d + k];
            for (int k = 0; k < nfeat; ++k) X[(size_t)q * (d + nfeat) + d + k] = (float)c->features[k];
        }
        prop.resize((size_t)Q * d);
        proposer_infer_host(c, X.data(), Q, prop.data());
    }
    for (int q = 0; q < Q; ++q) {
        QState& s = qs[q];
        s.t.assign(T + (size_t)q * d, T + (size_t)(q + 1) * d);
        s.t_down = s.t;
        s.t_up.assign(d, -INFINITY);
        s.w.assign(d, 0.0);
        s.w[0] = 1.0;
        if (W0) {
            double sum = 0;
            for (int k = 0; k < d; ++k) {
                const double v = W0[(size_t)q * d + k];
                MORAP_CHECK(std::isfinite(v) && v >= 0, MORAP_E_INVALID, "first weights must be finite and >= 0");
                sum += v;
            }
            MORAP_CHECK(std::fabs(sum - 1.0) <= 1e-9, MORAP_E_INVALID, "first weight rows must sum to 1");
            s.w.assign(W0 + (size_t)q * d, W0 + (size_t)(q + 1) * d);
        } else if (o.use_proposer) {
            bool ok = learned;
            std::vector<double> w(d);
            double sum = 0;
            for (int k = 0; ok && k < d; ++k) {
                const double v = learned ? prop[(size_t)q * d + k] : 0.0;
                ok &= std::isfinite(v) && v >= 0;
                w[k] = v;
                sum += v;
            }
            ok &= std::fabs(sum - 1.0) <= 1e-3 && sum > 0;
            if (ok) {
                for (auto& v : w) v /= sum;
                s.w = w;
                s.learned_passes = 1;
                s.gap_before = INFINITY;
            } else {
                s.fallback = 1;   // plain rule: start from (1, 0, ..., 0)
            }
        }
    }
    morap_vi_opts vo = o.vi;
    // MORAP_PROGRESS=1: one line per Alg. 1 pass on stderr (long lockstep
    // batches report as they go)
    static const bool progress = [] {
        const char* p = std::getenv("MORAP_PROGRESS");
        return p && *p && *p != '0';
    }();
    // groups of at most 64 queries, each run to its end before the next
    // (a group's solves can then start from its previous pass's values)
    std::vector<int> prev_col(Q, -1);
    double last_ms[3] = {0, 0, 0};   // solve, assignment + evaluation, geometry of the last pass
    int64_t last_sweeps = 0;
    for (int g0 = 0; g0 < Q; g0 += 64) {
        const int g1 = std::min(Q, g0 + 64);
        for (int it = 0; it < o.max_iter; ++it) {
            std::vector<int> act;
            for (int q = g0; q < g1; ++q)
                if (!qs[q].done) act.push_back(q);
            if (act.empty()) break;
            if (progress) {
                std::fprintf(stderr,
                             "[morap] Alg. 1 pass %d: %zu of %d queries running (%.0f ms; last pass: solve %.0f ms in %lld "
                             "sweeps, assignment and evaluation %.0f, geometry %.0f ms)\n",
                             it + 1, act.size(), g1 - g0,
                             std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start)
                                 .count(),
                             last_ms[0], (long long)last_sweeps, last_ms[1], last_ms[2]);
                std::fflush(stderr);
            }
            {
                const int K = (int)act.size();
                std::vector<double> W((size_t)K * d), C((size_t)K * nI * nJ), R((size_t)K * d);
                std::vector<int32_t> A((size_t)K * nJ), warm_map(K);
                for (int kk = 0; kk < K; ++kk) {
                    // re-normalise so the row sums to 1 to the last bit
                    const auto& w = qs[act[kk]].w;
                    double sum = 0;
                    for (double v : w) sum += v;
                    for (int q = 0; q < d; ++q) W[(size_t)kk * d + q] = w[q] / sum;
                    warm_map[kk] = prev_col[act[kk]];
                    prev_col[act[kk]] = kk;
                }
                Stats st;
                const auto t0 = std::chrono::steady_clock::now();
                solve(c, W.data(), K, vo, C.data(), st, o.warm_start && it > 0 ? warm_map.data() : nullptr);
                const auto t1 = std::chrono::steady_clock::now();
                // a team model's policy assigns by itself (A stays 0)
                if (!c->team) assign_columns(nI, nJ, C.data(), K, A.data());
                // after an FP32 solve the assignment is checked on FP64 values
                std::vector<int32_t> F(A);
                evaluate(c, A.data(), K, vo, R.data(), st, o.warm_start && it > 0 ? warm_map.data() : nullptr,
                         c->team ? nullptr : F.data());
                if (!c->team) A = F;
                const auto t2 = std::chrono::steady_clock::now();
                const double ms = std::chrono::duration<double, std::milli>(t2 - t0).count();
                last_ms[0] = std::chrono::duration<double, std::milli>(t1 - t0).count();
                last_sweeps = st.sweeps;
                last_ms[1] = std::chrono::duration<double, std::milli>(t2 - t1).count();
                // the geometry of each query (both projections, the stop test and
                // the next weight vector) on host threads: queries share nothing
                parallel_for(K, [&](int kk) {
                    QState& s = qs[act[kk]];
                    s.backups += st.backups / K;
                    s.ms += ms / K;
                    std::vector<double> r(R.begin() + (size_t)kk * d, R.begin() + (size_t)(kk + 1) * d);
                    std::vector<double> w(W.begin() + (size_t)kk * d, W.begin() + (size_t)(kk + 1) * d);
                    s.Phi.push_back(r);
                    s.Ws.push_back(w);
                    s.Fs.emplace_back(A.begin() + (size_t)kk * nJ, A.begin() + (size_t)(kk + 1) * nJ);
                    double wr = 0, wt = 0;
                    for (int k = 0; k < d; ++k) {
                        wr += w[k] * r[k];
                        wt += w[k] * s.t_down[k];
                    }
                    const int n = (int)s.Phi.size();
                    std::vector<double> Pf((size_t)n * d), Wf((size_t)n * d);
                    for (int i = 0; i < n; ++i)
                        for (int k = 0; k < d; ++k) {
                            Pf[(size_t)i * d + k] = s.Phi[i][k];
                            Wf[(size_t)i * d + k] = s.Ws[i][k];
                        }
                    if (wr < wt) {
                        if (o.verification_only) s.separated = true;
                        project_outer(Wf.data(), Pf.data(), n, d, s.t.data(), M, s.t_down.data());
                    }
                    s.lam.assign(n, 0.0);
                    project_inner(Pf.data(), n, d, s.t.data(), M, s.t_up.data(), s.lam.data());
                    std::vector<double> diff(d);
                    for (int k = 0; k < d; ++k) diff[k] = s.t_down[k] - s.t_up[k];
                    s.gap = mnorm(diff, M);
                    if (s.separated || s.gap <= o.eps) {
                        s.done = true;
                        return;
                    }
                    // w = M (t - t_up) / ||M (t - t_up)||_1.  Components at or
                    // below 1e-12 max(1, ||t||_inf) are rounding noise of the
                    // projection (like negative ones) and become 0: a positive
                    // noise entry would otherwise be the whole objective of the
                    // models it touches.
                    std::vector<double> v(d), mv(d, 0.0);
                    double tmax = 1.0;
                    for (int k = 0; k < d; ++k) {
                        v[k] = s.t[k] - s.t_up[k];
                        tmax = std::max(tmax, std::fabs(s.t[k]));
                    }
                    for (int k = 0; k < d; ++k) {
                        if (!M) mv[k] = v[k];
                        else
                            for (int l = 0; l < d; ++l) mv[k] += M[(size_t)k * d + l] * v[l];
                    }
                    const double floor = 1e-12 * tmax;
                    double sum = 0;
                    for (int k = 0; k < d; ++k) {
                        mv[k] = mv[k] > floor ? mv[k] : 0.0;
                        sum += mv[k];
                    }
                    if (!(sum > 0)) {
                        s.done = true;   // t_up == t up to rounding
                        return;
                    }
                    for (int k = 0; k < d; ++k) s.w[k] = mv[k] / sum;
                });
                last_ms[2] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t2).count();
            }
            if (learned && o.proposer_passes > 1) propose_later(c, qs, act, d, o.proposer_passes);
            const double now = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
            for (int q : act)
                if (qs[q].done && qs[q].latency_ms < 0) qs[q].latency_ms = now;
        }
    }
    const double total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    for (int q = 0; q < Q; ++q) {
        QState& s = qs[q];
        morap_query_result& r = res[q];
        std::vector<double> diff(d);
        for (int k = 0; k < d; ++k) diff[k] = s.t[k] - s.t_up[k];
        int verdict = MORAP_UNDECIDED;
        if (mnorm(diff, M) <= 1e-9) {
            verdict = MORAP_FEASIBLE;
        } else {
            for (size_t i = 0; i < s.Phi.size(); ++i) {
                double wr = 0, wt = 0;
                for (int k = 0; k < d; ++k) {
                    wr += s.Ws[i][k] * s.Phi[i][k];
                    wt += s.Ws[i][k] * s.t[k];
                }
                if (wr < wt - 1e-12) verdict = MORAP_INFEASIBLE;
            }
        }
        r.verdict = verdict;
        r.iterations = (int32_t)s.Phi.size();
        r.fallback = s.fallback;
        r.gap = s.gap;
        r.ms = Q == 1 ? total_ms : s.ms;
        r.latency_ms = s.latency_ms < 0 ? total_ms : s.latency_ms;
        r.backups = s.backups;
        if (r.t_up) std::copy(s.t_up.begin(), s.t_up.end(), r.t_up);
        if (r.t_down) std::copy(s.t_down.begin(), s.t_down.end(), r.t_down);
        if (r.lam) {
            std::fill(r.lam, r.lam + o.max_iter, 0.0);
            std::copy(s.lam.begin(), s.lam.end(), r.lam);
        }
        if (o.keep_trace) {
            for (size_t i = 0; i < s.Phi.size(); ++i) {
                if (r.trace_w) std::copy(s.Ws[i].begin(), s.Ws[i].end(), r.trace_w + i * d);
                if (r.trace_r) std::copy(s.Phi[i].begin(), s.Phi[i].end(), r.trace_r + i * d);
                if (r.trace_f) std::copy(s.Fs[i].begin(), s.Fs[i].end(), r.trace_f + i * nJ);
            }
        }
    }
}

}  // namespace morap

extern "C" int morap_proposer_target(const double* t, const double* t_down, const double* w_last, int d,
                                     const double* M, double* w_out) {
    if (!t || !t_down || !w_last || !w_out || d < 1) return MORAP_E_INVALID;
    for (int k = 0; k < d; ++k)
        if (!std::isfinite(t[k]) || !std::isfinite(t_down[k]) || !std::isfinite(w_last[k])) return MORAP_E_INVALID;
    if (M)
        for (int64_t k = 0; k < (int64_t)d * d; ++k)
            if (!std::isfinite(M[k])) return MORAP_E_INVALID;
    std::vector<double> diff(d), w(d);
    double dmax = 0;
    for (int k = 0; k < d; ++k) {
        diff[k] = t[k] - t_down[k];
        dmax = std::max(dmax, std::fabs(diff[k]));
    }
    if (dmax > 1e-9) {
        for (int k = 0; k < d; ++k) {
            double v = 0;
            if (!M) v = diff[k];
            else
                for (int l = 0; l < d; ++l) v += M[(size_t)k * d + l] * diff[l];
            w[k] = v;
        }
    } else {
        w.assign(w_last, w_last + d);
    }
    double sum = 0;
    for (int k = 0; k < d; ++k) {
        w[k] = std::max(w[k], 0.0);
        sum += w[k];
    }
    for (int k = 0; k < d; ++k) w_out[k] = sum > 0 ? w[k] / sum : 1.0 / d;
    return MORAP_OK;
}
