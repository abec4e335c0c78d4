// Assignment step of Alg. 2: for each weight column, the assignment f of
// tasks to agents maximising sum_j c[f(j)][j] (Hungarian method, O(n^3)).
// With more tasks than agents each agent may take ceil(|J|/|I|) tasks: every
// agent row is repeated that many times and missing tasks are zero-value
// dummies, which keeps the problem a square assignment.
#include "common.h"

#include <atomic>
#include <thread>

#include <algorithm>
#include <cmath>
#include <limits>

namespace morap {

// Minimum-cost perfect matching of a square n x n matrix (Kuhn-Munkres in
// its successive-shortest-path form).  Dual potentials u (rows) and v
// (columns) keep every reduced cost c(i,j) - u(i) - v(j) >= 0 and those of
// matched pairs at 0.  Each row in turn is matched by a Dijkstra search over
// alternating paths (a column leads on to the row matched to it at reduced
// cost 0) until a free column is reached at distance D; the potentials of
// the columns settled on the way, and of their rows, move by D minus their
// distance (which keeps the reduced costs >= 0 and zeroes them along the
// path), and the path is flipped.  Returns col_of_row; u_out / v_out
// (nullable) receive the final potentials.
static std::vector<int> min_cost_matching(const std::vector<double>& cost, int n, std::vector<double>* u_out = nullptr,
                                          std::vector<double>* v_out = nullptr) {
    const double INF = std::numeric_limits<double>::infinity();
    std::vector<double> u(n, 0.0), v(n, 0.0), dist(n);
    std::vector<int> row_of_col(n, -1), col_of_row(n, -1), pred_row(n), settled;
    std::vector<char> done(n);
    settled.reserve(n);
    auto reduced = [&](int i, int j) { return cost[(size_t)i * n + j] - u[i] - v[j]; };
    for (int r = 0; r < n; ++r) {
        for (int j = 0; j < n; ++j) {
            dist[j] = reduced(r, j);
            pred_row[j] = r;
            done[j] = 0;
        }
        settled.clear();
        int sink = -1;
        while (sink < 0) {
            int j = -1;
            double best = INF;
            for (int k = 0; k < n; ++k)
                if (!done[k] && (j < 0 || dist[k] < best)) {
                    best = dist[k];
                    j = k;
                }
            done[j] = 1;
            if (row_of_col[j] < 0) {
                sink = j;
                break;
            }
            settled.push_back(j);
            const int i = row_of_col[j];
            for (int k = 0; k < n; ++k) {
                if (done[k]) continue;
                const double via = dist[j] + reduced(i, k);
                if (via < dist[k]) {
                    dist[k] = via;
                    pred_row[k] = i;
                }
            }
        }
        const double D = dist[sink];
        for (int j : settled) {
            const double shift = D - dist[j];
            v[j] -= shift;
            u[row_of_col[j]] += shift;
        }
        u[r] += D;
        for (int k = sink;;) {
            const int i = pred_row[k];
            const int prev = col_of_row[i];
            row_of_col[k] = i;
            col_of_row[i] = k;
            if (i == r) break;
            k = prev;
        }
    }
    if (u_out) *u_out = u;
    if (v_out) *v_out = v;
    return col_of_row;
}

// The replicated square problem of one column (every agent row repeated
// ceil(|J|/|I|) times, zero-value dummy tasks), as costs -c.
static void column_costs(int nI, int nJ, int cap, const double* ck, std::vector<double>& cost) {
    const int n = nI * cap;
    cost.assign((size_t)n * n, 0.0);
    for (int r = 0; r < n; ++r) {
        const int i = r / cap;
        for (int j = 0; j < nJ; ++j) cost[(size_t)r * n + j] = -ck[(size_t)i * nJ + j];
    }
}

void assign_columns(int nI, int nJ, const double* c, int K, int32_t* out) {
    MORAP_CHECK(nI > 0 && nJ > 0 && c && out && K > 0, MORAP_E_INVALID, "bad assignment arguments");
    for (int64_t q = 0; q < (int64_t)K * nI * nJ; ++q)
        MORAP_CHECK(std::isfinite(c[q]), MORAP_E_INVALID, "non-finite assignment value");
    const int cap = std::max(1, (nJ + nI - 1) / nI);
    const int n = nI * cap;   // >= nJ
    // the K columns are independent: one Hungarian solve per column, spread
    // over host threads
    std::atomic<int> next{0};
    auto worker = [&] {
        std::vector<double> cost((size_t)n * n);
        for (int k; (k = next++) < K;) {
            column_costs(nI, nJ, cap, c + (size_t)k * nI * nJ, cost);
            const auto match = min_cost_matching(cost, n);
            for (int r = 0; r < n; ++r)
                if (match[r] >= 0 && match[r] < nJ) out[(size_t)k * nJ + match[r]] = r / cap;
        }
    };
    const int nt = std::max(1, std::min<int>(K, std::min(16u, std::thread::hardware_concurrency())));
    if (nt == 1 || (int64_t)K * n * n < (int64_t)1 << 16) {
        worker();
        return;
    }
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t) th.emplace_back(worker);
    for (auto& t : th) t.join();
}

// Slack of every (agent, task) pair against an optimal assignment of column
// c[nI][nJ]: with the optimal dual potentials u (agent rows) and v (tasks)
// of the cost form -c, slack(i, j) = min over agent i's rows r of
// -c(i, j) - u(r) - v(j) >= 0, zero on the assigned pairs.  Any other
// assignment's value falls short of the optimum by the sum of its pairs'
// slacks.  Returns the assignment (agent of each task).
std::vector<int32_t> assignment_slack(int nI, int nJ, const double* ck, double* slack) {
    const int cap = std::max(1, (nJ + nI - 1) / nI);
    const int n = nI * cap;
    std::vector<double> cost, u, v;
    column_costs(nI, nJ, cap, ck, cost);
    const auto match = min_cost_matching(cost, n, &u, &v);
    std::vector<int32_t> f(nJ, -1);
    for (int r = 0; r < n; ++r)
        if (match[r] >= 0 && match[r] < nJ) f[match[r]] = r / cap;
    for (int i = 0; i < nI; ++i)
        for (int j = 0; j < nJ; ++j) {
            double best = INFINITY;
            for (int r = i * cap; r < (i + 1) * cap; ++r) best = std::min(best, cost[(size_t)r * n + j] - u[r] - v[j]);
            slack[(size_t)i * nJ + j] = std::max(0.0, best);
        }
    return f;
}

}  // namespace morap
