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

// Minimum-cost perfect matching of a square n x n matrix by shortest
// augmenting paths with row / column potentials.  Returns match[row] = col.
static std::vector<int> min_cost_matching(const std::vector<double>& cost, int n) {
    const double INF = std::numeric_limits<double>::infinity();
    std::vector<double> u(n + 1, 0.0), v(n + 1, 0.0);
    std::vector<int> p(n + 1, 0), way(n + 1, 0);   // p[col] = row matched to col (1-based)
    for (int i = 1; i <= n; ++i) {
        p[0] = i;
        int j0 = 0;
        std::vector<double> minv(n + 1, INF);
        std::vector<char> used(n + 1, 0);
        do {
            used[j0] = 1;
            const int i0 = p[j0];
            double delta = INF;
            int j1 = 0;
            for (int j = 1; j <= n; ++j) {
                if (used[j]) continue;
                const double cur = cost[(size_t)(i0 - 1) * n + (j - 1)] - u[i0] - v[j];
                if (cur < minv[j]) {
                    minv[j] = cur;
                    way[j] = j0;
                }
                if (minv[j] < delta) {
                    delta = minv[j];
                    j1 = j;
                }
            }
            for (int j = 0; j <= n; ++j) {
                if (used[j]) {
                    u[p[j]] += delta;
                    v[j] -= delta;
                } else {
                    minv[j] -= delta;
                }
            }
            j0 = j1;
        } while (p[j0] != 0);
        do {
            const int j1 = way[j0];
            p[j0] = p[j1];
            j0 = j1;
        } while (j0);
    }
    std::vector<int> match(n, -1);
    for (int j = 1; j <= n; ++j)
        if (p[j] > 0) match[p[j] - 1] = j - 1;
    return match;
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
            const double* ck = c + (size_t)k * nI * nJ;
            for (int r = 0; r < n; ++r) {
                const int i = r / cap;
                for (int j = 0; j < n; ++j) cost[(size_t)r * n + j] = j < nJ ? -ck[(size_t)i * nJ + j] : 0.0;
            }
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

}  // namespace morap
