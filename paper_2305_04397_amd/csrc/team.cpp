// The team MDP of the decentralised model (Sec. 3.1, Def. teamMDP) for n
// agents and n tasks, built on the host: scalarised for one weight vector (a
// single-objective model for the device's CSR sweep), or with its d = 2n
// objectives (the two rewards of every row and the objective each belongs
// to) for the team mode of the library.
//
// A state is (agent i, task j, agent state s, task location q, committed set
// U), numbered with U fastest, then q, s, j, i.  Rows, in this order:
//   * agent i committed and task j not done at q: agent i's enabled actions,
//     moving (s, q) as in the product; reward w_i * (-cost) + w_{n+j} * (mass
//     entering acceptance in this step);
//   * task j at its start (s = s0 of agent i, q = q0) and agent i not
//     committed: commit agent i (b1), then hand task j to the next
//     uncommitted agent after i if there is one (b2), both reward 0;
//   * agent i committed and task j done (accepted or trapped), j < n - 1: the
//     first uncommitted agent starts task j + 1 (b3), reward 0;
//   * a state with none of these gets one empty row (all mass to done,
//     reward 0), so its value is 0.
// The state count is n * n * (sum of agent states x locations) * 2^n: small
// instances only, as a reference for Alg. 2 (Lemma lem:ct-mdp-prop).
#include <cmath>

#include "common.h"

namespace morap {

// The team MDP with the two rewards of every row and the objective each one
// belongs to: rew[r] = (-cost, mass entering acceptance), obj[r] = (i, n + j)
// for agent i acting on task j (switch and empty rows: rewards 0, objectives
// (0, n)).  w (nullable) scalarises instead: rew[r] = (w . objective vector, 0).
static void team_build(const morap_agent* agents, int n_agents, const morap_dfa* tasks, int n_tasks,
                       const int32_t* const* letters, const double* w, int32_t* sizes, int32_t* state_row,
                       int32_t* row_ptr, int32_t* col, double* prob, double* rew, int32_t* obj,
                       uint8_t* to_done) {
    const int n = n_agents;
    MORAP_CHECK(agents && tasks && letters && sizes && n >= 1 && n <= 16 && n_tasks == n, MORAP_E_INVALID,
                "bad arguments (1 <= agents = tasks <= 16)");
    for (int i = 0; i < n; ++i) check_agent(agents[i], i);
    for (int j = 0; j < n; ++j) check_dfa(tasks[j], j);
    if (w)
        for (int q = 0; q < 2 * n; ++q) MORAP_CHECK(std::isfinite(w[q]), MORAP_E_INVALID, "non-finite weight");
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            const int32_t* l = letters[(size_t)i * n + j];
            MORAP_CHECK(l != nullptr, MORAP_E_INVALID, "NULL letters");
            for (int s = 0; s < agents[i].n_states; ++s)
                MORAP_CHECK(l[s] >= 0 && l[s] < tasks[j].n_letters, MORAP_E_INVALID, "letter out of range");
        }
    const int64_t U = int64_t(1) << n;
    std::vector<int64_t> base((size_t)n * n + 1, 0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            base[(size_t)i * n + j + 1] = base[(size_t)i * n + j] + (int64_t)agents[i].n_states * tasks[j].n_locs * U;
    const int64_t S = base.back();
    MORAP_CHECK(S < 0x7fffffff / 32, MORAP_E_UNSUPPORTED, "team MDP too large");
    auto id = [&](int i, int j, int s, int q, int64_t used) -> int32_t {
        return (int32_t)(base[(size_t)i * n + j] + ((int64_t)s * tasks[j].n_locs + q) * U + used);
    };
    std::vector<std::vector<uint8_t>> done(n);
    for (int j = 0; j < n; ++j) done[j] = dfa_done(tasks[j]);

    std::vector<int32_t> sr{0}, rp{0}, cl, ob;
    std::vector<double> pr, rw;
    // a row with cost reward rc for agent oc and probability reward rq for
    // objective oq
    auto end_row = [&](double rc, double rq, int32_t oc, int32_t oq) {
        rp.push_back((int32_t)cl.size());
        rw.push_back(rc);
        rw.push_back(rq);
        ob.push_back(oc);
        ob.push_back(oq);
    };
    auto jump = [&](int32_t target) {
        cl.push_back(target);
        pr.push_back(1.0);
        end_row(0.0, 0.0, 0, n);
    };
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            const morap_agent& ag = agents[i];
            const morap_dfa& tk = tasks[j];
            const int32_t* let = letters[(size_t)i * n + j];
            for (int s = 0; s < ag.n_states; ++s)
                for (int q = 0; q < tk.n_locs; ++q)
                    for (int64_t used = 0; used < U; ++used) {
                        const bool mine = (used >> i) & 1;
                        const size_t rows_before = rp.size();
                        if (mine && !done[j][q]) {
                            for (int a = 0; a < ag.n_actions; ++a) {
                                const int64_t r = (int64_t)s * ag.n_actions + a;
                                const int32_t lo = ag.sa_ptr[r], hi = ag.sa_ptr[r + 1];
                                if (hi == lo) continue;
                                double mass = 0.0;
                                for (int32_t e = lo; e < hi; ++e) {
                                    const int s2 = ag.succ[e];
                                    const int q2 = tk.delta[(int64_t)q * tk.n_letters + let[s2]];
                                    if (tk.accepting[q2] && !tk.accepting[q]) mass += ag.prob[e];
                                    cl.push_back(id(i, j, s2, q2, used));
                                    pr.push_back(ag.prob[e]);
                                }
                                end_row(-ag.cost[r], mass, i, n + j);
                            }
                        }
                        if (s == ag.init && q == tk.q0 && !mine) {
                            jump(id(i, j, s, q, used | (int64_t(1) << i)));                        // b1
                            int k = i + 1;
                            while (k < n && ((used >> k) & 1)) ++k;
                            if (k < n) jump(id(k, j, agents[k].init, q, used));                   // b2
                        }
                        if (mine && done[j][q] && j + 1 < n) {
                            int k = 0;
                            while (k < n && ((used >> k) & 1)) ++k;
                            if (k < n) jump(id(k, j + 1, agents[k].init, tasks[j + 1].q0, used)); // b3
                        }
                        if (rp.size() == rows_before) end_row(0.0, 0.0, 0, n);
                        sr.push_back((int32_t)rp.size() - 1);
                    }
        }
    MORAP_CHECK(rp.size() < 0x7fffffff && cl.size() < 0x7fffffff, MORAP_E_UNSUPPORTED, "team MDP too large");
    const int32_t R = (int32_t)rp.size() - 1, N = (int32_t)cl.size();
    sizes[0] = (int32_t)S;
    sizes[1] = R;
    sizes[2] = N;
    sizes[3] = id(0, 0, agents[0].init, tasks[0].q0, 0);
    if (state_row) std::copy(sr.begin(), sr.end(), state_row);
    if (row_ptr) std::copy(rp.begin(), rp.end(), row_ptr);
    if (col) std::copy(cl.begin(), cl.end(), col);
    if (prob) std::copy(pr.begin(), pr.end(), prob);
    if (rew)
        for (int32_t r = 0; r < R; ++r) {
            if (w) {
                // the objective vector of the row, dotted with w
                rew[2 * (size_t)r] = w[ob[2 * (size_t)r]] * rw[2 * (size_t)r] +
                                     w[ob[2 * (size_t)r + 1]] * rw[2 * (size_t)r + 1];
                rew[2 * (size_t)r + 1] = 0.0;
            } else {
                rew[2 * (size_t)r] = rw[2 * (size_t)r];
                rew[2 * (size_t)r + 1] = rw[2 * (size_t)r + 1];
            }
        }
    if (obj) std::copy(ob.begin(), ob.end(), obj);
    if (to_done)
        for (int32_t r = 0; r < R; ++r) {
            double sum = 0.0;
            for (int32_t e = rp[r]; e < rp[r + 1]; ++e) sum += pr[e];
            to_done[r] = sum < 1.0 - 1e-12 ? 1 : 0;
        }
}

void team_model_host(const morap_agent* agents, int n_agents, const morap_dfa* tasks, int n_tasks,
                     const int32_t* const* letters, const double* w, int32_t* sizes, int32_t* state_row,
                     int32_t* row_ptr, int32_t* col, double* prob, double* rew, uint8_t* to_done) {
    MORAP_CHECK(w, MORAP_E_INVALID, "NULL weights");
    team_build(agents, n_agents, tasks, n_tasks, letters, w, sizes, state_row, row_ptr, col, prob, rew, nullptr,
               to_done);
}

void team_model_mo_host(const morap_agent* agents, int n_agents, const morap_dfa* tasks, int n_tasks,
                        const int32_t* const* letters, int32_t* sizes, int32_t* state_row, int32_t* row_ptr,
                        int32_t* col, double* prob, double* rew, int32_t* obj, uint8_t* to_done) {
    team_build(agents, n_agents, tasks, n_tasks, letters, nullptr, sizes, state_row, row_ptr, col, prob, rew, obj,
               to_done);
}

}  // namespace morap
