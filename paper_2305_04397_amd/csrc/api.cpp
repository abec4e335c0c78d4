// extern "C" entry points of libmorap (declared in include/morap.h): argument
// checks, device selection, and translation of internal errors into return
// codes.  No C++ exception leaves this file.
#include "common.h"

#include <algorithm>
#include <cmath>

using namespace morap;

namespace morap {
thread_local AllocMeter* g_meter = nullptr;
}

morap_ctx::~morap_ctx() {
    for (int g = 0; g < 3; ++g) {
        if (chunk_exec[g]) (void)hipGraphExecDestroy(chunk_exec[g]);
        if (chunk_graph[g]) (void)hipGraphDestroy(chunk_graph[g]);
    }
    for (hipEvent_t e : event_pool) (void)hipEventDestroy(e);
    if (prop_mlp) proposer_destroy(prop_mlp);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
}

namespace {

void to_abi(const Stats& s, morap_stats* out) {
    if (!out) return;
    out->backups = s.backups;
    out->sweeps = s.sweeps;
    out->max_pair_sweeps = s.max_pair_sweeps;
    out->eval_sweeps = s.eval_sweeps;
    out->polish_sweeps = s.polish_sweeps;
    out->rank_rounds = s.rank_rounds;
    out->floor_stops = s.floor_stops;
    out->bytes = s.bytes;
    out->ms_vi = s.ms_vi;
    out->ms_eval = s.ms_eval;
    out->ms_total = s.ms_total;
    out->ms_sweep_kernel = s.ms_sweep_kernel;
    out->sweep_launches = s.sweep_launches;
    out->bytes_refine = s.bytes_refine;
    out->ms_sweep_kernel_refine = s.ms_sweep_kernel_refine;
    out->sweep_launches_refine = s.sweep_launches_refine;
    out->variant = s.variant;
    out->variant_refine = s.variant_refine;
    out->sweeps_tail = s.sweeps_tail;
    out->sweep_launches_tail = s.sweep_launches_tail;
    out->bytes_tail = s.bytes_tail;
    out->ms_sweep_kernel_tail = s.ms_sweep_kernel_tail;
    out->variant_tail = s.variant_tail;
    out->reserved = 0;
    out->refine_pairs = s.refine_pairs;
    out->refine_columns = s.refine_columns;
}

}  // namespace

extern "C" {

int morap_create(morap_ctx** out, int device, void* hip_stream) {
    if (!out) return MORAP_E_INVALID;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return MORAP_E_INVALID;
    morap_ctx* c = nullptr;
    try {
        c = new morap_ctx();
    } catch (...) {
        return MORAP_E_OOM;
    }
    c->device = device;
    const int rc = guarded(c, [&] {
        MORAP_HIP(hipGetDeviceProperties(&c->prop, device));
        proposer_scratch_init(device);   // the allocation-free inference's scratch address
        if (hip_stream) {
            c->stream = static_cast<hipStream_t>(hip_stream);
        } else {
            // a stream of our own (default priority) so sweep chunks can be
            // captured into graphs
            MORAP_HIP(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
            c->own_stream = true;
        }
    });
    if (rc != MORAP_OK) {
        delete c;
        return rc;
    }
    *out = c;
    return MORAP_OK;
}

int morap_set_memory_budget(morap_ctx* ctx, int64_t bytes, int64_t* used_out) {
    return guarded(ctx, [&] {
        MORAP_CHECK(bytes >= 0, MORAP_E_INVALID, "the budget must be >= 0 (0 = none)");
        ctx->meter.budget = bytes;
        if (used_out) *used_out = ctx->meter.used;
    });
}

int morap_destroy(morap_ctx* ctx) {
    if (!ctx) return MORAP_OK;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    delete ctx;
    return MORAP_OK;
}

const char* morap_last_error(const morap_ctx* ctx) { return ctx ? ctx->err.c_str() : "no context"; }

int morap_build_products(morap_ctx* ctx, const morap_agent* agents, int n_agents, const morap_dfa* tasks,
                         int n_tasks, const int32_t* const* letters) {
    return guarded(ctx, [&] { build_products(ctx, agents, n_agents, tasks, n_tasks, letters); });
}

int morap_load_models(morap_ctx* ctx, const morap_model* models, int n_models, int n_agents, int n_tasks) {
    return guarded(ctx, [&] { load_models(ctx, models, n_models, n_agents, n_tasks); });
}

int morap_model_info(const morap_ctx* cctx, int m, int32_t* sizes) {
    morap_ctx* ctx = const_cast<morap_ctx*>(cctx);
    return guarded(ctx, [&] {
        MORAP_CHECK(ctx->loaded, MORAP_E_STATE, "no models loaded");
        MORAP_CHECK(sizes && m >= 0 && m < ctx->hm.M, MORAP_E_INVALID, "model index out of range");
        const auto& h = ctx->hm;
        const int32_t s0 = h.state_base[m], s1 = h.state_base[m + 1];
        sizes[0] = s1 - s0;
        sizes[1] = h.state_row[s1] - h.state_row[s0];
        sizes[2] = h.row_ptr[h.state_row[s1]] - h.row_ptr[h.state_row[s0]];
        sizes[3] = h.init[m] >= 0 ? h.init[m] - s0 : -1;
        sizes[4] = (int32_t)ctx->S;
    });
}

int morap_get_model(const morap_ctx* cctx, int m, int32_t* state_row, int32_t* row_ptr, int32_t* col, double* prob,
                    double* rew, uint8_t* to_done, int32_t* states) {
    morap_ctx* ctx = const_cast<morap_ctx*>(cctx);
    return guarded(ctx, [&] {
        MORAP_CHECK(ctx->loaded, MORAP_E_STATE, "no models loaded");
        MORAP_CHECK(m >= 0 && m < ctx->hm.M, MORAP_E_INVALID, "model index out of range");
        const auto& h = ctx->hm;
        const int32_t s0 = h.state_base[m], s1 = h.state_base[m + 1];
        const int32_t r0 = h.state_row[s0], r1 = h.state_row[s1];
        const int32_t e0 = h.row_ptr[r0], e1 = h.row_ptr[r1];
        if (state_row)
            for (int32_t s = s0; s <= s1; ++s) state_row[s - s0] = h.state_row[s] - r0;
        if (row_ptr)
            for (int32_t r = r0; r <= r1; ++r) row_ptr[r - r0] = h.row_ptr[r] - e0;
        if (col)
            for (int32_t e = e0; e < e1; ++e) col[e - e0] = h.col[e] - s0;
        if (prob) std::copy(h.prob.begin() + e0, h.prob.begin() + e1, prob);
        if (rew) std::copy(h.rew.begin() + 2 * (size_t)r0, h.rew.begin() + 2 * (size_t)r1, rew);
        if (to_done) std::copy(h.to_done.begin() + r0, h.to_done.begin() + r1, to_done);
        if (states) std::copy(h.states_sq.begin() + 2 * (size_t)s0, h.states_sq.begin() + 2 * (size_t)s1, states);
    });
}

void morap_default_opts(morap_vi_opts* o) {
    if (!o) return;
    o->eps_vi = 1e-6;
    o->eps_eval = 1e-6;
    o->tau = 1e-9;
    o->precision = MORAP_F32;
    o->max_sweeps = 1000000;
    o->check_every = 32;
    o->schedule = 0;
    o->use_graph = 1;
    o->time_kernels = 0;
    o->eval_start = 0;
}

int morap_solve(morap_ctx* ctx, const double* W, int K, const morap_vi_opts* opts, double* c_out,
                morap_stats* stats) {
    return guarded(ctx, [&] {
        MORAP_CHECK(opts, MORAP_E_INVALID, "opts is NULL");
        Stats st;
        solve(ctx, W, K, *opts, c_out, st);
        to_abi(st, stats);
    });
}

int morap_solve_staged(morap_ctx* ctx, const double* W, int K, const morap_vi_opts* opts, double* c_out,
                       morap_stats* stats) {
    return guarded(ctx, [&] {
        MORAP_CHECK(opts, MORAP_E_INVALID, "opts is NULL");
        Stats st;
        solve_staged(ctx, W, K, *opts, c_out, st);
        to_abi(st, stats);
    });
}

int morap_evaluate(morap_ctx* ctx, const int32_t* assign, int K, const morap_vi_opts* opts, double* r_out,
                   morap_stats* stats) {
    return guarded(ctx, [&] {
        MORAP_CHECK(opts, MORAP_E_INVALID, "opts is NULL");
        Stats st;
        evaluate(ctx, assign, K, *opts, r_out, st);
        to_abi(st, stats);
    });
}

int morap_assign(morap_ctx* ctx, const double* c, int K, int32_t* assign_out) {
    return guarded(ctx, [&] {
        MORAP_CHECK(ctx->loaded, MORAP_E_STATE, "no models loaded");
        assign_columns(ctx->hm.nI, ctx->hm.nJ, c, K, assign_out);
    });
}

int morap_product_host(const morap_agent* agent, const morap_dfa* task, const int32_t* letters,
                       int32_t* sizes_out, int32_t* state_row, int32_t* row_ptr, int32_t* col, double* prob,
                       double* rew, uint8_t* to_done, int32_t* states) {
    try {
        product_host(agent, task, letters, sizes_out, state_row, row_ptr, col, prob, rew, to_done, states);
        return MORAP_OK;
    } catch (const MorapError& e) {
        return e.code;
    } catch (...) {
        return MORAP_E_OOM;
    }
}

int morap_team_model_host(const morap_agent* agents, int n_agents, const morap_dfa* tasks, int n_tasks,
                          const int32_t* const* letters, const double* w, int32_t* sizes_out, int32_t* state_row,
                          int32_t* row_ptr, int32_t* col, double* prob, double* rew, uint8_t* to_done) {
    try {
        team_model_host(agents, n_agents, tasks, n_tasks, letters, w, sizes_out, state_row, row_ptr, col, prob, rew,
                        to_done);
        return MORAP_OK;
    } catch (const MorapError& e) {
        return e.code;
    } catch (...) {
        return MORAP_E_OOM;
    }
}

int morap_team_model_mo_host(const morap_agent* agents, int n_agents, const morap_dfa* tasks, int n_tasks,
                             const int32_t* const* letters, int32_t* sizes_out, int32_t* state_row,
                             int32_t* row_ptr, int32_t* col, double* prob, double* rew, int32_t* obj,
                             uint8_t* to_done) {
    try {
        team_model_mo_host(agents, n_agents, tasks, n_tasks, letters, sizes_out, state_row, row_ptr, col, prob, rew,
                           obj, to_done);
        return MORAP_OK;
    } catch (const MorapError& e) {
        return e.code;
    } catch (...) {
        return MORAP_E_OOM;
    }
}

int morap_load_team_model(morap_ctx* ctx, int n_agents, int n_tasks, const morap_model* model, const int32_t* obj) {
    return guarded(ctx, [&] { load_team_model(ctx, n_agents, n_tasks, model, obj); });
}

int morap_assign_host(const double* c, int n_agents, int n_tasks, int K, int32_t* assign_out) {
    try {
        assign_columns(n_agents, n_tasks, c, K, assign_out);
        return MORAP_OK;
    } catch (const MorapError& e) {
        return e.code;
    } catch (...) {
        return MORAP_E_INVALID;
    }
}

int morap_support(morap_ctx* ctx, const double* W, int K, const morap_vi_opts* opts, double* r_out,
                  int32_t* assign_out, double* c_out, morap_stats* stats) {
    return guarded(ctx, [&] {
        MORAP_CHECK(opts && r_out, MORAP_E_INVALID, "opts / r_out is NULL");
        MORAP_CHECK(ctx->loaded, MORAP_E_STATE, "no models loaded");
        const int nI = ctx->hm.nI, nJ = ctx->hm.nJ;
        std::vector<double> C((size_t)std::max(K, 1) * nI * nJ);
        std::vector<int32_t> A((size_t)std::max(K, 1) * nJ);
        Stats st;
        solve(ctx, W, K, *opts, C.data(), st);
        // a team model's policy does the assignment itself: no assignment step
        if (!ctx->team) assign_columns(nI, nJ, C.data(), K, A.data());
        // after an FP32 solve the assignment is checked on FP64 values
        std::vector<int32_t> F(A);
        evaluate(ctx, A.data(), K, *opts, r_out, st, nullptr, ctx->team ? nullptr : F.data());
        if (!ctx->team) A = F;
        if (assign_out && ctx->team) std::fill(assign_out, assign_out + (size_t)K * n_tasks_of(ctx), 0);
        else if (assign_out) std::copy(A.begin(), A.begin() + (size_t)K * nJ, assign_out);
        if (c_out) std::copy(C.begin(), C.begin() + (size_t)K * nI * nJ, c_out);
        to_abi(st, stats);
    });
}

// Synthesis after Alg. 1 (Sec. 3.3): re-solve the weight vectors of the
// passes with v > 0 and evaluate exactly their recorded assignments.
int morap_synthesize(morap_ctx* ctx, const double* W, const int32_t* F, const double* v, int n,
                     const morap_vi_opts* opts, int32_t* n_picked, int32_t* picked_out, double* r_out,
                     double* matrix_out) {
    return guarded(ctx, [&] {
        MORAP_CHECK(W && F && v && opts && n_picked && picked_out && r_out && n >= 1, MORAP_E_INVALID,
                    "bad synthesis arguments");
        MORAP_CHECK(ctx->loaded, MORAP_E_STATE, "no models loaded");
        MORAP_CHECK(!ctx->team, MORAP_E_UNSUPPORTED, "synthesis needs the decentralised products");
        const int nI = ctx->hm.nI, nJ = ctx->hm.nJ, d = nI + nJ;
        std::vector<int32_t> pick;
        double vsum = 0;
        for (int i = 0; i < n; ++i) {
            MORAP_CHECK(std::isfinite(v[i]) && v[i] >= 0, MORAP_E_INVALID, "v must be finite and >= 0");
            if (v[i] > 0) {
                pick.push_back(i);
                vsum += v[i];
            }
        }
        MORAP_CHECK(!pick.empty(), MORAP_E_INVALID, "no pass has v > 0");
        const int m = (int)pick.size();
        std::vector<double> Wp((size_t)m * d), C((size_t)m * nI * nJ);
        std::vector<int32_t> Fp((size_t)m * nJ);
        for (int q = 0; q < m; ++q) {
            std::copy(W + (size_t)pick[q] * d, W + (size_t)(pick[q] + 1) * d, &Wp[(size_t)q * d]);
            for (int j = 0; j < nJ; ++j) {
                const int32_t a = F[(size_t)pick[q] * nJ + j];
                MORAP_CHECK(a >= 0 && a < nI, MORAP_E_INVALID, "assignment entry out of range");
                Fp[(size_t)q * nJ + j] = a;
            }
        }
        Stats st;
        solve(ctx, Wp.data(), m, *opts, C.data(), st);
        evaluate(ctx, Fp.data(), m, *opts, r_out, st);
        if (matrix_out) {
            std::fill(matrix_out, matrix_out + (size_t)nI * nJ, 0.0);
            for (int q = 0; q < m; ++q)
                for (int j = 0; j < nJ; ++j)
                    matrix_out[(size_t)Fp[(size_t)q * nJ + j] * nJ + j] += v[pick[q]] / vsum;
        }
        std::copy(pick.begin(), pick.end(), picked_out);
        *n_picked = m;
    });
}

int morap_get_stats(const morap_ctx* cctx, morap_stats* out) {
    morap_ctx* ctx = const_cast<morap_ctx*>(cctx);
    return guarded(ctx, [&] {
        MORAP_CHECK(out, MORAP_E_INVALID, "out is NULL");
        to_abi(ctx->cum, out);
    });
}

int morap_reset_stats(morap_ctx* ctx) {
    return guarded(ctx, [&] { ctx->cum = Stats(); });
}

int morap_get_policy(const morap_ctx* cctx, int k, int j, int8_t* mu_out) {
    morap_ctx* ctx = const_cast<morap_ctx*>(cctx);
    return guarded(ctx, [&] {
        MORAP_CHECK(ctx->evaluated, MORAP_E_STATE, "no morap_evaluate yet");
        // a team model: one policy per column (j = 0), held by each of the
        // column's (d + 1) / 2 evaluation instances
        const int per_col = ctx->team ? (n_obj_of(ctx) + 1) / 2 : ctx->hm.nJ;
        MORAP_CHECK(mu_out && k >= 0 && k < ctx->eK && j >= 0 && j < ctx->hm.nJ, MORAP_E_INVALID,
                    "index out of range");
        const int q = k * per_col + j;
        const int64_t b = ctx->inst_base[q], e = ctx->inst_base[q + 1];
        if (e > b)
            MORAP_HIP(hipMemcpy(mu_out, ctx->d_mu.as<int8_t>() + b, (size_t)(e - b), hipMemcpyDeviceToHost));
    });
}

int morap_get_values(const morap_ctx* cctx, int k, int m, double* x_out) {
    morap_ctx* ctx = const_cast<morap_ctx*>(cctx);
    return guarded(ctx, [&] {
        MORAP_CHECK(ctx->solved, MORAP_E_STATE, "no morap_solve yet");
        MORAP_CHECK(x_out && k >= 0 && k < ctx->K && m >= 0 && m < ctx->hm.M, MORAP_E_INVALID,
                    "index out of range");
        const int32_t s0 = ctx->hm.state_base[m], s1 = ctx->hm.state_base[m + 1];
        const int Kp = ctx->Kp;
        uint8_t par = 0;
        MORAP_HIP(hipMemcpy(&par, ctx->vmain.final_par.as<uint8_t>() + (size_t)m * Kp + k, 1,
                            hipMemcpyDeviceToHost));
        const size_t el = ctx->prec == MORAP_F32 ? 4 : 8;
        std::vector<char> buf((size_t)(s1 - s0) * Kp * el + 8);
        if (s1 > s0)
            MORAP_HIP(hipMemcpy(buf.data(), ctx->vmain.x[par].as<char>() + (size_t)s0 * Kp * el,
                                (size_t)(s1 - s0) * Kp * el, hipMemcpyDeviceToHost));
        for (int32_t s = 0; s < s1 - s0; ++s) {
            if (el == 4) x_out[s] = reinterpret_cast<const float*>(buf.data())[(size_t)s * Kp + k];
            else x_out[s] = reinterpret_cast<const double*>(buf.data())[(size_t)s * Kp + k];
        }
    });
}

int morap_query(morap_ctx* ctx, const double* t, const double* M, const morap_query_opts* opts,
                morap_query_result* result) {
    return guarded(ctx, [&] {
        MORAP_CHECK(opts, MORAP_E_INVALID, "opts is NULL");
        query_batch(ctx, t, nullptr, 1, M, *opts, result);
    });
}

int morap_query_batch(morap_ctx* ctx, const double* T, const double* W0, int Q, const double* M,
                      const morap_query_opts* opts, morap_query_result* results) {
    return guarded(ctx, [&] {
        MORAP_CHECK(opts, MORAP_E_INVALID, "opts is NULL");
        query_batch(ctx, T, W0, Q, M, *opts, results);
    });
}

int morap_project_inner(const double* Phi, int m, int d, const double* t, const double* M, double* x_out,
                        double* lam_out) {
    try {
        project_inner(Phi, m, d, t, M, x_out, lam_out);
        return MORAP_OK;
    } catch (const MorapError& e) {
        return e.code;
    } catch (...) {
        return MORAP_E_INVALID;
    }
}

int morap_project_outer(const double* W, const double* R, int n, int d, const double* t, const double* M,
                        double* z_out) {
    try {
        project_outer(W, R, n, d, t, M, z_out);
        return MORAP_OK;
    } catch (const MorapError& e) {
        return e.code;
    } catch (...) {
        return MORAP_E_INVALID;
    }
}

int morap_set_features(morap_ctx* ctx, const double* phi, int n_feat) {
    return guarded(ctx, [&] {
        MORAP_CHECK(n_feat >= 0 && (n_feat == 0 || phi), MORAP_E_INVALID, "bad features");
        for (int i = 0; i < n_feat; ++i) MORAP_CHECK(std::isfinite(phi[i]), MORAP_E_INVALID, "non-finite feature");
        ctx->features.assign(phi, phi + n_feat);
    });
}

}  // extern "C"
