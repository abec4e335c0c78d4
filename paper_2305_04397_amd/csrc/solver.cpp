// Host orchestration of the batched value iteration (Alg. 3 for K weight
// columns at once), policy extraction and per-objective evaluation (Alg. 4)
// of the assigned (column, model) instances.
//
// Precision: an FP32 solve runs FP32 backups (FP64 residual) over every
// (model, column) pair and yields the values that choose the assignment.  The
// evaluation then repeats the value iteration in FP64 from 0, with the same
// stopping rule, on the assigned pairs only (one pair per task and column);
// policies and per-objective values come from those FP64 values.
#include "common.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <thread>
#include <cmath>
#include <cstdio>
#include <cstdlib>

namespace morap {

// ---------------------------------------------------------------------------
// sweep-kernel variants: kernel family x columns per lane x lanes per state.
// Ids 1-18 are the CSR-tile sweep, 19-36 the same shapes of the
// neighbourhood-block sweep, 37-38 the wave-per-state block sweep with other
// numbers of states in flight, 39-40 the LDS-staged sweep over halo tiles.
// ---------------------------------------------------------------------------
const std::vector<Variant>& variants() {
    static const std::vector<Variant> v = [] {
        std::vector<Variant> out;
        const int pairs[][2] = {{1, 1},  {1, 2},  {2, 1},  {1, 4},  {2, 2},  {4, 1},
                                {1, 8},  {2, 4},  {4, 2},  {1, 16}, {2, 8},  {4, 4},
                                {1, 32}, {2, 16}, {4, 8},  {1, 64}, {2, 32}, {4, 16}};
        int id = 1;
        for (auto& p : pairs) out.push_back({id++, p[0], p[1], std::min(256, 64 * p[1]), SWEEP_CSR, 0});
        for (auto& p : pairs) out.push_back({id++, p[0], p[1], 256, SWEEP_BLOCK, p[1] == 64 ? 4 : 2});
        // the wave-per-state block sweep with 2 and 8 states in flight
        out.push_back({id++, 1, 64, 256, SWEEP_BLOCK, 2});
        out.push_back({id++, 1, 64, 256, SWEEP_BLOCK, 8});
        // the LDS-staged sweep over halo tiles (FP32), 2 and 4 states in flight
        out.push_back({id++, 1, 64, 256, SWEEP_HALO, 2});
        out.push_back({id++, 1, 64, 256, SWEEP_HALO, 4});
        return out;
    }();
    return v;
}

static int kt_of(const Variant& v) { return v.cpl * v.lps; }
static bool uses_halo_tiles(const Variant& v) { return v.kind == SWEEP_HALO; }

static int padded_k(int K) {
    if (K <= 64) {
        int p = 1;
        while (p < K) p <<= 1;
        return std::max(p, 1);
    }
    return (K + 63) / 64 * 64;
}

// candidate variants for a padded width: k-tiles of min(Kp, 64) columns and
// of half that; a restricted solve (few active columns per model) also tries
// narrower k-tiles, which skip the k-tiles without active columns
static std::vector<Variant> candidates(int Kp, bool restricted, bool blocks, bool halo) {
    std::vector<Variant> out;
    const int kt_full = std::min(Kp, 64);
    for (const auto& v : variants()) {
        if (v.kind == SWEEP_BLOCK && !blocks) continue;
        if (v.kind == SWEEP_HALO && !halo) continue;
        const int kt = kt_of(v);
        if (Kp % kt) continue;
        if (kt == kt_full || (kt * 2 == kt_full && kt >= 8) || (restricted && kt >= 8 && kt <= kt_full))
            out.push_back(v);
    }
    return out;
}

static const Variant& variant_by_id(int id) {
    for (const auto& v : variants())
        if (v.id == id) return v;
    fail(MORAP_E_INVALID, "unknown sweep variant id " + std::to_string(id));
}

// ---------------------------------------------------------------------------
// buffers
// ---------------------------------------------------------------------------
static void ensure_scratch(morap_ctx* c, int Kp) {
    const int M = c->hm.M;
    const size_t pairs = (size_t)M * Kp;
    bool moved = false;
    moved |= c->d_wc32.ensure(pairs * 4);
    moved |= c->d_wp32.ensure(pairs * 4);
    moved |= c->d_wc64.ensure(pairs * 8);
    moved |= c->d_wp64.ensure(pairs * 8);
    moved |= c->d_res.ensure(pairs * 8);
    moved |= c->d_ymax.ensure(pairs * 8);
    moved |= c->d_active.ensure(pairs);
    moved |= c->d_pair_mask.ensure(pairs);
    moved |= c->d_pair_sweeps.ensure(pairs * 4);
    moved |= c->d_model_active.ensure(M);
    moved |= c->d_act_models.ensure((size_t)M * 4 + 4);
    moved |= c->d_act_prefix.ensure((size_t)(M + 1) * 4 + 4);
    moved |= c->d_act_tiles.ensure(std::max<size_t>(c->tiles.size(), (size_t)c->n_htiles) * 4 + 4);
    moved |= c->d_best_res.ensure(pairs * 8);
    moved |= c->d_stall.ensure(pairs * 4);
    moved |= c->d_counters.ensure(9 * 8);
    c->h_counters.ensure(9 * 8);
    // a captured sweep graph holds these addresses: it must not replay
    // after any of them moved
    if (moved) ++c->buf_gen;
}

static void ensure_values(morap_ctx* c, ValueSet& vs, int K, int Kp, int prec) {
    const size_t el = prec == MORAP_F32 ? 4 : 8;
    bool moved = false;
    // one row past the last state: the zero row of the block sweep
    moved |= vs.x[0].ensure((size_t)(c->S + 1) * Kp * el);
    moved |= vs.x[1].ensure((size_t)(c->S + 1) * Kp * el);
    moved |= vs.final_par.ensure((size_t)c->hm.M * Kp);
    moved |= vs.c.ensure((size_t)K * c->hm.M * 8);
    if (moved) ++c->buf_gen;
    vs.prec = prec;
    vs.K = K;
    vs.Kp = Kp;
    vs.valid = false;
}

// `halo`: the active tile list is built over the halo tiles (LDS-staged
// sweep) instead of the CSR / block tiles
static k::ConvergeArgs converge_args(morap_ctx* c, ValueSet& vs, const uint8_t* mask, double eps, int out_par,
                                     bool halo) {
    k::ConvergeArgs a{};
    a.res = c->d_res.as<unsigned long long>();
    a.ymax = c->d_ymax.as<unsigned long long>();
    a.active = c->d_active.as<uint8_t>();
    a.final_par = vs.final_par.as<uint8_t>();
    a.pair_sweeps = c->d_pair_sweeps.as<int32_t>();
    a.model_active = c->d_model_active.as<uint8_t>();
    a.c = vs.c.as<double>();
    a.init = c->d_init.as<int32_t>();
    a.mask = mask;
    a.x_out = vs.x[out_par].p;
    a.counters = c->d_counters.as<int64_t>();
    a.M = c->hm.M;
    a.K = vs.K;
    a.Kp = vs.Kp;
    a.prec = vs.prec;
    a.out_par = out_par;
    a.eps = eps;
    // FP32 backups cannot resolve changes below a few units in the last
    // place of the values: stop there too (FP64: the bound is below eps)
    a.unit = vs.prec == MORAP_F32 ? 8.0 * std::ldexp(1.0, -24) : 8.0 * std::ldexp(1.0, -53);
    a.best_res = c->d_best_res.as<double>();
    a.stall = c->d_stall.as<int32_t>();
    a.stall_sweeps = vs.prec == MORAP_F32 ? 64 : 0;
    a.floor = 256.0 * std::ldexp(1.0, -24);
    a.tile_base = halo ? c->d_htile_base.as<int32_t>() : c->d_tile_base.as<int32_t>();
    a.act_models = c->d_act_models.as<int32_t>();
    a.act_prefix = c->d_act_prefix.as<int32_t>();
    a.rows_per_model = c->d_rows_per_model.as<int32_t>();
    a.states_per_model = c->d_states_per_model.as<int32_t>();
    a.csr_bytes = vs.prec == MORAP_F32 ? c->d_csr_bytes32.as<int64_t>() : c->d_csr_bytes64.as<int64_t>();
    a.act_tiles = c->d_act_tiles.as<int32_t>();
    return a;
}

static k::SweepArgs sweep_args(morap_ctx* c, ValueSet& vs, int in_par) {
    k::SweepArgs a{};
    a.tiles = c->d_tiles.as<Tile>();
    a.tile_base = c->d_tile_base.as<int32_t>();
    a.act_models = c->d_act_models.as<int32_t>();
    a.act_prefix = c->d_act_prefix.as<int32_t>();
    a.counters = c->d_counters.as<int64_t>();
    a.state_row = c->d_state_row.as<int32_t>();
    a.row_ptr = c->d_row_ptr.as<int32_t>();
    a.col = c->d_col.as<int32_t>();
    const bool f32 = vs.prec == MORAP_F32;
    a.prob = f32 ? c->d_prob32.p : c->d_prob64.p;
    a.rew = f32 ? c->d_rew32.p : c->d_rew64.p;
    a.wc = f32 ? c->d_wc32.p : c->d_wc64.p;
    a.wp = f32 ? c->d_wp32.p : c->d_wp64.p;
    a.active = c->d_active.as<uint8_t>();
    a.x_in = vs.x[in_par].p;
    a.x_out = vs.x[1 - in_par].p;
    a.res = c->d_res.as<unsigned long long>();
    a.ymax = c->d_ymax.as<unsigned long long>();
    a.Kp = vs.Kp;
    a.rec = c->has_blocks ? c->d_blk_rec.as<int32_t>() : nullptr;
    a.ablk = c->has_blocks ? (f32 ? c->d_blk32.p : c->d_blk64.p) : nullptr;
    a.zero_row = (int32_t)c->S;
    a.pattern = c->hm.blk_pattern;
    a.act_tiles = c->d_act_tiles.as<int32_t>();
    a.htiles = c->has_halo ? c->d_htiles.as<HTile>() : nullptr;
    a.hrec = c->has_halo ? c->d_hrec.as<uint2>() : nullptr;
    a.hlist = c->has_halo ? c->d_hlist.as<int32_t>() : nullptr;
    a.rewk = c->team ? (f32 ? c->d_rewk32.p : c->d_rewk64.p) : nullptr;
    return a;
}

// Persistent grid: as many workgroups as the kernel keeps resident on the
// whole chip at once (a second, partial round of workgroups would double the
// time of a balanced sweep), a multiple of 8 (one share per XCD), and no more
// than the tiles need.
static int persistent_grid(morap_ctx* c, int prec, const Variant& v) {
    const int64_t key = ((int64_t)v.id << 8) | prec;
    int per_cu = 0;
    for (auto& r : c->resident)
        if (r.first == key) per_cu = r.second;
    if (per_cu == 0) {
        per_cu = v.kind == SWEEP_HALO                                   ? k::sweep_halo_resident(v, c->hm.blk_pattern)
                 : v.kind == SWEEP_BLOCK                              ? k::sweep_block_resident(prec, v)
                                                                        : k::sweep_resident(prec, v);
        per_cu = std::max(1, per_cu);
        c->resident.push_back({key, per_cu});
    }
    int g = c->prop.multiProcessorCount * per_cu;
    const int tiles = uses_halo_tiles(v) ? (int)c->n_htiles : (int)c->tiles.size();
    g = std::min(g, (tiles + 7) / 8 * 8);
    return std::max(8, g / 8 * 8);
}

using EventPairs = std::vector<std::pair<hipEvent_t, hipEvent_t>>;

// With time_kernels, every kTimedEvery-th sweep launch of a chunk is timed
// (a uniform sample: its average duration is the launches' average, with a
// quarter of the events in the stream)
constexpr int kTimedEvery = 4;

// per-launch timing events come from a pool: creating and destroying two
// events per sweep costs host time on every launch
static hipEvent_t take_event(morap_ctx* c) {
    if (!c->event_pool.empty()) {
        const hipEvent_t e = c->event_pool.back();
        c->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    MORAP_HIP(hipEventCreate(&e));
    return e;
}
static void give_events(morap_ctx* c, const std::pair<hipEvent_t, hipEvent_t>& e) {
    if (e.first) c->event_pool.push_back(e.first);
    if (e.second) c->event_pool.push_back(e.second);
}

// Sampled launch events held by a loop; whatever is still held when the
// scope ends (an error thrown mid-chunk included) goes back to the pool.
struct PooledEvents {
    morap_ctx* c;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> v;
    explicit PooledEvents(morap_ctx* ctx) : c(ctx) {}
    PooledEvents(const PooledEvents&) = delete;
    PooledEvents& operator=(const PooledEvents&) = delete;
    ~PooledEvents() {
        for (auto& e : v) give_events(c, e);
    }
};

// Two HIP events bracketing a timed region, destroyed on every way out of
// the scope that owns them.
struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    EventPair() {
        MORAP_HIP(hipEventCreate(&a));
        const hipError_t e = hipEventCreate(&b);
        if (e != hipSuccess) {
            (void)hipEventDestroy(a);
            a = nullptr;
            fail(MORAP_E_HIP, std::string("hipEventCreate: ") + hipGetErrorString(e));
        }
    }
    EventPair(const EventPair&) = delete;
    EventPair& operator=(const EventPair&) = delete;
    ~EventPair() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
    float elapsed_ms() const {
        float ms = 0;
        MORAP_HIP(hipEventElapsedTime(&ms, a, b));
        return ms;
    }
};

// Optional per-launch log (environment variable MORAP_SWEEP_LOG = file path):
// the autotuner's timings and, for solves run with time_kernels, one line per
// sweep launch with its active tile count and duration.
static FILE* sweep_log() {
    static FILE* f = [] {
        const char* p = std::getenv("MORAP_SWEEP_LOG");
        return p && *p ? std::fopen(p, "a") : nullptr;
    }();
    return f;
}

// one chunk of `n` sweeps (n even): sweep, converge, compact per sweep;
// `ev` (optional) receives an event pair around every sweep kernel
static void enqueue_chunk(morap_ctx* c, ValueSet& vs, const uint8_t* mask, const Variant& v, double eps, int n,
                          EventPairs* ev = nullptr) {
    const int grid = persistent_grid(c, vs.prec, v);
    const int ktiles = vs.Kp / kt_of(v);
    for (int i = 0; i < n; ++i) {
        const int in_par = i & 1;
        const bool timed = ev && i % kTimedEvery == 0;
        if (timed) {
            if (sweep_log() && ev->size() < 4096) {
                c->h_log.ensure(4096 * 8);
                MORAP_HIP(hipMemcpyAsync(c->h_log.as<int64_t>() + ev->size(), c->d_counters.as<int64_t>() + 1, 8,
                                         hipMemcpyDeviceToHost, c->stream));
            }
            ev->emplace_back(take_event(c), nullptr);
            ev->back().second = take_event(c);
            MORAP_HIP(hipEventRecord(ev->back().first, c->stream));
        }
        if (v.kind == SWEEP_HALO)
            k::sweep_halo(c->stream, vs.prec, v, grid, ktiles, sweep_args(c, vs, in_par));
        else if (v.kind == SWEEP_BLOCK)
            k::sweep_block(c->stream, vs.prec, v, grid, ktiles, sweep_args(c, vs, in_par));
        else
            k::sweep(c->stream, vs.prec, v, grid, ktiles, sweep_args(c, vs, in_par));
        if (timed) MORAP_HIP(hipEventRecord(ev->back().second, c->stream));
        const auto ca = converge_args(c, vs, mask, eps, 1 - in_par, uses_halo_tiles(v));
        k::converge(c->stream, ca);
        k::compact(c->stream, ca);
    }
}

static void reset_solve(morap_ctx* c, ValueSet& vs, const uint8_t* mask, double eps, const Variant& v) {
    const int64_t n = (c->S + 1) * vs.Kp;
    if (vs.prec == MORAP_F32) {
        k::fill_f32(c->stream, vs.x[0].as<float>(), 0.f, n);
        k::fill_f32(c->stream, vs.x[1].as<float>(), 0.f, n);
    } else {
        k::fill_f64(c->stream, vs.x[0].as<double>(), 0.0, n);
        k::fill_f64(c->stream, vs.x[1].as<double>(), 0.0, n);
    }
    k::init_solve(c->stream, converge_args(c, vs, mask, eps, 1, uses_halo_tiles(v)));
}

static void release_graph(morap_ctx* c, int g) {
    if (c->chunk_exec[g]) (void)hipGraphExecDestroy(c->chunk_exec[g]);
    if (c->chunk_graph[g]) (void)hipGraphDestroy(c->chunk_graph[g]);
    c->chunk_exec[g] = nullptr;
    c->chunk_graph[g] = nullptr;
    c->graph_key[g].clear();
}

// run one chunk, replaying a captured graph (slot g) when asked to
static void run_chunk(morap_ctx* c, int g, ValueSet& vs, const uint8_t* mask, const Variant& v, double eps, int n,
                      bool graph, EventPairs* ev) {
    if (!graph || ev) {
        enqueue_chunk(c, vs, mask, v, eps, n, ev);
        return;
    }
    char key[320];
    // the key names everything the captured launches hold: the model upload
    // and the solve buffers (by generation, so a buffer reallocated at an
    // old address still counts as new), the variant and the sizes
    snprintf(key, sizeof key, "%llu/%llu/%d/%d/%d/%d/%d/%.17g/%p/%p/%p/%p/%zu", (unsigned long long)c->load_gen,
             (unsigned long long)c->buf_gen, v.id, vs.K, vs.Kp, vs.prec, n, eps, vs.x[0].p, vs.x[1].p,
             (const void*)mask, vs.c.p, c->tiles.size());
    if (c->graph_key[g] != key) {
        release_graph(c, g);
        MORAP_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        try {
            enqueue_chunk(c, vs, mask, v, eps, n);
        } catch (...) {
            hipGraph_t gr = nullptr;
            (void)hipStreamEndCapture(c->stream, &gr);
            if (gr) (void)hipGraphDestroy(gr);
            throw;
        }
        MORAP_HIP(hipStreamEndCapture(c->stream, &c->chunk_graph[g]));
        MORAP_HIP(hipGraphInstantiate(&c->chunk_exec[g], c->chunk_graph[g], nullptr, nullptr, 0));
        c->graph_key[g] = key;
    }
    MORAP_HIP(hipGraphLaunch(c->chunk_exec[g], c->stream));
}

static void read_counters(morap_ctx* c) {
    MORAP_HIP(hipMemcpyAsync(c->h_counters.p, c->d_counters.p, 9 * 8, hipMemcpyDeviceToHost, c->stream));
    MORAP_HIP(hipStreamSynchronize(c->stream));
}

// time 6 sweeps of variant v from a fresh start (autotuner)
static double time_variant(morap_ctx* c, ValueSet& vs, const uint8_t* mask, const Variant& v, double eps) {
    EventPair t;
    reset_solve(c, vs, mask, eps, v);
    enqueue_chunk(c, vs, mask, v, eps, 2);
    MORAP_HIP(hipEventRecord(t.a, c->stream));
    enqueue_chunk(c, vs, mask, v, eps, 6);
    MORAP_HIP(hipEventRecord(t.b, c->stream));
    MORAP_HIP(hipEventSynchronize(t.b));
    return t.elapsed_ms();
}

// autotuner: the fastest candidate variant for (precision, padded width,
// restricted or not), timed on the loaded models and cached on the context
static const Variant& choose_variant(morap_ctx* c, ValueSet& vs, const uint8_t* mask, double eps, int schedule) {
    if (schedule > 0) {
        const Variant& v = variant_by_id(schedule);
        MORAP_CHECK(vs.Kp % kt_of(v) == 0, MORAP_E_INVALID, "variant does not divide the padded column count");
        MORAP_CHECK(v.kind != SWEEP_BLOCK || c->has_blocks, MORAP_E_UNSUPPORTED,
                    "the neighbourhood-block sweep needs products built from agents with at most 5 actions "
                    "and 5 successors per state");
        MORAP_CHECK(v.kind != SWEEP_HALO || (c->has_halo && vs.prec == MORAP_F32), MORAP_E_UNSUPPORTED,
                    "the LDS-staged sweep needs halo tiles (built with the block form) and FP32 values");
        return v;
    }
    const int64_t key = ((int64_t)vs.prec << 40) | ((int64_t)(mask != nullptr) << 32) | vs.Kp;
    for (auto& t : c->tuned)
        if (t.first == key) return variant_by_id(t.second);
    auto cand = candidates(vs.Kp, mask != nullptr, c->has_blocks, c->has_halo && vs.prec == MORAP_F32);
    MORAP_CHECK(!cand.empty(), MORAP_E_UNSUPPORTED, "no sweep variant for this column count");
    int best = cand[0].id;
    if (cand.size() > 1) {
        double best_ms = 1e300;
        // the timing covers full sweeps only; a wave-per-state gather sweep
        // also gets the LDS-staged kernel for the last sweeps of a solve
        // (~4 % of its time saved on the 50 x 100 workload), so the others
        // must beat it by 3 %
        const bool tail_possible = !mask && c->has_halo && vs.prec == MORAP_F32 && vs.Kp % 64 == 0;
        for (const auto& v : cand) {
            const bool gets_tail = tail_possible && v.kind == SWEEP_BLOCK && v.cpl == 1 && v.lps == 64;
            const double raw = time_variant(c, vs, mask, v, eps);
            const double ms = raw * (tail_possible && !gets_tail ? 1.03 : 1.0);
            if (sweep_log())
                std::fprintf(sweep_log(), "tune prec=%d mask=%d Kp=%d variant=%d kind=%d cpl=%d lps=%d grid=%d ms=%.4f\n",
                             vs.prec, mask != nullptr, vs.Kp, v.id, v.kind, v.cpl, v.lps,
                             persistent_grid(c, vs.prec, v), raw);
            if (ms < best_ms) {
                best_ms = ms;
                best = v.id;
            }
        }
    }
    c->tuned.push_back({key, best});
    return variant_by_id(best);
}

// Batched value iteration into `vs` until every (masked) pair has converged.
static void swap_buf(DevBuf& a, DevBuf& b) {
    std::swap(a.p, b.p);
    std::swap(a.bytes, b.bytes);
    std::swap(a.meter, b.meter);
}

// For the message of a solve that hit its sweep limit: the first pairs still
// active, each with its two weights and the change between the last two
// iterates (the two value buffers) at its most-changing state.
static std::string describe_active(morap_ctx* c, ValueSet& vs) {
    const int M = c->hm.M, Kp = vs.Kp;
    std::vector<uint8_t> act((size_t)M * Kp);
    MORAP_HIP(hipMemcpy(act.data(), c->d_active.p, act.size(), hipMemcpyDeviceToHost));
    const size_t el = vs.prec == MORAP_F32 ? 4 : 8;
    std::string out;
    int shown = 0;
    for (int m = 0; m < M && shown < 4; ++m)
        for (int k = 0; k < vs.K && shown < 4; ++k) {
            if (!act[(size_t)m * Kp + k]) continue;
            const int32_t s0 = c->hm.state_base[m], s1 = c->hm.state_base[m + 1];
            std::vector<char> b0((size_t)(s1 - s0) * Kp * el + 8), b1(b0.size());
            MORAP_HIP(hipMemcpy(b0.data(), vs.x[0].as<char>() + (size_t)s0 * Kp * el, b0.size() - 8,
                                hipMemcpyDeviceToHost));
            MORAP_HIP(hipMemcpy(b1.data(), vs.x[1].as<char>() + (size_t)s0 * Kp * el, b1.size() - 8,
                                hipMemcpyDeviceToHost));
            double dmax = -1, v0 = 0, v1 = 0;
            int at = -1;
            for (int32_t s = 0; s < s1 - s0; ++s) {
                const size_t i = (size_t)s * Kp + k;
                const double a = el == 4 ? reinterpret_cast<float*>(b0.data())[i] : reinterpret_cast<double*>(b0.data())[i];
                const double b = el == 4 ? reinterpret_cast<float*>(b1.data())[i] : reinterpret_cast<double*>(b1.data())[i];
                if (std::fabs(a - b) > dmax) {
                    dmax = std::fabs(a - b);
                    at = s;
                    v0 = a;
                    v1 = b;
                }
            }
            const int d = n_obj_of(c);
            const int i = m / c->hm.nJ, j = m % c->hm.nJ;
            const double wc = c->team ? 1.0 : c->W[(size_t)k * d + i];
            const double wp = c->team ? 0.0 : c->W[(size_t)k * d + c->hm.nI + j];
            char buf[320];
            std::snprintf(buf, sizeof buf,
                          "%s (model %d, column %d: weights %.9g, %.9g; last change %.6g at state %d, %.9g -> "
                          "%.9g)",
                          shown ? "," : ":", m, k, wc, wp, dmax, at, v0, v1);
            out += buf;
            ++shown;
        }
    return out;
}

// warm: the solve starts from the values prepared in d_xwarm (they become
// the first sweep's input buffer)
// The LDS-staged sweep for the last sweeps of a solve whose kernel is the
// wave-per-state gather sweep: the two give identical values, and once few
// tiles stay active (the last large models) the staged one is faster.
static const Variant* tail_variant(morap_ctx* c, const ValueSet& vs, const uint8_t* mask, const Variant& v,
                                   int schedule) {
    if (mask || schedule != 0 || !c->has_halo || vs.prec != MORAP_F32 || vs.Kp % 64 != 0) return nullptr;
    if (v.kind != SWEEP_BLOCK || v.cpl != 1 || v.lps != 64) return nullptr;
    for (const auto& t : variants())
        if (t.kind == SWEEP_HALO && t.unroll == 2) return &t;
    return nullptr;
}
// switch below this share of the tiles (MORAP_TAIL_PERCENT overrides it,
// 0 never switches)
static int tail_percent() {
    static const int p = [] {
        const char* e = std::getenv("MORAP_TAIL_PERCENT");
        return e && *e ? std::max(0, std::min(100, std::atoi(e))) : 20;
    }();
    return p;
}

static void run_vi(morap_ctx* c, int g, ValueSet& vs, const uint8_t* mask, const morap_vi_opts& o, Stats& st,
                   bool warm = false) {
    const Variant& v0 = choose_variant(c, vs, mask, o.eps_vi, o.schedule);
    c->last_variant = v0.id;
    const Variant* vt = tail_variant(c, vs, mask, v0, o.schedule);
    const Variant* vp = &v0;   // the kernel of the next chunk
    double bytes_at_switch = -1;
    int64_t sweeps_at_switch = 0;
    const int chunk = std::max(2, (o.check_every + 1) / 2 * 2);
    EventPair wall;
    reset_solve(c, vs, mask, o.eps_vi, v0);
    if (warm) {
        swap_buf(vs.x[0], c->d_xwarm);
        ++c->buf_gen;   // graphs hold the value buffers' addresses
    } else if (c->team) {
        // a team model starts below its optimum over proper policies (the
        // values of a fixed proper policy), which value iteration then
        // reaches instead of an improper fixed point above it
        k::team_start(c->stream, c->S, vs.K, vs.Kp, n_obj_of(c), c->d_team_w.as<double>(),
                      c->d_team_E.as<double>(), vs.prec, vs.x[0].p);
    }
    MORAP_HIP(hipEventRecord(wall.a, c->stream));
    int64_t launched = 0;
    int64_t* h = c->h_counters.as<int64_t>();
    PooledEvents held(c);
    EventPairs& ev = held.v;
    auto harvest = [&] {
        for (size_t i = 0; i < ev.size(); ++i) {
            auto& e = ev[i];
            float t = 0;
            MORAP_HIP(hipEventElapsedTime(&t, e.first, e.second));
            if (sweep_log() && i < 4096)
                std::fprintf(sweep_log(), "sweep prec=%d mask=%d variant=%d tiles=%lld ms=%.4f\n", vs.prec,
                             mask != nullptr, vp->id, (long long)c->h_log.as<int64_t>()[i], t);
            if (mask) {
                st.ms_sweep_kernel_refine += t;
                st.sweep_launches_refine += 1;
            } else if (vp != &v0) {
                st.ms_sweep_kernel_tail += t;
                st.sweep_launches_tail += 1;
            } else {
                st.ms_sweep_kernel += t;
                st.sweep_launches += 1;
            }
            give_events(c, e);
            e = {nullptr, nullptr};
        }
        ev.clear();
    };
    const size_t el = vs.prec == MORAP_F32 ? 4 : 8;
    const int64_t main_tiles = (int64_t)c->tiles.size();
    while (true) {
        run_chunk(c, vp == &v0 ? g : 2, vs, mask, *vp, o.eps_vi, chunk, o.use_graph != 0,
                  o.time_kernels ? &ev : nullptr);
        launched += chunk;
        read_counters(c);
        harvest();
        if (h[3] == 0) break;
        if (vt && vp == &v0 && h[1] * 100 < main_tiles * tail_percent()) {
            // the same active models listed over the halo tiles
            bytes_at_switch = (double)h[6] + 2.0 * el * (double)h[7];
            sweeps_at_switch = h[5];
            vp = vt;
            k::relist(c->stream, converge_args(c, vs, mask, o.eps_vi, 0, true));
        }
        if (launched >= o.max_sweeps)
            fail(MORAP_E_NOT_CONVERGED, "value iteration: " + std::to_string(h[3]) +
                                            " (model, column) pairs still active after " +
                                            std::to_string(launched) + " sweeps" + describe_active(c, vs));
    }
    MORAP_HIP(hipEventRecord(wall.b, c->stream));
    MORAP_HIP(hipEventSynchronize(wall.b));
    const float ms = wall.elapsed_ms();
    std::vector<int32_t> ps((size_t)c->hm.M * vs.Kp);
    MORAP_HIP(hipMemcpy(ps.data(), c->d_pair_sweeps.p, ps.size() * 4, hipMemcpyDeviceToHost));
    st.backups += h[4];
    st.floor_stops += h[8];
    const double bytes = (double)h[6] + 2.0 * el * (double)h[7];
    if (mask) {
        st.bytes_refine += bytes;
    } else if (bytes_at_switch >= 0) {
        st.bytes += bytes_at_switch;
        st.bytes_tail += bytes - bytes_at_switch;
        st.sweeps_tail += h[5] - sweeps_at_switch;
        st.variant_tail = vt->id;
    } else {
        st.bytes += bytes;
    }
    st.max_pair_sweeps = std::max<int64_t>(st.max_pair_sweeps, *std::max_element(ps.begin(), ps.end()));
    st.ms_vi += ms;
    if (mask) st.variant_refine = v0.id;
    else st.variant = v0.id;
    if (mask) st.polish_sweeps += h[5];
    else st.sweeps += h[5];
    vs.valid = true;
}

// ---------------------------------------------------------------------------
// solve
// ---------------------------------------------------------------------------
static void add_stats(Stats& a, const Stats& b) {
    a.backups += b.backups;
    a.sweeps += b.sweeps;
    a.max_pair_sweeps = std::max(a.max_pair_sweeps, b.max_pair_sweeps);
    a.eval_sweeps += b.eval_sweeps;
    a.polish_sweeps += b.polish_sweeps;
    a.rank_rounds += b.rank_rounds;
    a.floor_stops += b.floor_stops;
    a.bytes += b.bytes;
    a.ms_vi += b.ms_vi;
    a.ms_eval += b.ms_eval;
    a.ms_total += b.ms_total;
    a.ms_sweep_kernel += b.ms_sweep_kernel;
    a.sweep_launches += b.sweep_launches;
    a.bytes_refine += b.bytes_refine;
    a.ms_sweep_kernel_refine += b.ms_sweep_kernel_refine;
    a.sweep_launches_refine += b.sweep_launches_refine;
    a.sweeps_tail += b.sweeps_tail;
    a.sweep_launches_tail += b.sweep_launches_tail;
    a.bytes_tail += b.bytes_tail;
    a.ms_sweep_kernel_tail += b.ms_sweep_kernel_tail;
    a.variant_tail = b.variant_tail ? b.variant_tail : a.variant_tail;
    a.refine_pairs += b.refine_pairs;
    a.refine_columns += b.refine_columns;
    a.variant = b.variant ? b.variant : a.variant;
    a.variant_refine = b.variant_refine ? b.variant_refine : a.variant_refine;
}

static void solve_impl(morap_ctx* c, const double* W, int K, const morap_vi_opts& o, double* c_out, Stats& st,
                       const int32_t* warm);
static void evaluate_impl(morap_ctx* c, const int32_t* assign, int K, const morap_vi_opts& o, double* r_out,
                          Stats& st, const int32_t* warm);

void solve(morap_ctx* c, const double* W, int K, const morap_vi_opts& o, double* c_out, Stats& st,
           const int32_t* warm) {
    Stats local;
    solve_impl(c, W, K, o, c_out, local, warm);
    add_stats(st, local);
    add_stats(c->cum, local);
}

static std::vector<double> resolve_pairs(morap_ctx* c, const std::vector<int32_t>& pk,
                                         const std::vector<int32_t>& pm, const morap_vi_opts& o, Stats& st);
static int refine_assignment(morap_ctx* c, const int32_t* assign, int K, const morap_vi_opts& o, Stats& st,
                             int32_t* out);

void evaluate(morap_ctx* c, const int32_t* assign, int K, const morap_vi_opts& o, double* r_out, Stats& st,
              const int32_t* warm, int32_t* refine) {
    Stats local;
    c->eval_prev_valid = c->eval_prev_valid && c->prev_eval_gen == c->load_gen;
    try {
        evaluate_impl(c, assign, K, o, r_out, local, warm);
        if (refine) {
            std::copy(assign, assign + (size_t)K * c->hm.nJ, refine);
            if (!c->team && c->prec == MORAP_F32 && c->has_blocks && c->last_c64_valid &&
                refine_assignment(c, assign, K, o, local, refine) > 0) {
                // again with the new assignment, each instance started from
                // the first evaluation's values where the pair is unchanged
                std::vector<int32_t> same(K);
                for (int k = 0; k < K; ++k) same[k] = k;
                evaluate_impl(c, refine, K, o, r_out, local, same.data());
            }
        }
    } catch (...) {
        c->eval_prev_valid = false;
        throw;
    }
    add_stats(st, local);
    add_stats(c->cum, local);
}

// rows of W[K][d] on the simplex: finite, >= 0, summing to 1 (1e-9)
static void check_weight_rows(const double* W, int K, int d) {
    for (int k = 0; k < K; ++k) {
        double sum = 0;
        for (int q = 0; q < d; ++q) {
            const double w = W[(size_t)k * d + q];
            MORAP_CHECK(std::isfinite(w) && w >= 0, MORAP_E_INVALID, "weights must be finite and >= 0");
            sum += w;
        }
        MORAP_CHECK(std::fabs(sum - 1.0) <= 1e-9, MORAP_E_INVALID, "weight rows must sum to 1");
    }
}

static void solve_impl(morap_ctx* c, const double* W, int K, const morap_vi_opts& o, double* c_out, Stats& st,
                       const int32_t* warm) {
    MORAP_CHECK(c->loaded, MORAP_E_STATE, "no models loaded");
    MORAP_CHECK(W && K >= 1 && K <= 4096, MORAP_E_INVALID, "need 1 <= K <= 4096 weight vectors");
    MORAP_CHECK(o.precision == MORAP_F32 || o.precision == MORAP_F64, MORAP_E_INVALID, "bad precision");
    MORAP_CHECK(o.eps_vi > 0 && std::isfinite(o.eps_vi), MORAP_E_INVALID, "eps_vi must be > 0");
    MORAP_CHECK(o.max_sweeps >= 1, MORAP_E_INVALID, "max_sweeps must be >= 1");
    const int nI = c->hm.nI, nJ = c->hm.nJ, M = c->hm.M, d = n_obj_of(c);
    check_weight_rows(W, K, d);
    const auto t0 = std::chrono::steady_clock::now();
    const int prec = o.precision;
    const int Kp = padded_k(K);
    // a warm start needs the previous FP32 values in buffers that already
    // fit this solve (they are read in place)
    const size_t need = (size_t)(c->S + 1) * Kp * 4;
    const bool warm_ok = warm && !c->team && prec == MORAP_F32 && c->vmain.valid && c->vmain.prec == MORAP_F32 &&
                         Kp <= c->vmain.Kp && c->vmain.x[0].bytes >= need && c->vmain.x[1].bytes >= need;
    const int Kp_old = c->vmain.Kp, K_old = c->vmain.K;
    // Per pair, the start a x_prev + b from the previous values x_prev, which
    // are (up to the stop rule) the optimal values V = wc_o C + wp_o P of the
    // previous weights, C <= 0 and P in [0, 1] the cost and probability
    // values of the previous optimal policy.  Every start is below the new
    // optimum V', so value iteration climbs to it as from 0 and zero-reward
    // loops (which admit larger fixed points) cannot hold it above:
    //  * probability only now and before: V' = (wp_n / wp_o) V exactly (the
    //    optimal policies do not depend on the scale); a relative 1e-6 below
    //    it covers the previous stop (FP32 stops at 8 2^-24 relative);
    //  * a cost weight now and before: V' >= wc_n C >= (wc_n / wc_o)(V - wp_o),
    //    the previous policy's value without its probability reward;
    //  * otherwise from 0, as Alg. 3.
    std::vector<float> warm_ab;
    if (warm_ok) {
        const std::vector<double>& Wp = c->W;   // the previous solve's weights [K_old][d]
        warm_ab.assign((size_t)M * Kp * 2, 0.f);
        for (int k = 0; k < K; ++k) {
            MORAP_CHECK(warm[k] >= -1 && warm[k] < K_old, MORAP_E_INVALID, "warm-start column out of range");
            if (warm[k] < 0) continue;
            for (int m = 0; m < M; ++m) {
                const int i = m / nJ, j = m % nJ;
                const double wc_n = W[(size_t)k * d + i], wp_n = W[(size_t)k * d + nI + j];
                const double wc_o = Wp[(size_t)warm[k] * d + i], wp_o = Wp[(size_t)warm[k] * d + nI + j];
                double a = 0, b = 0;
                if (wc_n == 0 && wc_o == 0 && wp_o > 0) {
                    a = wp_n / wp_o * (1.0 - 1e-6);
                } else if (wc_n > 0 && wc_o > 0) {
                    a = wc_n / wc_o;
                    b = -a * wp_o;
                }
                warm_ab[((size_t)m * Kp + k) * 2] = (float)a;
                warm_ab[((size_t)m * Kp + k) * 2 + 1] = (float)b;
            }
        }
    }
    c->solved = false;
    c->evaluated = false;
    ensure_scratch(c, Kp);
    c->K = K;
    c->Kp = Kp;
    c->prec = prec;
    c->W.assign(W, W + (size_t)K * d);

    // per-(model, column) weights of the model's two objectives (a team
    // model: its rows are scalarised per column on the device instead, and
    // (1, 0) marks the column in use)
    std::vector<double> wc((size_t)M * Kp, 0.0), wp((size_t)M * Kp, 0.0);
    std::vector<float> wc32((size_t)M * Kp, 0.f), wp32((size_t)M * Kp, 0.f);
    for (int m = 0; m < M; ++m) {
        const int i = m / nJ, j = m % nJ;
        for (int k = 0; k < K; ++k) {
            wc[(size_t)m * Kp + k] = c->team ? 1.0 : W[(size_t)k * d + i];
            wp[(size_t)m * Kp + k] = c->team ? 0.0 : W[(size_t)k * d + nI + j];
            wc32[(size_t)m * Kp + k] = (float)wc[(size_t)m * Kp + k];
            wp32[(size_t)m * Kp + k] = (float)wp[(size_t)m * Kp + k];
        }
    }
    MORAP_HIP(hipMemcpyAsync(c->d_wc64.p, wc.data(), wc.size() * 8, hipMemcpyHostToDevice, c->stream));
    MORAP_HIP(hipMemcpyAsync(c->d_wp64.p, wp.data(), wp.size() * 8, hipMemcpyHostToDevice, c->stream));
    MORAP_HIP(hipMemcpyAsync(c->d_wc32.p, wc32.data(), wc32.size() * 4, hipMemcpyHostToDevice, c->stream));
    MORAP_HIP(hipMemcpyAsync(c->d_wp32.p, wp32.data(), wp32.size() * 4, hipMemcpyHostToDevice, c->stream));
    if (c->team) {
        // every (row, column)'s reward w[obj[r][0]] rew[r][0] + w[obj[r][1]] rew[r][1]
        const int64_t R = c->hm.state_row.back();
        bool moved = c->d_team_w.ensure((size_t)K * d * 8);
        moved |= c->d_rewk64.ensure((size_t)R * Kp * 8 + 8);
        moved |= c->d_rewk32.ensure((size_t)R * Kp * 4 + 8);
        if (moved) ++c->buf_gen;
        MORAP_HIP(hipMemcpyAsync(c->d_team_w.p, W, (size_t)K * d * 8, hipMemcpyHostToDevice, c->stream));
        k::team_rewards(c->stream, R, K, Kp, d, c->d_team_w.as<double>(), c->d_obj.as<int32_t>(),
                        c->d_rew64.as<double>(), c->d_rewk64.as<double>(), c->d_rewk32.as<float>());
    }
    if (warm_ok) {
        c->d_warm_map.ensure((size_t)K * 4);
        c->d_warm_ab.ensure(warm_ab.size() * 4);
        c->d_xwarm.ensure(need);
        MORAP_HIP(hipMemcpyAsync(c->d_warm_map.p, warm, (size_t)K * 4, hipMemcpyHostToDevice, c->stream));
        MORAP_HIP(hipMemcpyAsync(c->d_warm_ab.p, warm_ab.data(), warm_ab.size() * 4, hipMemcpyHostToDevice,
                                 c->stream));
        k::warm_columns(c->stream, c->S, Kp, K, c->d_warm_map.as<int32_t>(), c->d_state_model.as<int32_t>(),
                        c->d_warm_ab.as<float>(), c->vmain.x[0].as<float>(), c->vmain.x[1].as<float>(),
                        c->vmain.final_par.as<uint8_t>(), Kp_old, c->d_xwarm.as<float>());
    }
    ensure_values(c, c->vmain, K, Kp, prec);
    MORAP_HIP(hipStreamSynchronize(c->stream));   // the host weight vectors go out of scope

    run_vi(c, 0, c->vmain, nullptr, o, st, warm_ok);
    if (c_out)
        MORAP_HIP(hipMemcpyAsync(c_out, c->vmain.c.p, (size_t)K * M * 8, hipMemcpyDeviceToHost, c->stream));
    MORAP_HIP(hipStreamSynchronize(c->stream));
    st.ms_total += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    c->solved = true;
}

// ---------------------------------------------------------------------------
// evaluate: FP64 values of the assigned pairs, policy extraction, Alg. 4
// ---------------------------------------------------------------------------
static k::InstArgs inst_args(morap_ctx* c, int n_tiles, int n_inst) {
    k::InstArgs a{};
    a.inst_model = c->d_inst_model.as<int32_t>();
    a.inst_k = c->d_inst_k.as<int32_t>();
    a.inst_base = c->d_inst_base.as<int64_t>();
    a.inst_tiles = c->d_inst_tiles.as<int32_t>();
    a.n_tiles = n_tiles;
    a.n_inst = n_inst;
    a.state_base = c->d_state_base.as<int32_t>();
    a.state_row = c->d_state_row.as<int32_t>();
    a.row_ptr = c->d_row_ptr.as<int32_t>();
    a.col = c->d_col.as<int32_t>();
    a.prob = c->d_prob64.as<double>();
    a.rew = c->d_rew64.as<double>();
    a.to_done = c->d_to_done.as<uint8_t>();
    a.init = c->d_init.as<int32_t>();
    a.cus = c->prop.multiProcessorCount;
    if (c->team) {
        a.rewk = c->d_rewk64.as<double>();
        a.rewk_ld = c->Kp;
        a.row_obj = c->d_obj.as<int32_t>();
        a.inst_obj = c->d_inst_obj.as<int32_t>();
    }
    return a;
}

// widenings of the tie tolerance in policy extraction (tau * 10^k, k <= 6)
constexpr int kTauSteps = 6;

// Stop of the FP64 values a pair's policy is chosen from (R16): eps_vi, or
// 1e-4 eps_vi (not below 1e-12, never above eps_vi) when the scaled cost
// weight vanishes.  Then every action that completes the task as surely as
// the best is optimal, and values stopped at eps_vi differ between such
// actions by their own error, far above the tie tolerance: the greedy
// choice among them is decided by that error and can be an action that
// progresses only through a slip (hundreds of thousands of expected steps,
// which no evaluation finishes).
static double policy_eps(double eps_vi, double wc, double wp) {
    if (wc < 1e-6 && wp > 0) return std::min(eps_vi, std::max(eps_vi * 1e-4, 1e-12));
    return eps_vi;
}

static void evaluate_impl(morap_ctx* c, const int32_t* assign, int K, const morap_vi_opts& o, double* r_out,
                          Stats& st, const int32_t* warm) {
    MORAP_CHECK(c->solved, MORAP_E_STATE, "morap_evaluate needs a morap_solve first");
    MORAP_CHECK(K == c->K, MORAP_E_INVALID, "K differs from the last morap_solve");
    MORAP_CHECK(assign != nullptr || c->team, MORAP_E_INVALID, "assign is NULL");
    MORAP_CHECK(o.eps_eval > 0 && o.eps_vi > 0 && o.tau >= 0, MORAP_E_INVALID, "bad tolerances");
    const bool team = c->team;
    const int nI = c->hm.nI, nJ = team ? (n_obj_of(c) + 1) / 2 : c->hm.nJ, d = team ? n_obj_of(c) : nI + nJ;
    // A team model has one policy per column; its instances (one per pair of
    // objectives, nJ per column) evaluate that policy's objectives 2p, 2p+1.
    std::vector<int32_t> team_assign;
    if (team) {
        team_assign.assign((size_t)K * nJ, 0);
        assign = team_assign.data();
    }
    const int cap = team ? nJ : std::max(1, (nJ + nI - 1) / nI);
    for (int kk = 0; kk < K; ++kk) {
        std::vector<int> load(nI, 0);
        for (int j = 0; j < nJ; ++j) {
            const int i = assign[(size_t)kk * nJ + j];
            MORAP_CHECK(i >= 0 && i < nI, MORAP_E_INVALID, "assigned agent out of range");
            MORAP_CHECK(++load[i] <= cap, MORAP_E_INVALID, "an agent received more than ceil(|J|/|I|) tasks");
        }
    }
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = c->stream;
    c->evaluated = false;
    // instances (k, m), task-major within each column
    const int n = K * nJ;
    c->assign.assign(assign, assign + (size_t)K * nJ);
    c->inst_k.resize(n);
    c->inst_m.resize(n);
    c->inst_base.assign(n + 1, 0);
    std::vector<int32_t> tiles;
    std::vector<double> iwc(n), iwp(n), iscale(n, 0.0);
    std::vector<int64_t> init_idx(n, -1);
    for (int kk = 0; kk < K; ++kk)
        for (int j = 0; j < nJ; ++j) {
            const int q = kk * nJ + j;
            const int i = assign[q];
            const int m = team ? 0 : i * nJ + j;
            c->inst_k[q] = kk;
            c->inst_m[q] = m;
            const int S_m = c->hm.state_base[m + 1] - c->hm.state_base[m];
            c->inst_base[q + 1] = c->inst_base[q] + S_m;
            for (int b = 0; b < S_m; b += 256) {
                tiles.push_back(q);
                tiles.push_back(b);
            }
            iwc[q] = team ? 1.0 : c->W[(size_t)kk * d + i];
            iwp[q] = team ? 0.0 : c->W[(size_t)kk * d + nI + j];
            const double sc = iwc[q] + iwp[q];   // policies come from the weights scaled to sum 1
            if (sc > 0) {
                iwc[q] /= sc;
                iwp[q] /= sc;
                iscale[q] = 1.0 / sc;
            }
            if (c->hm.init[m] >= 0) init_idx[q] = c->inst_base[q] + (c->hm.init[m] - c->hm.state_base[m]);
        }
    const int64_t NS = c->inst_base[n];
    const int n_tiles = (int)(tiles.size() / 2);
    c->d_inst_model.ensure((size_t)n * 4);
    c->d_inst_k.ensure((size_t)n * 4);
    c->d_inst_base.ensure((size_t)(n + 1) * 8);
    c->d_inst_tiles.ensure(tiles.size() * 4 + 8);
    c->d_iwc.ensure((size_t)n * 8);
    c->d_iwp.ensure((size_t)n * 8);
    c->d_iscale.ensure((size_t)n * 8);
    c->d_xi.ensure((size_t)NS * 8 + 8);
    c->d_ires.ensure((size_t)2 * n * 8);
    c->d_iactive.ensure((size_t)2 * n);
    c->d_ipar.ensure((size_t)2 * n);
    c->d_mask.ensure((size_t)NS * 4 + 4);
    c->d_rank.ensure((size_t)NS * 4 + 4);
    c->d_mu.ensure((size_t)NS + 4);
    c->d_xe[0].ensure((size_t)NS * 16 + 16);
    c->d_xe[1].ensure((size_t)NS * 16 + 16);
    c->d_init_idx.ensure((size_t)n * 8);
    c->d_init_val.ensure((size_t)2 * n * 8);
    MORAP_HIP(hipMemcpyAsync(c->d_inst_model.p, c->inst_m.data(), (size_t)n * 4, hipMemcpyHostToDevice, s));
    MORAP_HIP(hipMemcpyAsync(c->d_inst_k.p, c->inst_k.data(), (size_t)n * 4, hipMemcpyHostToDevice, s));
    MORAP_HIP(hipMemcpyAsync(c->d_inst_base.p, c->inst_base.data(), (size_t)(n + 1) * 8, hipMemcpyHostToDevice, s));
    if (!tiles.empty())
        MORAP_HIP(hipMemcpyAsync(c->d_inst_tiles.p, tiles.data(), tiles.size() * 4, hipMemcpyHostToDevice, s));
    MORAP_HIP(hipMemcpyAsync(c->d_iwc.p, iwc.data(), (size_t)n * 8, hipMemcpyHostToDevice, s));
    MORAP_HIP(hipMemcpyAsync(c->d_iwp.p, iwp.data(), (size_t)n * 8, hipMemcpyHostToDevice, s));
    MORAP_HIP(hipMemcpyAsync(c->d_iscale.p, iscale.data(), (size_t)n * 8, hipMemcpyHostToDevice, s));
    std::vector<double> ieps(n);
    double eps_pol = o.eps_vi;
    for (int q = 0; q < n; ++q) {
        ieps[q] = team ? o.eps_vi : policy_eps(o.eps_vi, iwc[q], iwp[q]);
        eps_pol = std::min(eps_pol, ieps[q]);
    }
    c->d_ieps.ensure((size_t)n * 8 + 8);
    MORAP_HIP(hipMemcpyAsync(c->d_ieps.p, ieps.data(), (size_t)n * 8, hipMemcpyHostToDevice, s));
    MORAP_HIP(hipMemcpyAsync(c->d_init_idx.p, init_idx.data(), (size_t)n * 8, hipMemcpyHostToDevice, s));
    std::vector<int32_t> iobj;
    if (team) {
        iobj.resize((size_t)2 * n);
        for (int q = 0; q < n; ++q) {
            const int p = q % nJ;
            iobj[2 * q] = 2 * p;
            iobj[2 * q + 1] = 2 * p + 1 < d ? 2 * p + 1 : -1;
        }
        c->d_inst_obj.ensure((size_t)2 * n * 4);
        MORAP_HIP(hipMemcpyAsync(c->d_inst_obj.p, iobj.data(), iobj.size() * 4, hipMemcpyHostToDevice, s));
    }
    const k::InstArgs a = inst_args(c, n_tiles, n);
    int64_t* dctr = c->d_counters.as<int64_t>();
    int64_t* h = c->h_counters.as<int64_t>();
    unsigned long long* ires = c->d_ires.as<unsigned long long>();
    uint8_t* iact = c->d_iactive.as<uint8_t>();
    uint8_t* ipar = c->d_ipar.as<uint8_t>();
    const int chunk = std::max(2, (o.check_every + 1) / 2 * 2);

    // Tiles of the instances that still have an active entry (width entries
    // per instance): the sweeps between two host checks launch only these.
    auto live_tiles = [&](const uint8_t* dflags, int width, k::InstArgs& out) {
        std::vector<uint8_t> f((size_t)width * n);
        MORAP_HIP(hipMemcpy(f.data(), dflags, f.size(), hipMemcpyDeviceToHost));
        c->h_live_tiles.clear();
        int64_t states = 0;
        for (size_t t = 0; t < tiles.size() / 2; ++t) {
            const int inst = tiles[2 * t];
            bool on = false;
            for (int w = 0; w < width; ++w) on |= f[(size_t)inst * width + w] != 0;
            if (!on) continue;
            c->h_live_tiles.push_back(tiles[2 * t]);
            c->h_live_tiles.push_back(tiles[2 * t + 1]);
            const int m = c->inst_m[inst];
            states += std::min<int64_t>(256, c->hm.state_base[m + 1] - c->hm.state_base[m] - tiles[2 * t + 1]);
        }
        c->d_live_tiles.ensure(c->h_live_tiles.size() * 4 + 8);
        if (!c->h_live_tiles.empty())
            MORAP_HIP(hipMemcpy(c->d_live_tiles.p, c->h_live_tiles.data(), c->h_live_tiles.size() * 4,
                                hipMemcpyHostToDevice));
        out = a;
        out.inst_tiles = c->d_live_tiles.as<int32_t>();
        out.n_tiles = (int)(c->h_live_tiles.size() / 2);
        return states;
    };

    // Values for the policies: FP64 value iteration from 0 on exactly the
    // assigned pairs, with each model's two weights scaled to sum 1.  Scaling
    // leaves the optimal policies unchanged; it keeps the absolute stop test
    // and the tie tolerance meaningful when both weights are tiny (the
    // unscaled iteration then stops after a sweep or two and its greedy
    // policy can take ~1e6 steps to finish).  With the neighbourhood-block
    // form the instances iterate in their own (instance-major) values;
    // otherwise the batched sweep re-solves the marked pairs.
    double* xi = c->d_xi.as<double>();
    if (c->has_blocks) {
        c->d_xr.ensure((size_t)NS * 8 + 8);
        double* x0 = xi;
        double* x1 = c->d_xr.as<double>();
        // after an FP32 solve the re-solve starts from its values (scaled to
        // the instance's weights); after an FP64 solve from 0, as Alg. 3
        if (c->prec == MORAP_F32 && c->vmain.valid)
            k::warm_start(s, a, c->vmain.x[0].p, c->vmain.x[1].p, c->vmain.final_par.as<uint8_t>(), c->vmain.Kp,
                          c->d_iscale.as<double>(), c->d_iwc.as<double>(), x0);
        else
            k::fill_f64(s, x0, 0.0, NS);
        k::fill_f64(s, x1, 0.0, NS);
        k::set_active(s, n, a, iact, ires, ipar, 1);
        EventPair wall;
        MORAP_HIP(hipEventRecord(wall.a, s));
        k::InstArgs av = a;
        int64_t live_states = NS;
        int64_t vsweeps = 0;
        PooledEvents held(c);
        EventPairs& ev = held.v;
        while (true) {
            for (int i = 0; i < chunk; ++i) {
                const bool even = (i & 1) == 0;
                const bool timed = o.time_kernels && i % kTimedEvery == 0;
                if (timed) {
                    ev.emplace_back(take_event(c), nullptr);
                    ev.back().second = take_event(c);
                    MORAP_HIP(hipEventRecord(ev.back().first, s));
                }
                k::inst_vi_sweep(s, av, c->d_blk_rec.as<int32_t>(), c->d_blk64.as<double>(), c->d_iwc.as<double>(),
                                 c->d_iwp.as<double>(), iact, even ? x0 : x1, even ? x1 : x0, ires, (int32_t)c->S,
                                 c->hm.blk_pattern);
                if (timed) MORAP_HIP(hipEventRecord(ev.back().second, s));
                k::inst_converge(s, n, ires, iact, ipar, even ? 1 : 0, o.eps_vi, dctr, c->d_ieps.as<double>());
            }
            vsweeps += chunk;
            // record + own value read + write per live instance state
            st.bytes_refine += (double)chunk * (double)live_states * 48.0;
            read_counters(c);
            for (auto& e : ev) {
                float t = 0;
                MORAP_HIP(hipEventElapsedTime(&t, e.first, e.second));
                st.ms_sweep_kernel_refine += t;
                st.sweep_launches_refine += 1;
                give_events(c, e);
                e = {nullptr, nullptr};
            }
            ev.clear();
            if (h[0] == 0) break;
            MORAP_CHECK(vsweeps < o.max_sweeps, MORAP_E_NOT_CONVERGED,
                        "value iteration of the assigned pairs: " + std::to_string(h[0]) +
                            " instances still active after " + std::to_string(vsweeps) + " sweeps");
            live_states = live_tiles(iact, 1, av);
        }
        k::select_final(s, a, x0, x1, ipar, 1);
        MORAP_HIP(hipEventRecord(wall.b, s));
        MORAP_HIP(hipEventSynchronize(wall.b));
        st.ms_vi += wall.elapsed_ms();
        st.polish_sweeps += vsweeps;
        st.variant_refine = -1;   // instance-major block iteration
        // the assigned pairs' FP64 values at their initial states, for the
        // weights of the column (the re-solve scaled them to sum 1)
        c->last_c64_valid = false;
        if (c->prec == MORAP_F32 && !team) {
            double* v = c->d_init_val.as<double>();
            k::gather_values(s, n, c->d_init_idx.as<int64_t>(), x0, v);
            c->last_c64.resize(n);
            MORAP_HIP(hipMemcpyAsync(c->last_c64.data(), v, (size_t)n * 8, hipMemcpyDeviceToHost, s));
            MORAP_HIP(hipStreamSynchronize(s));
            for (int q = 0; q < n; ++q) c->last_c64[q] = iscale[q] > 0 ? c->last_c64[q] / iscale[q] : 0.0;
            c->last_c64_valid = true;
        }
    } else {
        const int M = c->hm.M, Kp = c->Kp;
        std::vector<double> wc((size_t)M * Kp, 0.0), wp((size_t)M * Kp, 0.0);
        for (int kk = 0; kk < K; ++kk)
            for (int m = 0; m < M; ++m) {
                const int i = m / c->hm.nJ, j = m % c->hm.nJ;
                double a0 = team ? 1.0 : c->W[(size_t)kk * d + i], a1 = team ? 0.0 : c->W[(size_t)kk * d + nI + j];
                const double sc = a0 + a1;
                if (sc > 0) {
                    a0 /= sc;
                    a1 /= sc;
                }
                wc[(size_t)m * Kp + kk] = a0;
                wp[(size_t)m * Kp + kk] = a1;
            }
        MORAP_HIP(hipMemcpyAsync(c->d_wc64.p, wc.data(), wc.size() * 8, hipMemcpyHostToDevice, s));
        MORAP_HIP(hipMemcpyAsync(c->d_wp64.p, wp.data(), wp.size() * 8, hipMemcpyHostToDevice, s));
        MORAP_HIP(hipStreamSynchronize(s));   // the host vectors go out of scope
        ensure_values(c, c->vref, K, c->Kp, MORAP_F64);
        uint8_t* pm = c->d_pair_mask.as<uint8_t>();
        k::fill_u8(s, pm, 0, (int64_t)c->hm.M * c->Kp);
        k::mark_pairs(s, a, c->Kp, pm);
        // one stop for the masked batched re-solve: the tightest any pair needs
        morap_vi_opts op = o;
        op.eps_vi = eps_pol;
        run_vi(c, 1, c->vref, pm, op, st);
        k::gather_columns(s, a, MORAP_F64, c->vref.x[0].p, c->vref.x[1].p, c->vref.final_par.as<uint8_t>(),
                          c->vref.Kp, xi);
    }

    EventPair wall;
    MORAP_HIP(hipEventRecord(wall.a, s));

    // Attractor rounds with the tolerance tau; states left unranked get the
    // tolerance widened tenfold (up to tau * 1e6) while ranked states keep
    // their choice.
    uint32_t* mask = c->d_mask.as<uint32_t>();
    int32_t* rank = c->d_rank.as<int32_t>();
    c->d_ichanged.ensure((size_t)n + 8);
    uint8_t* ichg = c->d_ichanged.as<uint8_t>();
    int8_t* mu = c->d_mu.as<int8_t>();
    k::opt_mask(s, a, c->d_iwc.as<double>(), c->d_iwp.as<double>(), xi, o.tau, mask, rank, mu, false);
    int base = 0, relax_sweeps = 0;
    double tau = o.tau;
    for (int widen = 0;; ++widen) {
        // ranks of this phase: relax to the fixed point (8 sweeps per check,
        // alternating direction; converged when the last sweep changed
        // nothing).  After a round only the tiles of instances that changed
        // in it are relaxed again: ranks spread only inside an instance.
        k::InstArgs ar = a;
        for (int round = 0;; ++round) {
            k::fill_i64(s, dctr, 0, 8);
            k::fill_u8(s, ichg, 0, n);
            for (int i = 0; i < 8; ++i) k::relax_ranks(s, ar, mask, rank, base, (i & 1) != 0, 16, dctr + i, ichg);
            relax_sweeps += 8;
            read_counters(c);
            if (h[7] == 0) break;
            MORAP_CHECK(round < 1000000, MORAP_E_IMPROPER, "attractor ranks did not settle");
            live_tiles(ichg, 1, ar);
        }
        k::fill_i64(s, dctr, 0, 1);
        k::choose_actions(s, a, mask, rank, mu, base, dctr);
        read_counters(c);
        base = std::max<int64_t>(base, h[0]);
        k::fill_i64(s, dctr, 0, 1);
        k::count_unranked(s, a, rank, dctr);
        read_counters(c);
        if (h[0] == 0 || widen == kTauSteps) break;
        tau *= 10.0;
        k::opt_mask(s, a, c->d_iwc.as<double>(), c->d_iwp.as<double>(), xi, tau, mask, rank, mu, true);
    }
    st.rank_rounds += relax_sweeps;
    if (h[0] != 0) {
        fail(MORAP_E_IMPROPER, std::to_string(h[0]) + " states cannot reach done through tau-optimal actions");
    }

    // Alg. 4 per objective, from 0, or (warm) each instance whose column's
    // previous column had an instance of the same task on the same model from
    // that instance's final values, and (eval_start) from the scalarised
    // values: the evaluation of a proper policy reaches its values from any
    // start, with the same bound on the error at its stop
    double* xe0 = c->d_xe[0].as<double>();
    double* xe1 = c->d_xe[1].as<double>();
    k::fill_f64(s, xe0, 0.0, 2 * NS);
    k::fill_f64(s, xe1, 0.0, 2 * NS);
    std::vector<uint8_t> iwarm(n, 0);
    if (warm && c->eval_prev_valid && c->prev_per_col == nJ) {
        std::vector<int64_t> runs;
        const int K_prev = (int)(c->prev_inst_m.size() / std::max(1, nJ));
        for (int kk = 0; kk < K; ++kk) {
            const int kp = warm[kk];
            MORAP_CHECK(kp >= -1, MORAP_E_INVALID, "warm-start column out of range");
            if (kp < 0 || kp >= K_prev) continue;
            for (int j = 0; j < nJ; ++j) {
                const int q = kk * nJ + j, qp = kp * nJ + j;
                if (c->prev_inst_m[qp] != c->inst_m[q]) continue;
                iwarm[q] = 1;
                runs.push_back(c->inst_base[q]);
                runs.push_back(c->prev_inst_base[qp]);
                runs.push_back(c->inst_base[q + 1] - c->inst_base[q]);
            }
        }
        if (!runs.empty()) {
            c->d_warm_copy.ensure(runs.size() * 8);
            MORAP_HIP(hipMemcpyAsync(c->d_warm_copy.p, runs.data(), runs.size() * 8, hipMemcpyHostToDevice, s));
            k::copy_runs(s, c->d_warm_copy.as<int64_t>(), (int)(runs.size() / 3), c->d_xe_prev.as<double>(), xe0);
            MORAP_HIP(hipStreamSynchronize(s));   // the host run list goes out of scope
        }
    }
    if (o.eval_start && !team) {
        // from the scalarised values the policies were chosen from (R15)
        c->d_iwarm.ensure((size_t)n + 16);
        MORAP_HIP(hipMemcpyAsync(c->d_iwarm.p, iwarm.data(), (size_t)n, hipMemcpyHostToDevice, s));
        k::eval_start(s, a, xi, c->d_iwc.as<double>(), c->d_iwp.as<double>(), c->d_iwarm.as<uint8_t>(), xe0);
        MORAP_HIP(hipStreamSynchronize(s));   // iwarm goes out of scope
    }
    k::set_active(s, n, a, iact, ires, ipar, 2);
    int64_t esweeps = 0;
    k::InstArgs ae = a;
    while (true) {
        for (int i = 0; i < chunk; ++i) {
            const bool even = (i & 1) == 0;
            if (c->has_blocks)
                k::eval_block_sweep(s, ae, c->d_blk_rec.as<int32_t>(), c->d_blk64.as<double>(), mu, iact,
                                    even ? xe0 : xe1, even ? xe1 : xe0, ires, (int32_t)c->S, c->hm.blk_pattern);
            else
                k::eval_sweep(s, ae, mu, iact, even ? xe0 : xe1, even ? xe1 : xe0, ires);
            k::inst_converge(s, 2 * n, ires, iact, ipar, even ? 1 : 0, o.eps_eval, dctr);
        }
        esweeps += chunk;
        read_counters(c);
        if (h[0] == 0) break;
        if (esweeps < o.max_sweeps) {
            live_tiles(iact, 2, ae);
            continue;
        }
        {
            // name the (column, task, objective) entries still running; the
            // policies stay readable through morap_get_policy
            std::vector<uint8_t> still((size_t)2 * n);
            MORAP_HIP(hipMemcpy(still.data(), iact, still.size(), hipMemcpyDeviceToHost));
            // current iterate at the initial states, for the message
            k::select_final(s, a, xe0, xe1, ipar, 2);
            k::gather_init(s, n, c->d_init_idx.as<int64_t>(), xe0, c->d_init_val.as<double>());
            std::vector<double> now((size_t)2 * n);
            MORAP_HIP(hipMemcpyAsync(now.data(), c->d_init_val.p, now.size() * 8, hipMemcpyDeviceToHost, s));
            MORAP_HIP(hipStreamSynchronize(s));
            std::string who;
            int shown = 0;
            for (int q = 0; q < 2 * n && shown < 8; ++q)
                if (still[q]) {
                    const int inst = q / 2;
                    char buf[256];
                    std::snprintf(buf, sizeof buf,
                                  " (k=%d, j=%d, %s: model %d, weights %.17g, %.17g, value at the initial state "
                                  "now %.6g / %.6g)",
                                  inst / nJ, inst % nJ, q % 2 ? "probability" : "cost", c->inst_m[inst],
                                  iwc[inst], iwp[inst], now[2 * inst], now[2 * inst + 1]);
                    who += buf;
                    ++shown;
                }
            c->eK = K;
            c->evaluated = true;
            fail(MORAP_E_NOT_CONVERGED, "policy evaluation did not converge after " + std::to_string(esweeps) +
                                            " sweeps:" + who);
        }
    }
    st.eval_sweeps += esweeps;
    k::select_final(s, a, xe0, xe1, ipar, 2);
    double* ival = c->d_init_val.as<double>();
    k::gather_init(s, n, c->d_init_idx.as<int64_t>(), xe0, ival);
    std::vector<double> vals((size_t)2 * n);
    MORAP_HIP(hipMemcpyAsync(vals.data(), ival, vals.size() * 8, hipMemcpyDeviceToHost, s));
    MORAP_HIP(hipEventRecord(wall.b, s));
    MORAP_HIP(hipEventSynchronize(wall.b));
    const float ms = wall.elapsed_ms();

    if (r_out) {
        std::fill(r_out, r_out + (size_t)K * d, 0.0);
        for (int kk = 0; kk < K; ++kk)
            for (int j = 0; j < nJ; ++j) {
                const int q = kk * nJ + j;
                if (team) {
                    r_out[(size_t)kk * d + 2 * j] = vals[2 * q];
                    if (2 * j + 1 < d) r_out[(size_t)kk * d + 2 * j + 1] = vals[2 * q + 1];
                    continue;
                }
                r_out[(size_t)kk * d + nI + j] = vals[2 * q + 1];
                r_out[(size_t)kk * d + assign[q]] += vals[2 * q];
            }
    }
    c->eK = K;
    c->evaluated = true;
    // keep the final values and the layout for a warm start of the next one
    std::swap(c->d_xe_prev.p, c->d_xe[0].p);
    std::swap(c->d_xe_prev.bytes, c->d_xe[0].bytes);
    std::swap(c->d_xe_prev.meter, c->d_xe[0].meter);
    c->prev_inst_base = c->inst_base;
    c->prev_inst_m = c->inst_m;
    c->prev_per_col = nJ;
    c->prev_eval_gen = c->load_gen;
    c->eval_prev_valid = true;
    st.ms_eval += ms;
    st.ms_total += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// ---------------------------------------------------------------------------
// the assignment check after an FP32 solve
// ---------------------------------------------------------------------------
// FP64 value iteration (to eps_vi, instance-major over the block form, from
// the FP32 values) of the (column k, model m) pairs listed; returns each
// pair's value at its model's initial state for the column's own weights.
// Uses buffers of its own: the last evaluation stays readable.
static std::vector<double> resolve_pairs(morap_ctx* c, const std::vector<int32_t>& pk,
                                         const std::vector<int32_t>& pm, const morap_vi_opts& o, Stats& st) {
    const int n = (int)pk.size();
    const int nI = c->hm.nI, nJ = c->hm.nJ, d = nI + nJ;
    hipStream_t s = c->stream;
    std::vector<int64_t> base(n + 1, 0), init_idx(n, -1);
    std::vector<int32_t> tiles;
    std::vector<double> iwc(n), iwp(n), iscale(n, 0.0);
    for (int q = 0; q < n; ++q) {
        const int m = pm[q], i = m / nJ, j = m % nJ;
        const int S_m = c->hm.state_base[m + 1] - c->hm.state_base[m];
        base[q + 1] = base[q] + S_m;
        for (int b = 0; b < S_m; b += 256) {
            tiles.push_back(q);
            tiles.push_back(b);
        }
        iwc[q] = c->W[(size_t)pk[q] * d + i];
        iwp[q] = c->W[(size_t)pk[q] * d + nI + j];
        const double sc = iwc[q] + iwp[q];
        if (sc > 0) {
            iwc[q] /= sc;
            iwp[q] /= sc;
            iscale[q] = 1.0 / sc;
        }
        if (c->hm.init[m] >= 0) init_idx[q] = base[q] + (c->hm.init[m] - c->hm.state_base[m]);
    }
    const int64_t NS = base[n];
    c->d_cand_model.ensure((size_t)n * 4);
    c->d_cand_k.ensure((size_t)n * 4);
    c->d_cand_base.ensure((size_t)(n + 1) * 8);
    c->d_cand_tiles.ensure(tiles.size() * 4 + 8);
    c->d_cand_iwc.ensure((size_t)n * 8);
    c->d_cand_iwp.ensure((size_t)n * 8);
    c->d_cand_iscale.ensure((size_t)n * 8);
    c->d_cand_x0.ensure((size_t)NS * 8 + 8);
    c->d_cand_x1.ensure((size_t)NS * 8 + 8);
    c->d_cand_res.ensure((size_t)n * 8);
    c->d_cand_act.ensure((size_t)n);
    c->d_cand_par.ensure((size_t)n);
    c->d_cand_init.ensure((size_t)n * 8);
    c->d_cand_val.ensure((size_t)n * 8);
    MORAP_HIP(hipMemcpyAsync(c->d_cand_model.p, pm.data(), (size_t)n * 4, hipMemcpyHostToDevice, s));
    MORAP_HIP(hipMemcpyAsync(c->d_cand_k.p, pk.data(), (size_t)n * 4, hipMemcpyHostToDevice, s));
    MORAP_HIP(hipMemcpyAsync(c->d_cand_base.p, base.data(), (size_t)(n + 1) * 8, hipMemcpyHostToDevice, s));
    MORAP_HIP(hipMemcpyAsync(c->d_cand_tiles.p, tiles.data(), tiles.size() * 4, hipMemcpyHostToDevice, s));
    MORAP_HIP(hipMemcpyAsync(c->d_cand_iwc.p, iwc.data(), (size_t)n * 8, hipMemcpyHostToDevice, s));
    MORAP_HIP(hipMemcpyAsync(c->d_cand_iwp.p, iwp.data(), (size_t)n * 8, hipMemcpyHostToDevice, s));
    MORAP_HIP(hipMemcpyAsync(c->d_cand_iscale.p, iscale.data(), (size_t)n * 8, hipMemcpyHostToDevice, s));
    MORAP_HIP(hipMemcpyAsync(c->d_cand_init.p, init_idx.data(), (size_t)n * 8, hipMemcpyHostToDevice, s));
    k::InstArgs a = inst_args(c, (int)(tiles.size() / 2), n);
    a.inst_model = c->d_cand_model.as<int32_t>();
    a.inst_k = c->d_cand_k.as<int32_t>();
    a.inst_base = c->d_cand_base.as<int64_t>();
    a.inst_tiles = c->d_cand_tiles.as<int32_t>();
    double* x0 = c->d_cand_x0.as<double>();
    double* x1 = c->d_cand_x1.as<double>();
    unsigned long long* res = c->d_cand_res.as<unsigned long long>();
    uint8_t* act = c->d_cand_act.as<uint8_t>();
    uint8_t* par = c->d_cand_par.as<uint8_t>();
    int64_t* dctr = c->d_counters.as<int64_t>();
    int64_t* h = c->h_counters.as<int64_t>();
    k::warm_start(s, a, c->vmain.x[0].p, c->vmain.x[1].p, c->vmain.final_par.as<uint8_t>(), c->vmain.Kp,
                  c->d_cand_iscale.as<double>(), c->d_cand_iwc.as<double>(), x0);
    k::fill_f64(s, x1, 0.0, NS);
    k::set_active(s, n, a, act, res, par, 1);
    const int chunk = std::max(2, (o.check_every + 1) / 2 * 2);
    int64_t sweeps = 0;
    while (true) {
        for (int i = 0; i < chunk; ++i) {
            const bool even = (i & 1) == 0;
            k::inst_vi_sweep(s, a, c->d_blk_rec.as<int32_t>(), c->d_blk64.as<double>(), c->d_cand_iwc.as<double>(),
                             c->d_cand_iwp.as<double>(), act, even ? x0 : x1, even ? x1 : x0, res, (int32_t)c->S,
                             c->hm.blk_pattern);
            k::inst_converge(s, n, res, act, par, even ? 1 : 0, o.eps_vi, dctr);
        }
        sweeps += chunk;
        read_counters(c);
        if (h[0] == 0) break;
        MORAP_CHECK(sweeps < o.max_sweeps, MORAP_E_NOT_CONVERGED,
                    "value iteration of the pairs of the assignment check did not converge");
    }
    k::select_final(s, a, x0, x1, par, 1);
    k::gather_values(s, n, c->d_cand_init.as<int64_t>(), x0, c->d_cand_val.as<double>());
    std::vector<double> out(n);
    MORAP_HIP(hipMemcpyAsync(out.data(), c->d_cand_val.p, (size_t)n * 8, hipMemcpyDeviceToHost, s));
    MORAP_HIP(hipStreamSynchronize(s));
    for (int q = 0; q < n; ++q) out[q] = iscale[q] > 0 ? out[q] / iscale[q] : 0.0;
    st.polish_sweeps += sweeps;
    return out;
}

// The assignment of each column was taken on FP32 values c.  Their error on
// the column's assigned pairs, e_k, is known from the FP64 re-solve; every
// unassigned pair whose slack (the value an assignment using it gives up,
// from the optimal duals) is at most 2 e_k could enter a better assignment
// once corrected by that much, so it is re-solved in FP64 too.  The column
// is then assigned again on c with the FP64 values of all these pairs; it
// takes the new assignment when that raises its value by more than 1e-9 of
// it.
// Returns the number of columns that changed (their assignments in out).
static int refine_assignment(morap_ctx* c, const int32_t* assign, int K, const morap_vi_opts& o, Stats& st,
                             int32_t* out) {
    const int nI = c->hm.nI, nJ = c->hm.nJ, M = c->hm.M;
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<double> C((size_t)K * M);
    MORAP_HIP(hipMemcpy(C.data(), c->vmain.c.p, C.size() * 8, hipMemcpyDeviceToHost));   // [K][M]
    // the pairs to re-solve, per column (columns on host threads)
    std::vector<std::vector<int32_t>> cand(K);
    std::atomic<int> next{0};
    auto worker = [&] {
        std::vector<double> slack((size_t)M);
        for (int k; (k = next++) < K;) {
            const double* ck = C.data() + (size_t)k * M;
            double e = 0, cmax = 0;
            for (int j = 0; j < nJ; ++j) {
                const int m = assign[(size_t)k * nJ + j] * nJ + j;
                e = std::max(e, std::fabs(ck[m] - c->last_c64[(size_t)k * nJ + j]));
            }
            for (int m = 0; m < M; ++m) cmax = std::max(cmax, std::fabs(ck[m]));
            const double theta = 2.0 * e + 1e-12 * std::max(1.0, cmax);
            assignment_slack(nI, nJ, ck, slack.data());
            // pairs whose two weights are 0 have the value 0 in any precision
            const double* w = c->W.data() + (size_t)k * (nI + nJ);
            for (int i = 0; i < nI; ++i)
                for (int j = 0; j < nJ; ++j)
                    if (assign[(size_t)k * nJ + j] != i && slack[(size_t)i * nJ + j] <= theta &&
                        w[i] + w[nI + j] > 0)
                        cand[k].push_back(i * nJ + j);
        }
    };
    {
        const int nt = std::max(1, std::min<int>(K, (int)std::min(16u, std::thread::hardware_concurrency())));
        std::vector<std::thread> th;
        for (int t = 1; t < nt; ++t) th.emplace_back(worker);
        worker();
        for (auto& t : th) t.join();
    }
    std::vector<int32_t> pk, pm;
    for (int k = 0; k < K; ++k)
        for (int32_t m : cand[k]) {
            pk.push_back(k);
            pm.push_back(m);
        }
    st.refine_pairs += (int64_t)pk.size();
    const auto t1 = std::chrono::steady_clock::now();
    if (pk.empty()) return 0;
    const std::vector<double> v = resolve_pairs(c, pk, pm, o, st);
    if (std::getenv("MORAP_PROGRESS"))
        std::fprintf(stderr, "[morap] assignment check: %zu pairs re-solved; slacks %.1f ms, re-solve %.1f ms\n",
                     pk.size(), std::chrono::duration<double, std::milli>(t1 - t0).count(),
                     std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t1).count());
    // c with the FP64 values of the assigned and the re-solved pairs
    for (int k = 0; k < K; ++k)
        for (int j = 0; j < nJ; ++j)
            C[(size_t)k * M + assign[(size_t)k * nJ + j] * nJ + j] = c->last_c64[(size_t)k * nJ + j];
    for (size_t q = 0; q < pk.size(); ++q) C[(size_t)pk[q] * M + pm[q]] = v[q];
    std::vector<int32_t> A((size_t)K * nJ);
    assign_columns(nI, nJ, C.data(), K, A.data());
    int changed = 0;
    for (int k = 0; k < K; ++k) {
        const double* ck = C.data() + (size_t)k * M;
        double v_old = 0, v_new = 0;
        for (int j = 0; j < nJ; ++j) {
            v_old += ck[assign[(size_t)k * nJ + j] * nJ + j];
            v_new += ck[A[(size_t)k * nJ + j] * nJ + j];
        }
        // gains below 1e-9 of the column's value are under the accuracy of
        // the FP64 values themselves (each stops at eps_vi)
        if (v_new > v_old + 1e-9 * std::max(1.0, std::fabs(v_old))) {
            std::copy(A.begin() + (size_t)k * nJ, A.begin() + (size_t)(k + 1) * nJ, out + (size_t)k * nJ);
            ++changed;
        }
    }
    st.refine_columns += changed;
    return changed;
}

// ---------------------------------------------------------------------------
// stage retirement inside the iteration (the staged form of Alg. 3)
// ---------------------------------------------------------------------------
template <class T>
static void upload_vec(DevBuf& d, const std::vector<T>& h, hipStream_t s) {
    d.ensure(h.size() * sizeof(T) + 16);
    if (!h.empty()) MORAP_HIP(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

// Stage of every state of model m: the location graph has an edge q -> q'
// for every live transition from a state at q to one at q'; its strongly
// connected groups form a DAG, and a group's stage is its height there (0
// for a group with no other group below it).  Every transition therefore
// leads to the same or a lower stage.
static int model_stages(const HostModels& hm, int m, std::vector<int32_t>& stage) {
    const int32_t s0 = hm.state_base[m], s1 = hm.state_base[m + 1];
    std::vector<int32_t> locs;
    for (int32_t g = s0; g < s1; ++g) locs.push_back(hm.states_sq[(size_t)2 * g + 1]);
    std::sort(locs.begin(), locs.end());
    locs.erase(std::unique(locs.begin(), locs.end()), locs.end());
    const int L = (int)locs.size();
    if (L == 0) return 0;
    auto idx = [&](int32_t g) {
        return (int)(std::lower_bound(locs.begin(), locs.end(), hm.states_sq[(size_t)2 * g + 1]) - locs.begin());
    };
    // reachability between locations (a handful per product)
    std::vector<uint8_t> reach((size_t)L * L, 0);
    for (int a = 0; a < L; ++a) reach[(size_t)a * L + a] = 1;
    for (int32_t g = s0; g < s1; ++g) {
        const int a = idx(g);
        for (int32_t r = hm.state_row[g]; r < hm.state_row[g + 1]; ++r)
            for (int32_t e = hm.row_ptr[r]; e < hm.row_ptr[r + 1]; ++e) {
                const int32_t h = hm.col[e];
                MORAP_CHECK(h >= s0 && h < s1, MORAP_E_STATE, "a transition leaves its model");
                reach[(size_t)a * L + idx(h)] = 1;
            }
    }
    for (int q = 0; q < L; ++q)
        for (int a = 0; a < L; ++a)
            if (reach[(size_t)a * L + q])
                for (int b = 0; b < L; ++b)
                    if (reach[(size_t)q * L + b]) reach[(size_t)a * L + b] = 1;
    // heights: a location reaches strictly more locations than every
    // location strictly below it, so count order is a topological order
    std::vector<int> n_reach(L, 0), order(L), height(L, 0);
    for (int a = 0; a < L; ++a)
        for (int b = 0; b < L; ++b) n_reach[a] += reach[(size_t)a * L + b];
    for (int a = 0; a < L; ++a) order[a] = a;
    std::sort(order.begin(), order.end(), [&](int x, int y) { return n_reach[x] < n_reach[y]; });
    int top = 0;
    for (int a : order) {
        for (int b = 0; b < L; ++b)
            if (reach[(size_t)a * L + b] && !reach[(size_t)b * L + a]) height[a] = std::max(height[a], height[b] + 1);
        top = std::max(top, height[a]);
    }
    for (int32_t g = s0; g < s1; ++g) stage[g] = height[idx(g)];
    return top + 1;
}

static void build_stage_layout(morap_ctx* c) {
    StagedLayout& L = c->staged;
    if (L.gen == c->load_gen) return;
    const HostModels& hm = c->hm;
    const int M = hm.M;
    const int64_t S = hm.S();
    MORAP_CHECK(c->has_blocks, MORAP_E_UNSUPPORTED,
                "stage retirement runs on the neighbourhood-block form (products built by morap_build_products)");
    MORAP_CHECK((int64_t)hm.states_sq.size() == 2 * S, MORAP_E_UNSUPPORTED,
                "stage retirement needs the DFA location of every state");
    std::vector<int32_t> stage((size_t)S, 0);
    L.unit_base.assign(M + 1, 0);
    std::vector<int32_t> init_unit(M, -1);
    for (int m = 0; m < M; ++m) {
        L.unit_base[m + 1] = L.unit_base[m] + model_stages(hm, m, stage);
        if (hm.init[m] >= 0) init_unit[m] = L.unit_base[m] + stage[hm.init[m]];
    }
    const int U = L.unit_base[M];
    std::vector<int32_t> rows(U, 0), states(U, 0), live(U, -1);
    std::vector<int64_t> csr(U, 0);
    for (int m = 0; m < M; ++m)
        for (int32_t g = hm.state_base[m]; g < hm.state_base[m + 1]; ++g) {
            const int u = L.unit_base[m] + stage[g];
            const int32_t nr = hm.state_row[g + 1] - hm.state_row[g];
            const int64_t nnz = hm.row_ptr[hm.state_row[g + 1]] - hm.row_ptr[hm.state_row[g]];
            rows[u] += nr;
            states[u] += 1;
            // state_row + row_ptr + col (int32) + prob and two rewards (FP64)
            csr[u] += 4 + 4 * (int64_t)nr + 12 * nnz + 16 * (int64_t)nr;
            live[u] = hm.init[m] >= 0 ? 0 : -1;
        }
    // records regrouped by unit inside every tile (stable), and the unit
    // tiles, consecutive per unit
    std::vector<int32_t> rec(hm.blk_rec.size());
    std::vector<std::vector<Tile>> per_unit(U);
    for (int m = 0; m < M; ++m) {
        const int nst = L.unit_base[m + 1] - L.unit_base[m];
        std::vector<int> cnt(nst + 1);
        for (int t = c->tile_base[m]; t < c->tile_base[m + 1]; ++t) {
            const Tile& tl = c->tiles[t];
            std::fill(cnt.begin(), cnt.end(), 0);
            for (int p = tl.s_begin; p < tl.s_end; ++p) ++cnt[stage[hm.blk_rec[(size_t)p * 8 + 7]] + 1];
            for (int q = 0; q < nst; ++q) cnt[q + 1] += cnt[q];
            for (int q = 0; q < nst; ++q)
                if (cnt[q + 1] > cnt[q])
                    per_unit[L.unit_base[m] + q].push_back(
                        Tile{L.unit_base[m] + q, tl.s_begin + cnt[q], tl.s_begin + cnt[q + 1], 0});
            for (int p = tl.s_begin; p < tl.s_end; ++p) {
                const int q = stage[hm.blk_rec[(size_t)p * 8 + 7]];
                std::copy(&hm.blk_rec[(size_t)p * 8], &hm.blk_rec[(size_t)p * 8 + 8],
                          &rec[(size_t)(tl.s_begin + cnt[q]++) * 8]);
            }
        }
    }
    std::vector<Tile> tiles;
    std::vector<int32_t> tile_base(U + 1, 0);
    for (int u = 0; u < U; ++u) {
        tile_base[u] = (int32_t)tiles.size();
        tiles.insert(tiles.end(), per_unit[u].begin(), per_unit[u].end());
    }
    tile_base[U] = (int32_t)tiles.size();
    hipStream_t s = c->stream;
    upload_vec(L.tiles, tiles, s);
    upload_vec(L.tile_base, tile_base, s);
    upload_vec(L.rec, rec, s);
    upload_vec(L.rows, rows, s);
    upload_vec(L.states, states, s);
    upload_vec(L.csr, csr, s);
    upload_vec(L.live, live, s);
    upload_vec(L.unit_base_d, L.unit_base, s);
    upload_vec(L.init_unit, init_unit, s);
    MORAP_HIP(hipStreamSynchronize(s));
    L.U = U;
    L.n_tiles = (int64_t)tiles.size();
    L.gen = c->load_gen;
}

// Alg. 3 for K columns with stage retirement: each sweep backs up the
// units still active, then per (model, column) the units are taken lowest
// first and a unit retires when all lower ones have and its own change is
// <= eps_vi; its values are copied into the other buffer.  A pair's value at
// the initial state is final when the initial state's unit retires.
static void solve_staged_impl(morap_ctx* c, const double* W, int K, const morap_vi_opts& o, double* c_out,
                              Stats& st) {
    MORAP_CHECK(c->loaded, MORAP_E_STATE, "no models loaded");
    MORAP_CHECK(!c->team, MORAP_E_UNSUPPORTED, "stage retirement runs on the decentralised products");
    MORAP_CHECK(o.precision == MORAP_F32 || o.precision == MORAP_F64, MORAP_E_INVALID, "bad precision");
    MORAP_CHECK(W && K >= 1 && K <= 4096, MORAP_E_INVALID, "need 1 <= K <= 4096 weight vectors");
    MORAP_CHECK(o.eps_vi > 0 && std::isfinite(o.eps_vi), MORAP_E_INVALID, "eps_vi must be > 0");
    MORAP_CHECK(o.max_sweeps >= 1, MORAP_E_INVALID, "max_sweeps must be >= 1");
    const int nI = c->hm.nI, nJ = c->hm.nJ, M = c->hm.M, d = nI + nJ;
    check_weight_rows(W, K, d);
    const auto t0 = std::chrono::steady_clock::now();
    build_stage_layout(c);
    StagedLayout& L = c->staged;
    const int U = L.U, Kp = padded_k(K), prec = o.precision;
    const size_t el = prec == MORAP_F32 ? 4 : 8;
    // a neighbourhood-block sweep: the one the autotuner chose for plain FP64
    // solves of this width if it is one, else the first with k-tiles of
    // min(Kp, 64) columns (the wave-per-state one where it fits)
    const Variant* v = nullptr;
    if (o.schedule > 0) {
        MORAP_CHECK(o.schedule <= (int)variants().size(), MORAP_E_INVALID, "unknown sweep variant");
        v = &variants()[o.schedule - 1];
        MORAP_CHECK(v->kind == SWEEP_BLOCK && Kp % kt_of(*v) == 0, MORAP_E_UNSUPPORTED,
                    "stage retirement runs a neighbourhood-block sweep whose k-tile divides the padded width");
    } else {
        const int64_t key = ((int64_t)prec << 40) | Kp;
        for (auto& t : c->tuned)
            if (t.first == key && variant_by_id(t.second).kind == SWEEP_BLOCK) v = &variant_by_id(t.second);
        if (!v)
            for (const auto& x : variants())
                if (x.kind == SWEEP_BLOCK && kt_of(x) == std::min(Kp, 64) &&
                    (!v || (x.cpl == 1 && x.lps == 64 && x.unroll == 2)))
                    v = &x;
    }
    MORAP_CHECK(v, MORAP_E_UNSUPPORTED, "no neighbourhood-block sweep for this width");
    hipStream_t s = c->stream;
    c->solved = false;
    c->evaluated = false;
    ensure_scratch(c, Kp);
    c->K = K;
    c->Kp = Kp;
    c->prec = prec;
    c->W.assign(W, W + (size_t)K * d);
    ValueSet& vs = c->vmain;
    ensure_values(c, vs, K, Kp, prec);

    const size_t pairs = (size_t)U * Kp;
    L.active.ensure(pairs);
    L.res.ensure(pairs * 8);
    L.ymax.ensure(pairs * 8);
    L.wc.ensure(pairs * el);
    L.wp.ensure(pairs * el);
    L.final_par.ensure(pairs);
    L.pair_sweeps.ensure(pairs * 4);
    L.best_res.ensure(pairs * 8);
    L.stall.ensure(pairs * 4);
    L.c_units.ensure((size_t)K * U * 8);
    L.model_active.ensure(U);
    L.act_models.ensure((size_t)U * 4 + 4);
    L.act_prefix.ensure((size_t)(U + 1) * 4 + 4);
    L.act_tiles.ensure((size_t)L.n_tiles * 4 + 4);
    L.retired.ensure(pairs * 8);
    L.counters.ensure(11 * 8);
    {
        std::vector<double> wc(pairs, 0.0), wp(pairs, 0.0);
        for (int m = 0; m < M; ++m) {
            const int i = m / nJ, j = m % nJ;
            for (int u = L.unit_base[m]; u < L.unit_base[m + 1]; ++u)
                for (int k = 0; k < K; ++k) {
                    wc[(size_t)u * Kp + k] = W[(size_t)k * d + i];
                    wp[(size_t)u * Kp + k] = W[(size_t)k * d + nI + j];
                }
        }
        std::vector<float> wc32, wp32;
        if (prec == MORAP_F32) {
            wc32.assign(wc.begin(), wc.end());
            wp32.assign(wp.begin(), wp.end());
        }
        MORAP_HIP(hipMemcpyAsync(L.wc.p, prec == MORAP_F32 ? (const void*)wc32.data() : (const void*)wc.data(),
                                 pairs * el, hipMemcpyHostToDevice, s));
        MORAP_HIP(hipMemcpyAsync(L.wp.p, prec == MORAP_F32 ? (const void*)wp32.data() : (const void*)wp.data(),
                                 pairs * el, hipMemcpyHostToDevice, s));
        MORAP_HIP(hipStreamSynchronize(s));
    }
    const int64_t nx = (c->S + 1) * Kp;
    if (prec == MORAP_F32) {
        k::fill_f32(s, vs.x[0].as<float>(), 0.f, nx);
        k::fill_f32(s, vs.x[1].as<float>(), 0.f, nx);
    } else {
        k::fill_f64(s, vs.x[0].as<double>(), 0.0, nx);
        k::fill_f64(s, vs.x[1].as<double>(), 0.0, nx);
    }
    k::fill_f64(s, vs.c.as<double>(), 0.0, (int64_t)K * M);
    k::fill_u8(s, vs.final_par.as<uint8_t>(), 0, (int64_t)M * Kp);
    k::fill_i32(s, c->d_pair_sweeps.as<int32_t>(), 0, (int64_t)M * Kp);
    k::fill_i64(s, L.counters.as<int64_t>(), 0, 11);

    // the units as models of the active-set machinery
    k::ConvergeArgs ca{};
    ca.res = L.res.as<unsigned long long>();
    ca.ymax = L.ymax.as<unsigned long long>();
    ca.active = L.active.as<uint8_t>();
    ca.final_par = L.final_par.as<uint8_t>();
    ca.pair_sweeps = L.pair_sweeps.as<int32_t>();
    ca.model_active = L.model_active.as<uint8_t>();
    ca.c = L.c_units.as<double>();
    ca.init = L.live.as<int32_t>();
    ca.x_out = vs.x[1].p;
    ca.counters = L.counters.as<int64_t>();
    ca.M = U;
    ca.K = K;
    ca.Kp = Kp;
    ca.prec = prec;
    ca.out_par = 1;
    ca.eps = o.eps_vi;
    // the stop rule of the plain solve (FP32: a few units in the last place,
    // and the rounding floor, R12)
    ca.unit = prec == MORAP_F32 ? 8.0 * std::ldexp(1.0, -24) : 8.0 * std::ldexp(1.0, -53);
    ca.best_res = L.best_res.as<double>();
    ca.stall = L.stall.as<int32_t>();
    ca.tile_base = L.tile_base.as<int32_t>();
    ca.act_models = L.act_models.as<int32_t>();
    ca.act_prefix = L.act_prefix.as<int32_t>();
    ca.rows_per_model = L.rows.as<int32_t>();
    ca.states_per_model = L.states.as<int32_t>();
    ca.csr_bytes = L.csr.as<int64_t>();
    ca.act_tiles = L.act_tiles.as<int32_t>();
    k::init_solve(s, ca);

    k::StageArgs sa{};
    sa.unit_base = L.unit_base_d.as<int32_t>();
    sa.init_unit = L.init_unit.as<int32_t>();
    sa.init = c->d_init.as<int32_t>();
    sa.rows = L.rows.as<int32_t>();
    sa.states = L.states.as<int32_t>();
    sa.active = ca.active;
    sa.res = ca.res;
    sa.ymax = ca.ymax;
    sa.model_active = ca.model_active;
    sa.c = vs.c.as<double>();
    sa.final_par = vs.final_par.as<uint8_t>();
    sa.pair_sweeps = c->d_pair_sweeps.as<int32_t>();
    sa.retired = L.retired.as<int64_t>();
    sa.counters = ca.counters;
    sa.tiles = L.tiles.as<Tile>();
    sa.tile_base = ca.tile_base;
    sa.rec = L.rec.as<int32_t>();
    sa.M = M;
    sa.K = K;
    sa.Kp = Kp;
    sa.eps = o.eps_vi;
    sa.unit = ca.unit;
    sa.prec = prec;
    sa.best_res = ca.best_res;
    sa.stall = ca.stall;
    sa.stall_sweeps = prec == MORAP_F32 ? 64 : 0;
    sa.floor = 256.0 * std::ldexp(1.0, -24);

    k::SweepArgs a = sweep_args(c, vs, 0);
    a.tiles = L.tiles.as<Tile>();
    a.tile_base = ca.tile_base;
    a.act_models = ca.act_models;
    a.act_prefix = ca.act_prefix;
    a.counters = ca.counters;
    a.wc = L.wc.p;
    a.wp = L.wp.p;
    a.active = ca.active;
    a.res = ca.res;
    a.ymax = ca.ymax;
    a.rec = sa.rec;
    a.act_tiles = ca.act_tiles;
    const int grid = persistent_grid(c, prec, *v);
    const int ktiles = Kp / kt_of(*v);
    const int check = std::max(2, o.check_every);
    int64_t h[11] = {0};
    EventPair wall;
    MORAP_HIP(hipEventRecord(wall.a, s));
    for (int n = 0;; ++n) {
        const int in_par = n & 1;
        a.x_in = vs.x[in_par].p;
        a.x_out = vs.x[1 - in_par].p;
        EventPair* ev = nullptr;
        std::unique_ptr<EventPair> timed;
        if (o.time_kernels) {
            timed.reset(new EventPair());
            ev = timed.get();
            MORAP_HIP(hipEventRecord(ev->a, s));
        }
        k::sweep_block(s, prec, *v, grid, ktiles, a);
        if (ev) MORAP_HIP(hipEventRecord(ev->b, s));
        sa.x_in = vs.x[in_par].p;
        sa.x_out = vs.x[1 - in_par].p;
        sa.out_par = 1 - in_par;
        sa.slot = 9 + (n & 1);
        k::stage_converge(s, sa);
        k::stage_copy(s, sa);
        k::compact(s, ca);
        if (ev) {
            MORAP_HIP(hipEventSynchronize(ev->b));
            st.ms_sweep_kernel += ev->elapsed_ms();
            st.sweep_launches += 1;
        }
        if ((n + 1) % check == 0 || n + 1 >= o.max_sweeps) {
            MORAP_HIP(hipMemcpyAsync(h, L.counters.p, sizeof(h), hipMemcpyDeviceToHost, s));
            MORAP_HIP(hipStreamSynchronize(s));
            if (h[3] == 0) break;
            if (n + 1 >= o.max_sweeps)
                fail(MORAP_E_NOT_CONVERGED, "value iteration with stage retirement: " + std::to_string(h[3]) +
                                                " (unit, column) pairs still active after " +
                                                std::to_string(n + 1) + " sweeps");
        }
    }
    MORAP_HIP(hipEventRecord(wall.b, s));
    MORAP_HIP(hipEventSynchronize(wall.b));
    std::vector<int32_t> ps((size_t)M * Kp);
    MORAP_HIP(hipMemcpy(ps.data(), c->d_pair_sweeps.p, ps.size() * 4, hipMemcpyDeviceToHost));
    st.backups += h[4];
    st.sweeps += h[5];
    st.bytes += (double)h[6] + 2.0 * (double)el * (double)h[7];
    st.floor_stops += h[8];
    st.max_pair_sweeps = std::max<int64_t>(st.max_pair_sweeps, *std::max_element(ps.begin(), ps.end()));
    st.ms_vi += wall.elapsed_ms();
    st.variant = v->id;
    if (c_out) MORAP_HIP(hipMemcpy(c_out, vs.c.p, (size_t)K * M * 8, hipMemcpyDeviceToHost));
    st.ms_total += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    vs.valid = true;
    c->solved = true;
}

void solve_staged(morap_ctx* c, const double* W, int K, const morap_vi_opts& o, double* c_out, Stats& st) {
    Stats local;
    solve_staged_impl(c, W, K, o, c_out, local);
    add_stats(st, local);
    add_stats(c->cum, local);
}

}  // namespace morap
