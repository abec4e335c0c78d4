// Internal declarations of libmorap: context, device arena, error handling,
// kernel launch wrappers.  Not part of the ABI (include/morap.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/morap.h"

namespace morap {

// ---------------------------------------------------------------------------
// errors: internal code throws MorapError; the ABI layer turns it into a
// return code and keeps the message on the context.
// ---------------------------------------------------------------------------
struct MorapError : std::runtime_error {
    int code;
    MorapError(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] inline void fail(int code, const std::string& msg) { throw MorapError(code, msg); }

#define MORAP_HIP(call)                                                                 \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            ::morap::fail(MORAP_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define MORAP_CHECK(cond, code, msg) \
    do {                             \
        if (!(cond)) ::morap::fail(code, msg); \
    } while (0)

// ---------------------------------------------------------------------------
// device buffers
// ---------------------------------------------------------------------------
// Device bytes held by a context and its optional budget (0 = none).  The
// context's meter is current on the thread during every call on it, and each
// buffer remembers the meter that paid for it.
struct AllocMeter {
    int64_t budget = 0, used = 0;
};
extern thread_local AllocMeter* g_meter;

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    AllocMeter* meter = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        if (p && meter) meter->used -= (int64_t)bytes;
        p = nullptr;
        bytes = 0;
        meter = nullptr;
    }
    // (re)allocate when the requested size exceeds the current one; true
    // when the buffer moved.  Over the context's budget: OOM, buffer released.
    bool ensure(size_t n) {
        if (n <= bytes && p) return false;
        release();
        if (n == 0) n = 16;
        AllocMeter* m = g_meter;
        if (m && m->budget > 0 && m->used + (int64_t)n > m->budget)
            fail(MORAP_E_OOM, "device memory budget of " + std::to_string(m->budget) + " bytes exceeded (" +
                                  std::to_string(m->used) + " held, " + std::to_string(n) + " more requested)");
        hipError_t e = hipMalloc(&p, n);
        if (e != hipSuccess) {
            p = nullptr;
            fail(MORAP_E_OOM, "hipMalloc of " + std::to_string(n) + " bytes failed: " + hipGetErrorString(e));
        }
        bytes = n;
        meter = m;
        if (m) m->used += (int64_t)n;
        return true;
    }
    template <class T> T* as() const { return static_cast<T*>(p); }
};

struct PinnedBuf {
    void* p = nullptr;
    size_t bytes = 0;
    ~PinnedBuf() { if (p) (void)hipHostFree(p); }
    void ensure(size_t n) {
        if (n <= bytes && p) return;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        MORAP_HIP(hipHostMalloc(&p, n, hipHostMallocDefault));
        bytes = n;
    }
    template <class T> T* as() const { return static_cast<T*>(p); }
};

// ---------------------------------------------------------------------------
// host-side model set (concatenated CSR with global indices)
// ---------------------------------------------------------------------------
struct HostModels {
    int nI = 0, nJ = 0, M = 0;
    std::vector<int32_t> state_base;   // [M+1] first global state of each model
    std::vector<int32_t> init;         // [M] global index of the initial state, -1 if done
    std::vector<int32_t> state_row;    // [S+1] global rows
    std::vector<int32_t> row_ptr;      // [R+1] global entries
    std::vector<int32_t> col;          // [N] global states
    std::vector<double>  prob;         // [N]
    std::vector<double>  rew;          // [2R]
    std::vector<uint8_t> to_done;      // [R]
    std::vector<int32_t> states_sq;    // [2S] (agent state, location), may be empty
    // neighbourhood-block form (products built from agents and automata whose
    // agent states have at most 5 actions and 5 distinct successors, the
    // state itself counted): per product state 8 int32
    //   [0..4] global successor state of agent slot d (S = the zero row:
    //          slot unused, or its successor is done), slot 0 = the agent
    //          state itself; [5] index of its agent state's block; [6] bits 0-4: slot
    //          d enters an accepting location, bits 8-12: action a enabled;
    //          [7] the record's own state (records are stored tile by tile,
    //          each tile's in the order the sweep walks it);
    // and per distinct agent-state block 32 values: P[a][d] (a-major, 25), -cost[a] (5), 0, 0,
    // where a disabled action repeats the first enabled one.
    // halo tiles (built with the block form): [4 * tiles] HTile fields, the
    // first tile of each model, per record position (tile by tile) two words
    //   w0 = halo place of slots 0..3 (8 bits each), w1 = slot 4 | accepting
    //   slots << 8 | block << 13   (HALO_MAX = the zero row),
    // and the halo lists (global states)
    std::vector<int32_t> hal_tile, hal_tile_base, hal_list;
    std::vector<uint32_t> hal_rec;
    std::vector<int32_t> blk_rec;      // [8S]
    std::vector<double>  blk_agent;    // [32 * distinct blocks]
    uint32_t blk_pattern = 0;          // bit 5a + d: some block has P[a][d] != 0
    int64_t S() const { return (int64_t)state_row.size() - 1; }
    int64_t R() const { return (int64_t)row_ptr.size() - 1; }
    int64_t N() const { return (int64_t)col.size(); }
};

// A tile is a run of consecutive states of one model whose rows and entries
// fit the LDS staging area of the sweep kernel.
struct Tile {
    int32_t model, s_begin, s_end, pad;
};

// A halo tile of the LDS-staged sweep: at most HALO_TILE states of one model
// whose value rows (own states and successors) number at most HALO_MAX.
// Its records are hal_rec[rec_begin .. rec_begin + n), its halo list
// hal_list[halo_begin .. halo_begin + H) (own states first, in record order).
#ifndef MORAP_HALO_TILE
#define MORAP_HALO_TILE 64
#endif
#ifndef MORAP_HALO_MAX
#define MORAP_HALO_MAX 96
#endif
constexpr int HALO_TILE = MORAP_HALO_TILE;
constexpr int HALO_MAX = MORAP_HALO_MAX;   // < 256: halo places are bytes
static_assert(HALO_MAX < 256 && HALO_TILE <= HALO_MAX && HALO_TILE <= 128, "halo tile limits");
struct HTile {
    int32_t model, rec_begin, n, halo_begin;   // n = states | H << 16
};

// sweep-kernel variants: kernel family x columns per lane x lanes per state
enum { SWEEP_CSR = 0, SWEEP_BLOCK = 1, SWEEP_HALO = 2 };
struct Variant {
    int id;        // > 0
    int cpl;       // columns per lane
    int lps;       // lanes per state
    int wg;        // threads per workgroup
    int kind;      // SWEEP_CSR (LDS-staged CSR tiles), SWEEP_BLOCK (neighbourhood blocks) or
                   // SWEEP_HALO (neighbourhood blocks, halo rows staged in LDS)
    int unroll;    // states in flight per lane group (block sweeps)
};

struct Stats {
    int64_t backups = 0, sweeps = 0, max_pair_sweeps = 0, eval_sweeps = 0, polish_sweeps = 0,
            rank_rounds = 0, floor_stops = 0;
    double bytes = 0, ms_vi = 0, ms_eval = 0, ms_total = 0, ms_sweep_kernel = 0;
    int64_t sweep_launches = 0;
    double bytes_refine = 0, ms_sweep_kernel_refine = 0;
    int64_t sweep_launches_refine = 0;
    int variant = 0, variant_refine = 0;
    // the last sweeps of batched solves, run by the LDS-staged kernel
    int64_t sweeps_tail = 0, sweep_launches_tail = 0;
    double bytes_tail = 0, ms_sweep_kernel_tail = 0;
    int variant_tail = 0;
    // the assignment check after FP32 solves: pairs re-solved, columns reassigned
    int64_t refine_pairs = 0, refine_columns = 0;
};

// Values of one batched value iteration: two Jacobi buffers [S][Kp], the
// buffer holding each (model, column) pair's result, and the value at every
// model's initial state.
struct ValueSet {
    DevBuf x[2];
    DevBuf final_par;   // [M][Kp] uint8
    DevBuf c;           // [K][M] FP64
    int prec = -1, K = 0, Kp = 0;
    bool valid = false;
};

struct Proposer;  // mlp.hip

// Stage retirement inside the iteration (the staged form of Alg. 3): the
// states of every model split by stage (the height of their location group
// in the product's location DAG) into units, lowest stage first, with the
// neighbourhood-block records reordered inside each tile so that a unit's
// records form runs; the tiles of a unit are consecutive.
struct StagedLayout {
    uint64_t gen = ~0ull;                 // model upload the layout belongs to
    int U = 0;                            // units
    int64_t n_tiles = 0;
    std::vector<int32_t> unit_base;       // [M+1] first unit of each model
    DevBuf tiles, tile_base, rec;         // unit tiles, [U+1], records [8S]
    DevBuf rows, states, csr, live;       // [U] rows, states, CSR bytes (FP64), 0 / -1 (dead model)
    DevBuf unit_base_d, init_unit;        // [M+1], [M] unit of the initial state (-1: done)
    // solve state
    DevBuf active, res, ymax, wc, wp, final_par, pair_sweeps, best_res, stall;   // [U][Kp]
    DevBuf c_units;                       // [K][U] (cleared at the start, unused)
    DevBuf model_active, act_models, act_prefix, act_tiles, retired, counters;
};

}  // namespace morap

// ---------------------------------------------------------------------------
// the context
// ---------------------------------------------------------------------------
struct morap_ctx {
    morap::AllocMeter meter;                        // first member: outlives every buffer
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;
    hipDeviceProp_t prop{};

    // models
    morap::HostModels hm;
    bool loaded = false;
    int64_t S = 0, R = 0, N = 0;
    int max_rows_per_state = 0;
    bool has_blocks = false;                        // the neighbourhood-block form exists
    morap::DevBuf d_blk_rec, d_blk32, d_blk64;
    bool team = false;                              // a team MDP with per-row objectives is loaded
    int team_nI = 0, team_nJ = 0;                   // its agents and tasks (d = team_nI + team_nJ)
    morap::DevBuf d_obj;                            // [R][2] objective of each reward of a row
    morap::DevBuf d_rewk32, d_rewk64, d_team_w;     // [R][Kp] scalarised rewards, [K][d] weights
    morap::DevBuf d_inst_obj;                       // [instances][2] objectives an instance evaluates
    morap::DevBuf d_team_pi;                        // [S] global row of a fixed proper policy
    morap::DevBuf d_team_E;                         // [S][d] its value per objective (the start of a solve)
    bool has_halo = false;                          // halo tiles exist
    morap::DevBuf d_htiles, d_htile_base, d_hrec, d_hlist;
    int64_t n_htiles = 0;
    morap::DevBuf d_state_row, d_row_ptr, d_col, d_prob32, d_prob64, d_rew32, d_rew64, d_to_done;
    morap::DevBuf d_state_base, d_init;
    morap::DevBuf d_state_model;                    // [S] model of every state
    morap::DevBuf d_xwarm, d_warm_map, d_warm_ab;    // warm start of a solve: values [S+1][Kp], column map,
                                                     // per-pair start a x + b [M][Kp][2]
    morap::DevBuf d_rows_per_model, d_states_per_model;  // [M] int32
    morap::DevBuf d_csr_bytes32, d_csr_bytes64;          // [M] int64: CSR bytes read per sweep

    // tiles of the batched sweep (built for the LDS limits below)
    std::vector<morap::Tile> tiles;
    std::vector<int32_t> tile_base;                 // [M+1] first tile of each model
    morap::DevBuf d_tiles, d_tile_base;

    // solve state (batched value iteration)
    int K = 0, Kp = 0, prec = -1;
    bool solved = false;
    morap::ValueSet vmain;                          // the solve's values (its precision)
    morap::ValueSet vref;                           // FP64 values of the assigned pairs after an FP32 solve
    morap::DevBuf d_pair_mask;                      // [M][Kp] uint8: pairs of a restricted solve
    morap::DevBuf d_wc32, d_wp32, d_wc64, d_wp64;   // [M][Kp]
    morap::DevBuf d_res, d_ymax;                    // [M][Kp] uint64 (bits of FP64)
    morap::DevBuf d_active;                         // [M][Kp] uint8
    morap::DevBuf d_pair_sweeps;                    // [M][Kp] int32
    morap::DevBuf d_model_active;                   // [M] uint8
    morap::DevBuf d_act_models, d_act_prefix;       // compacted active model list
    morap::DevBuf d_act_tiles;                      // the active models' tiles, in order
    morap::DevBuf d_best_res, d_stall;              // [M][Kp] FP32 rounding-floor detection
    morap::DevBuf d_counters;                       // int64 [9] (see the convergence kernel)
    morap::PinnedBuf h_counters;
    morap::PinnedBuf h_log;                         // per-launch tile counts (sweep log)
    std::vector<double> W;                          // [K][d] of the last solve
    int last_variant = 0;
    std::vector<hipEvent_t> event_pool;             // reusable per-launch timing events
    // captured chunks of sweeps: main, FP64 refine, and main again for the
    // sweep kernel of a solve's last, small active sets
    hipGraph_t chunk_graph[3] = {nullptr, nullptr, nullptr};
    hipGraphExec_t chunk_exec[3] = {nullptr, nullptr, nullptr};
    std::string graph_key[3];
    uint64_t load_gen = 0;                          // bumped by every model upload (graph keys)
    uint64_t buf_gen = 0;                           // bumped when a solve buffer moves (graph keys)

    // evaluation state
    int eK = 0;
    bool evaluated = false;
    std::vector<int32_t> assign;                    // [K][nJ]
    std::vector<int32_t> inst_k, inst_m;            // instances (column, model)
    std::vector<int64_t> inst_base;                 // [n_inst+1] state offsets
    morap::DevBuf d_inst_model, d_inst_k, d_inst_base, d_inst_tiles;
    morap::DevBuf d_xi;                             // final FP64 values [inst states]
    morap::DevBuf d_ires, d_iactive, d_ipar;        // per (instance, objective)
    morap::DevBuf d_mask, d_rank, d_mu;             // per instance state
    morap::DevBuf d_xe[2];                          // evaluation values [inst states][2]
    // the last evaluation's final values and instance layout (a warm start
    // of the next one)
    morap::DevBuf d_xe_prev, d_warm_copy;
    morap::DevBuf d_iwarm;                          // per instance: warm-started (evaluation start)
    morap::DevBuf d_ieps;                           // per instance: stop of the FP64 policy values
    std::vector<int64_t> prev_inst_base;
    std::vector<int32_t> prev_inst_m;
    int prev_per_col = 0;
    bool eval_prev_valid = false;
    uint64_t prev_eval_gen = 0;
    // FP64 values at the initial states of the assigned pairs of the last
    // evaluation after an FP32 solve (valid when set), and the buffers of
    // the re-solve of other pairs for the assignment check
    std::vector<double> last_c64;
    bool last_c64_valid = false;
    morap::DevBuf d_cand_model, d_cand_k, d_cand_base, d_cand_tiles, d_cand_iwc, d_cand_iwp, d_cand_iscale;
    morap::DevBuf d_cand_x0, d_cand_x1, d_cand_res, d_cand_act, d_cand_par, d_cand_init, d_cand_val;
    morap::DevBuf d_iwc, d_iwp;                     // per instance FP64 weights
    morap::DevBuf d_iscale;                         // per instance 1 / (w_i + w_j) (warm start)
    morap::DevBuf d_ichanged;                       // per instance: ranks changed in the last round
    morap::DevBuf d_init_idx, d_init_val;           // instance initial states, their values
    morap::DevBuf d_xr;                             // second buffer of the instance value iteration
    std::vector<int32_t> h_live_tiles;              // instance tiles still active
    morap::DevBuf d_live_tiles;
    std::vector<int8_t> h_mu;                       // policies of the last evaluate

    // units of the stage-retiring solve (built on first use per upload)
    morap::StagedLayout staged;

    // autotuner cache: key (prec, Kp) -> variant id
    std::vector<std::pair<int64_t, int>> tuned;
    // resident workgroups per compute unit: key (variant, prec) -> count
    std::vector<std::pair<int64_t, int>> resident;

    // statistics since the last reset
    morap::Stats cum;

    // proposer
    morap::Proposer* prop_mlp = nullptr;
    std::vector<double> features;

    ~morap_ctx();
};

namespace morap {

// Run f with the context's device current; errors become return codes and
// the message stays on the context (no exception crosses the ABI).
template <class F>
int guarded(morap_ctx* c, F&& f) {
    if (!c) return MORAP_E_INVALID;
    struct MeterScope {   // the context pays for what the call allocates
        AllocMeter* prev;
        explicit MeterScope(AllocMeter* m) : prev(g_meter) { g_meter = m; }
        ~MeterScope() { g_meter = prev; }
    } scope(&c->meter);
    try {
        c->err.clear();
        MORAP_HIP(hipSetDevice(c->device));
        f();
        return MORAP_OK;
    } catch (const MorapError& e) {
        c->err = e.what();
        return e.code;
    } catch (const std::bad_alloc&) {
        c->err = "host allocation failed";
        return MORAP_E_OOM;
    } catch (const std::exception& e) {
        c->err = e.what();
        return MORAP_E_INVALID;
    } catch (...) {
        c->err = "unknown error";
        return MORAP_E_INVALID;
    }
}

// product.cpp
void build_products(morap_ctx* ctx, const morap_agent* agents, int nI, const morap_dfa* tasks, int nJ,
                    const int32_t* const* letters);
void load_models(morap_ctx* ctx, const morap_model* models, int n, int nI, int nJ);
// agent / automaton validation (INVALID on malformed input) and the done
// locations of an automaton (accepting, or no run reaches acceptance)
void check_agent(const morap_agent& a, int i);
void check_dfa(const morap_dfa& t, int j);
std::vector<uint8_t> dfa_done(const morap_dfa& t);
// the team MDP of Def. teamMDP scalarised for one weight vector, as a
// single-objective model (host only): sizes = {S, R, N, init}
void team_model_host(const morap_agent* agents, int n_agents, const morap_dfa* tasks, int n_tasks,
                     const int32_t* const* letters, const double* w, int32_t* sizes, int32_t* state_row,
                     int32_t* row_ptr, int32_t* col, double* prob, double* rew, uint8_t* to_done);
// the team MDP with its d = 2n objectives: per row the two rewards and the
// objective each belongs to (host only)
void team_model_mo_host(const morap_agent* agents, int n_agents, const morap_dfa* tasks, int n_tasks,
                        const int32_t* const* letters, int32_t* sizes, int32_t* state_row, int32_t* row_ptr,
                        int32_t* col, double* prob, double* rew, int32_t* obj, uint8_t* to_done);
// one product on the host (no context, no device): sizes = {S, R, N, init},
// arrays filled where non-NULL
void product_host(const morap_agent* a, const morap_dfa* t, const int32_t* letters, int32_t* sizes,
                  int32_t* state_row, int32_t* row_ptr, int32_t* col, double* prob, double* rew, uint8_t* to_done,
                  int32_t* states);
void upload_models(morap_ctx* ctx);
void load_team_model(morap_ctx* ctx, int n_agents, int n_tasks, const morap_model* model, const int32_t* obj);
// agents, tasks and objectives of the loaded models (a team model: its own)
inline int n_agents_of(const morap_ctx* c) { return c->team ? c->team_nI : c->hm.nI; }
inline int n_tasks_of(const morap_ctx* c) { return c->team ? c->team_nJ : c->hm.nJ; }
inline int n_obj_of(const morap_ctx* c) { return n_agents_of(c) + n_tasks_of(c); }

// solver.cpp
// warm (nullable, [K]): column of the previous solve each column starts from
// (-1: from 0); used when the previous solve was FP32 with at least as many
// padded columns, ignored otherwise
void solve(morap_ctx* ctx, const double* W, int K, const morap_vi_opts& o, double* c_out, Stats& st,
           const int32_t* warm = nullptr);
// the same value iteration with stage retirement inside it (FP64, block form)
void solve_staged(morap_ctx* ctx, const double* W, int K, const morap_vi_opts& o, double* c_out, Stats& st);
// warm (nullable): per column, the column of the previous evaluation whose
// instance of the same task on the same model starts the policy evaluation
// from its final values (-1: from 0, as Alg. 4)
//
// refine (nullable, FP32 solves of block-form products): the assignment
// (assign) is checked against FP64 values -- every pair whose slack lies
// within twice the column's largest FP32 error on its assigned pairs is
// re-solved in FP64, the column is assigned again on the FP64 values, and a
// column whose value rises takes the new assignment, which is then
// evaluated; refine receives the assignment evaluated
void evaluate(morap_ctx* ctx, const int32_t* assign, int K, const morap_vi_opts& o, double* r_out, Stats& st,
              const int32_t* warm = nullptr, int32_t* refine = nullptr);
const std::vector<Variant>& variants();

// assign.cpp
void assign_columns(int nI, int nJ, const double* c, int K, int32_t* out);
// one column's optimal assignment and the slack of every pair against it
std::vector<int32_t> assignment_slack(int nI, int nJ, const double* ck, double* slack);

// qp.cpp
void project_inner(const double* Phi, int m, int d, const double* t, const double* M, double* x,
                   double* lam);
void project_outer(const double* W, const double* R, int n, int d, const double* t, const double* M,
                   double* z);

// query.cpp
void query_batch(morap_ctx* ctx, const double* T, const double* W0, int Q, const double* M,
                 const morap_query_opts& o, morap_query_result* res);

// mlp.hip
void proposer_destroy(Proposer* p);
// device address of the fixed inference scratch, taken once per device
void proposer_scratch_init(int device);

// kernels (vi.hip): launch wrappers
namespace k {
void fill_u8(hipStream_t s, uint8_t* p, uint8_t v, int64_t n);
void fill_i32(hipStream_t s, int32_t* p, int32_t v, int64_t n);
void fill_u64(hipStream_t s, uint64_t* p, uint64_t v, int64_t n);
void fill_f32(hipStream_t s, float* p, float v, int64_t n);
void fill_f64(hipStream_t s, double* p, double v, int64_t n);
void fill_i64(hipStream_t s, int64_t* p, int64_t v, int64_t n);
void to_f32(hipStream_t s, const double* in, float* out, int64_t n);

struct SweepArgs {
    const Tile* tiles;
    const int32_t* tile_base;
    const int32_t* act_models;
    const int32_t* act_prefix;
    const int64_t* counters;
    const int32_t* state_row;
    const int32_t* row_ptr;
    const int32_t* col;
    const void* prob;
    const void* rew;
    const void* wc;
    const void* wp;
    const uint8_t* active;
    const void* x_in;
    void* x_out;
    unsigned long long* res;
    unsigned long long* ymax;
    int Kp;
    const int32_t* rec;     // neighbourhood-block records [8S]
    const void* ablk;       // agent blocks [32 * agent states] (precision of the sweep)
    int32_t zero_row;       // S: the value row that always holds 0
    uint32_t pattern;       // union of the blocks' nonzero (action, slot) entries
    const int32_t* act_tiles;  // global index of every active tile, in order
    const void* rewk;          // team models: scalarised reward of every (row, column) [R][Kp] (nullable)
    const HTile* htiles;       // halo tiles (LDS-staged sweep)
    const uint2* hrec;         // their records
    const int32_t* hlist;      // their halo lists
};
// batched Bellman sweep: variant v, precision prec (MORAP_F32/F64)
void sweep(hipStream_t s, int prec, const Variant& v, int grid, int ktiles, const SweepArgs& a);
void sweep_block(hipStream_t s, int prec, const Variant& v, int grid, int ktiles, const SweepArgs& a);
// workgroups of the variant's kernel that fit one compute unit at once
int sweep_resident(int prec, const Variant& v);
int sweep_block_resident(int prec, const Variant& v);
// LDS-staged sweep over halo tiles (halo.hip): FP32, k-tiles of 64 columns
void sweep_halo(hipStream_t s, int prec, const Variant& v, int grid, int ktiles, const SweepArgs& a);
int sweep_halo_resident(const Variant& v, uint32_t pattern);
int sweep_lds_rows();
int sweep_lds_nnz();
int sweep_tile_states(const Variant& v);

struct ConvergeArgs {
    unsigned long long* res;
    unsigned long long* ymax;
    uint8_t* active;
    uint8_t* final_par;
    int32_t* pair_sweeps;
    uint8_t* model_active;
    double* c;              // [K][M]
    const int32_t* init;    // [M]
    const uint8_t* mask;    // [M][Kp] pairs to solve (nullable: all)
    const void* x_out;      // buffer written by the sweep just finished
    int64_t* counters;
    int M, K, Kp, prec, out_par;
    double eps, unit;       // stop at res <= max(eps, unit * ymax)
    // FP32 rounding floor: a pair whose change has set no new minimum for
    // stall_sweeps sweeps (0: off) and is within floor * ymax stops too
    double* best_res;       // [M][Kp] smallest change so far
    int32_t* stall;         // [M][Kp] sweeps since it was set
    int stall_sweeps;
    double floor;
    const int32_t* tile_base;
    int32_t* act_models;
    int32_t* act_prefix;
    const int32_t* rows_per_model;   // [M] rows (backups per active column)
    const int32_t* states_per_model; // [M] states (value traffic per active column)
    const int64_t* csr_bytes;        // [M] CSR bytes read per sweep of an active model
    int32_t* act_tiles;              // [tiles] global index of every active tile, in order
    int relist;                      // compaction only re-lists the active models (no sweep is counted)
};
void converge(hipStream_t s, const ConvergeArgs& a);
void compact(hipStream_t s, const ConvergeArgs& a);
// the same active models listed over the tiles of a.tile_base (a change of
// sweep kernel between the gather and the LDS-staged tiles)
void relist(hipStream_t s, ConvergeArgs a);
void init_solve(hipStream_t s, const ConvergeArgs& a);

// stage retirement (staged.hip)
struct StageArgs {
    const int32_t* unit_base;   // [M+1]
    const int32_t* init_unit;   // [M] unit of the initial state, -1 if done
    const int32_t* init;        // [M] initial state
    const int32_t* rows;        // [U] rows (backups per active column)
    const int32_t* states;      // [U] states
    uint8_t* active;            // [U][Kp]
    unsigned long long* res;    // [U][Kp]
    unsigned long long* ymax;   // [U][Kp]
    uint8_t* model_active;      // [U]
    double* c;                  // [K][M] values at the initial states
    uint8_t* final_par;         // [M][Kp]
    int32_t* pair_sweeps;       // [M][Kp] sweep in which the initial state's unit retired
    int64_t* retired;           // [U * Kp] (unit, column) pairs retired in this sweep
    int64_t* counters;          // as the convergence kernel's, [9] / [10] the list counts
    const Tile* tiles;          // unit tiles
    const int32_t* tile_base;   // [U+1]
    const int32_t* rec;         // reordered block records [8S]
    const void* x_out;          // the buffer the sweep wrote (precision prec)
    void* x_in;                 // the buffer it read
    double* best_res;           // [U][Kp] FP32 rounding floor: smallest change so far
    int32_t* stall;             // [U][Kp] sweeps since it was set
    int stall_sweeps;           // 0: no floor stop (FP64)
    double floor;
    int M, K, Kp, out_par, slot, prec;   // slot: 9 or 10, the list count of this sweep
    double eps, unit;
};
void stage_converge(hipStream_t s, const StageArgs& a);
void stage_copy(hipStream_t s, const StageArgs& a);

// instances (polish, policy extraction, evaluation)
struct InstArgs {
    const int32_t* inst_model;
    const int32_t* inst_k;
    const int64_t* inst_base;
    const int32_t* inst_tiles;     // (instance, local state begin) pairs
    int n_tiles;
    int n_inst;
    const int32_t* state_base;
    const int32_t* state_row;
    const int32_t* row_ptr;
    const int32_t* col;
    const double* prob;
    const double* rew;
    const uint8_t* to_done;
    const int32_t* init;
    int cus;                       // compute units (resident-sized grids of the striding kernels)
    // team models (nullable otherwise): FP64 scalarised reward of every
    // (row, column) with its leading dimension, every row's two objectives
    // and the two objectives each instance evaluates (-1: none)
    const double* rewk;
    int rewk_ld;
    const int32_t* row_obj;
    const int32_t* inst_obj;
};
// team models: one Jacobi sweep of the per-objective evaluation of the fixed
// policy pi (E[s][o], res = max change as FP64 bits), and the start values
// x[s][k] = sum_o W[k][o] E[s][o] minus a margin (FP32 or FP64 x, [S+1][Kp])
void team_eval_sweep(hipStream_t s, int64_t S, int d, const int32_t* pi, const int32_t* row_ptr,
                     const int32_t* col, const double* prob, const double* rew, const int32_t* obj,
                     const double* E_in, double* E_out, unsigned long long* res);
void team_start(hipStream_t s, int64_t S, int K, int Kp, int d, const double* W, const double* E, int prec,
                void* x);
// out[q] = x[idx[q]] (0 where idx[q] < 0): one value per instance state
void gather_values(hipStream_t s, int n, const int64_t* idx, const double* x, double* out);
// runs (dst, src, length) of instance states [.][2] copied from prev to x
void copy_runs(hipStream_t s, const int64_t* runs, int n_runs, const double* prev, double* x);
// evaluation start from the instances' scalarised values xi (iwarm: per
// instance, 1 where its values were warm-started)
void eval_start(hipStream_t s, const InstArgs& a, const double* xi, const double* iwc, const double* iwp,
                const uint8_t* iwarm, double* xe);
// team models: out[r][k] = W[k][obj[r][0]] rew[r][0] + W[k][obj[r][1]] rew[r][1]
void team_rewards(hipStream_t s, int64_t R, int K, int Kp, int d, const double* W, const int32_t* obj,
                  const double* rew, double* out64, float* out32);
void gather_columns(hipStream_t s, const InstArgs& a, int prec, const void* x0, const void* x1,
                    const uint8_t* final_par, int Kp, double* xi);
// start of an FP32 solve from the previous one's final values: out[s][k] =
// a x_prev[s][map[k]] + b (the buffer its pair froze in; ab[m][k] = (a, b))
// where map[k] >= 0 and a != 0, 0 elsewhere (and on the zero row)
void warm_columns(hipStream_t s, int64_t S, int Kp, int K, const int32_t* map, const int32_t* state_model,
                  const float* ab, const float* x0, const float* x1, const uint8_t* final_par, int Kp_old,
                  float* out);
// FP64 start of the instances from the FP32 solve's values, scaled by
// scale[inst] (instances with a zero cost weight start from 0)
void warm_start(hipStream_t s, const InstArgs& a, const void* x0, const void* x1, const uint8_t* final_par, int Kp,
                const double* scale, const double* iwc, double* xi);
// stop test of n entries: residual <= eps, or <= eps_i[i] where eps_i is given
void inst_converge(hipStream_t s, int n, unsigned long long* res, uint8_t* active, uint8_t* par, int out_par,
                   double eps, int64_t* counter, const double* eps_i = nullptr);
void opt_mask(hipStream_t s, const InstArgs& a, const double* wc, const double* wp, const double* x,
              double tau, uint32_t* mask, int32_t* rank, int8_t* mu, bool only_unranked);
void eval_sweep(hipStream_t s, const InstArgs& a, const int8_t* mu, const uint8_t* active,
                const double* x_in, double* x_out, unsigned long long* res);
void count_unranked(hipStream_t s, const InstArgs& a, const int32_t* rank, int64_t* counter);
// attractor ranks as BFS distances (in-place relaxation sweep) and the action
// choice once they are final
void relax_ranks(hipStream_t s, const InstArgs& a, const uint32_t* mask, int32_t* rank, int base, bool reverse,
                 int local, int64_t* changed, uint8_t* inst_changed);
void choose_actions(hipStream_t s, const InstArgs& a, const uint32_t* mask, const int32_t* rank, int8_t* mu,
                    int base, int64_t* max_rank);
// per-instance flags: `width` entries per instance, active when the instance
// has a live initial state
void set_active(hipStream_t s, int n, const InstArgs& a, uint8_t* active, unsigned long long* res,
                uint8_t* par, int width);
// copy the values of entries frozen in buffer 1 into buffer 0
void select_final(hipStream_t s, const InstArgs& a, double* x0, const double* x1, const uint8_t* par,
                  int width);
// pair mask of a restricted solve: mask[m][k] = 1 for the instances' pairs
void mark_pairs(hipStream_t s, const InstArgs& a, int Kp, uint8_t* mask);
// one FP64 value-iteration sweep of instances over the neighbourhood blocks
// (block.hip); residuals per instance
void inst_vi_sweep(hipStream_t s, const InstArgs& a, const int32_t* rec, const double* ablk, const double* wc,
                   const double* wp, const uint8_t* active, const double* x_in, double* x_out,
                   unsigned long long* res, int32_t zero_row, uint32_t pattern);
// one Alg. 4 sweep (both objectives) of instances over the neighbourhood
// blocks (block.hip)
void eval_block_sweep(hipStream_t s, const InstArgs& a, const int32_t* rec, const double* ablk, const int8_t* mu,
                      const uint8_t* active, const double* x_in, double* x_out, unsigned long long* res,
                      int32_t zero_row, uint32_t pattern);
// out[2q + o] = x[2 idx[q] + o] (0 when idx[q] < 0)
void gather_init(hipStream_t s, int n, const int64_t* idx, const double* x, double* out);
}  // namespace k

}  // namespace morap
