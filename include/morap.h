/*
 * morap.h -- C ABI of libmorap, an MI355X (gfx950) engine for the batched
 * scalarised value-iteration path of point-oriented Pareto queries over
 * agent-task product MDPs (Robinson & Su, "Multi-Objective Task Assignment
 * and Multiagent Planning with Hybrid GPU-CPU Acceleration").
 *
 * Conventions shared by every entry point:
 *   - Return MORAP_OK (0) on success or a negative MORAP_E_* code.  The text
 *     of the last error of a context is available from morap_last_error().
 *     No C++ exception crosses this boundary.
 *   - Every pointer argument is a HOST pointer unless its comment says
 *     otherwise.  Buffers are owned by the caller; the library copies what it
 *     keeps and never frees caller memory.  Sizes are explicit.
 *   - Device work is enqueued on the context's stream.  Entry points that
 *     return host results synchronise that stream before returning.
 *   - A context belongs to one host thread at a time (a model is owned by one
 *     thread at a time in the paper's implementation, Sec. 4); calls on the
 *     same context from several threads at once are not allowed.
 *   - Objective order: d = |I| + |J|; objectives 0..|I|-1 are the agents'
 *     costs (as negative rewards) and |I|..d-1 the tasks' completion
 *     probabilities (Alg. 1 input t = (c, p), Def. MORAP).
 *   - Model index m = i * |J| + j for agent i and task j.
 *   - Calls without a context (morap_product_host, morap_team_model_host,
 *     morap_assign_host, morap_project_inner, morap_project_outer) run on
 *     the host only, touch no device, and report errors by their return code
 *     alone.
 */
#ifndef MORAP_H
#define MORAP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MORAP_OK               0
#define MORAP_E_INVALID       -1  /* bad argument or malformed model data          */
#define MORAP_E_OOM           -2  /* device or host allocation failed / over budget */
#define MORAP_E_NOT_CONVERGED -3  /* an iteration hit its sweep limit               */
#define MORAP_E_IMPROPER      -4  /* no policy among eps-optimal actions reaches done */
#define MORAP_E_HIP           -5  /* HIP runtime error                               */
#define MORAP_E_UNSUPPORTED   -6  /* sizes beyond what this build handles            */
#define MORAP_E_STATE         -7  /* call order (e.g. evaluate before solve)         */

#define MORAP_F64 0               /* value iteration in FP64                         */
#define MORAP_F32 1               /* FP32 backups, FP64 residual / polish / evaluation */

#define MORAP_FEASIBLE   1
#define MORAP_INFEASIBLE 0
#define MORAP_UNDECIDED  2

typedef struct morap_ctx morap_ctx;

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t
 * (NULL = the device's null stream); the caller keeps ownership of it and must
 * keep it alive until morap_destroy.  *out receives the context.
 * Errors: INVALID (out NULL, bad device), HIP. */
int morap_create(morap_ctx** out, int device, void* hip_stream);

/* Release all device and host memory of the context.  NULL is accepted. */
int morap_destroy(morap_ctx* ctx);

/* Device memory budget of the context in bytes (0 = none, the default).  An
 * allocation that would take the context's device memory beyond it fails
 * with MORAP_E_OOM, as a failed hipMalloc does; what the context already
 * holds is kept.  used_out (nullable) receives the bytes the context holds
 * now.  Errors: INVALID (negative budget). */
int morap_set_memory_budget(morap_ctx* ctx, int64_t bytes, int64_t* used_out);

/* Text of the last error on this context ("" if none).  Valid until the next
 * call on the context. */
const char* morap_last_error(const morap_ctx* ctx);

/* ---------------------------------------------------------------------------
 * Models
 * ------------------------------------------------------------------------- */

/* An agent MDP M_i = (S, s0, A, P, L) with its cost structure (Sec. 2,
 * "Markov Decision Process"; Sec. 3.1).  Row (s, a) = s * n_actions + a owns
 * successors succ[sa_ptr[row] .. sa_ptr[row+1]) with probabilities prob[..].
 * A row with no successors is a disabled action; an enabled row's
 * probabilities must sum to 1 (within 1e-9).  cost[row] > 0 is the cost of
 * taking a in s; its reward is -cost. */
typedef struct {
    int32_t n_states, n_actions, init;
    const int32_t* sa_ptr;    /* [n_states * n_actions + 1] */
    const int32_t* succ;      /* [sa_ptr[last]], values in [0, n_states)  */
    const double*  prob;      /* [sa_ptr[last]]                           */
    const double*  cost;      /* [n_states * n_actions]                   */
} morap_agent;

/* A task DFA (Q, q0, Q_F, Sigma, delta) whose accepting locations are sinks
 * (Sec. 2, "Deterministic Finite Automata").  Letters are small integers: the
 * caller encodes each label L(s) as a letter index. */
typedef struct {
    int32_t n_locs, n_letters, q0;
    const int32_t* delta;     /* [n_locs * n_letters], values in [0, n_locs) */
    const uint8_t* accepting; /* [n_locs], 1 = accepting                      */
} morap_dfa;

/* A product model M_{i(x)j} in CSR form over its live states (states whose
 * DFA location is neither accepting nor a trap; transitions into done states
 * are dropped), as produced by morap_build_products or supplied by the caller:
 *   state_row[S+1]  rows of state s are state_row[s] .. state_row[s+1]-1,
 *                   in action order (at most 32 rows per state);
 *   row_ptr[R+1]    entries of row r are row_ptr[r] .. row_ptr[r+1]-1;
 *   col[N]          live successor state, in [0, S);
 *   prob[N]         transition probability (row sums in [0, 1]);
 *   rew[2R]         per row: (cost reward rho_i = -cost, probability reward
 *                   rho_{|I|+j} = mass of first acceptance);
 *   to_done[R]      1 if the row moves mass into a done state;
 *   init            index of the initial state (s0, q0), -1 if it is done. */
typedef struct {
    int32_t agent, task;
    int32_t n_states, n_rows, nnz, init;
    const int32_t* state_row;
    const int32_t* row_ptr;
    const int32_t* col;
    const double*  prob;
    const double*  rew;
    const uint8_t* to_done;
} morap_model;

/* Build every agent-task product M_i (x) A_j (Sec. 2, "Product MDP"; Sec. 3.1,
 * proposition done_j and reward rho_{j+|I|}) on the host, for i < n_agents,
 * j < n_tasks, and upload them to the device.  letters[i * n_tasks + j] points
 * to agent i's labelling as seen by task j: [agents[i].n_states] letters in
 * [0, tasks[j].n_letters).  Reachable states are explored from (s0, q0);
 * states are numbered in (q, s) order.  Replaces any loaded models.
 * Errors: INVALID (malformed agent / DFA / letters), OOM, UNSUPPORTED (more
 * than 2^31-1 rows or entries in total, more than 32 rows in a state). */
int morap_build_products(morap_ctx* ctx, const morap_agent* agents, int n_agents,
                         const morap_dfa* tasks, int n_tasks,
                         const int32_t* const* letters);

/* One product M_i (x) A_j on the host only (no context, no device touched):
 * the model morap_build_products makes for (agent, task, letters), with the
 * layout of morap_get_model.  sizes_out[4] = {S, R, N, init}.  Call once with
 * NULL arrays to get the sizes, then with caller-owned arrays of
 * state_row[S+1], row_ptr[R+1], col[N], prob[N], rew[R][2], to_done[R],
 * states[S][2] (agent state, location); each array may be NULL.
 * Errors: INVALID (malformed agent / DFA / letters), OOM, UNSUPPORTED (more
 * than 2^31-1 states, rows or entries). */
int morap_product_host(const morap_agent* agent, const morap_dfa* task, const int32_t* letters,
                       int32_t* sizes_out, int32_t* state_row, int32_t* row_ptr, int32_t* col,
                       double* prob, double* rew, uint8_t* to_done, int32_t* states);

/* Load caller-built product models (same semantics as above).  models[m] must
 * have agent = m / n_tasks and task = m % n_tasks, m < n_agents * n_tasks.
 * Errors: INVALID (structure, ranges, row sums outside [0, 1+1e-6],
 * non-finite rewards), OOM, UNSUPPORTED. */
int morap_load_models(morap_ctx* ctx, const morap_model* models, int n_models,
                      int n_agents, int n_tasks);

/* sizes[0..4] = (S, R, N, init, total states) of model m. Errors: INVALID, STATE. */
int morap_model_info(const morap_ctx* ctx, int m, int32_t* sizes);

/* Copy model m back to the host; any output may be NULL.  states[2S] gets the
 * (agent state, DFA location) pair of every state when the model was built by
 * morap_build_products (zeros otherwise).  Errors: INVALID, STATE. */
int morap_get_model(const morap_ctx* ctx, int m, int32_t* state_row, int32_t* row_ptr,
                    int32_t* col, double* prob, double* rew, uint8_t* to_done,
                    int32_t* states);

/* ---------------------------------------------------------------------------
 * Value iteration, assignment, evaluation (Alg. 2, Alg. 3, Alg. 4)
 * ------------------------------------------------------------------------- */

typedef struct {
    double  eps_vi;       /* Alg. 3 stop: first sweep with max_s |y-x| <= eps_vi   */
    double  eps_eval;     /* Alg. 4 stop, per objective                             */
    double  tau;          /* tie tolerance of the eps-optimal action sets (1e-9)    */
    int32_t precision;    /* MORAP_F64 or MORAP_F32                                 */
    int32_t max_sweeps;   /* per iteration; exceeding it returns NOT_CONVERGED      */
    int32_t check_every;  /* sweeps per host convergence check (even, >= 2)         */
    int32_t schedule;     /* 0 = autotuned sweep kernel, > 0 = fixed variant id     */
    int32_t use_graph;    /* 1 = replay sweep chunks as a captured hipGraph         */
    int32_t time_kernels; /* 1 = time every sweep kernel with HIP events (eager)    */
    int32_t eval_start;   /* Alg. 4 start: 0 = from 0; 1 = from the scalarised      */
                          /* values of the policy's solve (probability 1, or the    */
                          /* warm value, and cost (V - w_p P) / w_c; same stop rule)*/
} morap_vi_opts;

/* Fill `opts` with the defaults: eps 1e-6, tau 1e-9, FP32, 1e6 sweeps, check
 * every 32 sweeps, autotuned, graphs on, no kernel timing, Alg. 4 from 0. */
void morap_default_opts(morap_vi_opts* opts);

typedef struct {
    int64_t backups;        /* state-action backups done (rows x active columns)   */
    int64_t sweeps;         /* sweeps launched (batched VI)                         */
    int64_t max_pair_sweeps;/* largest sweep count of one (model, column) pair     */
    int64_t eval_sweeps;    /* sweeps of the policy evaluation                      */
    int64_t polish_sweeps;  /* FP64 sweeps after an FP32 solve (evaluate)          */
    int64_t rank_rounds;    /* attractor-rank relaxation sweeps (policy extraction)  */
    int64_t floor_stops;    /* FP32 pairs stopped at the rounding floor: no new     */
                            /* smallest change in 64 sweeps, last change within     */
                            /* 256 units in the last place of the largest value     */
    double  bytes;          /* algorithmic bytes moved by the sweep kernel          */
    double  ms_vi, ms_eval, ms_total;   /* device / host wall time of the phases   */
    double  ms_sweep_kernel;/* summed sweep-kernel time (time_kernels = 1)          */
    int64_t sweep_launches; /* sweep kernels timed (every 4th launch)               */
    double  bytes_refine;   /* the three fields above for the FP64 re-solve of the   */
    double  ms_sweep_kernel_refine; /* assigned pairs after an FP32 solve           */
    int64_t sweep_launches_refine;
    int32_t variant;        /* sweep-kernel variant of the last batched solve       */
    int32_t variant_refine; /* variant of the last FP64 re-solve of assigned pairs  */
    int64_t sweeps_tail;    /* sweeps of batched solves run by the LDS-staged kernel */
                            /* once few tiles stay active (included in sweeps;      */
                            /* bytes, ms_sweep_kernel, sweep_launches: main kernel) */
    int64_t sweep_launches_tail; /* their timed launches, bytes and kernel time     */
    double  bytes_tail;
    double  ms_sweep_kernel_tail;
    int32_t variant_tail;   /* that kernel's variant (0: no switch)                 */
    int32_t reserved;
    int64_t refine_pairs;   /* support / query after FP32 solves: unassigned pairs   */
                            /* within the FP32 error of the assignment re-solved in  */
                            /* FP64 ...                                              */
    int64_t refine_columns; /* ... and columns whose assignment they improved        */
} morap_stats;

/* Alg. 2 first loop / Alg. 3 for K weight vectors W[K][d] at once: for every
 * model m = (i, j) and column k, value iteration of the scalarised reward
 * W[k][i] * rho_i + W[k][|I|+j] * rho_{|I|+j} from 0 (Jacobi, do-while, each
 * (model, column) pair stopping at its first sweep with residual <= eps_vi).
 * c_out[K][|I|][|J|] (nullable) receives the value at each model's initial
 * state.  Rows of W must be >= 0 and sum to 1 (1e-9).  The final values stay
 * on the device for morap_evaluate / morap_get_values.
 * Errors: INVALID, STATE (no models), OOM, NOT_CONVERGED, HIP. */
int morap_solve(morap_ctx* ctx, const double* W, int K, const morap_vi_opts* opts,
                double* c_out, morap_stats* stats);

/* Alg. 3 as morap_solve, with stages retiring inside the Jacobi iteration
 * (the staged form of value iteration that ordering by strongly connected
 * components allows, Sec. 6).  A state's stage is the height of its DFA
 * location group (a strongly connected set of locations) in the DAG those
 * groups form in its product; every transition leads to the same or a lower
 * stage.  Each sweep backs up the stages still active in a column; after it,
 * a stage retires in that column when every lower stage has retired and the
 * largest change over its own states is <= eps_vi, and keeps the values of
 * that sweep from then on.  A pair is done when the stage of its initial
 * state retires; c_out as morap_solve.  The stop rule is morap_solve's per
 * stage (FP32: also the rounding floor of a stage whose change has stopped
 * falling).  Products built by morap_build_products (block form) only;
 * opts.schedule, when > 0, must name a neighbourhood-block sweep (ids
 * 19-38).  The values stay on the device as after morap_solve.
 * stats->backups counts the rows of the active stages only.
 * Errors: INVALID, STATE, UNSUPPORTED (team model, caller-loaded models),
 * OOM, NOT_CONVERGED, HIP. */
int morap_solve_staged(morap_ctx* ctx, const double* W, int K, const morap_vi_opts* opts,
                       double* c_out, morap_stats* stats);

/* Alg. 2 second loop for the columns of the last morap_solve: assign[K][|J|]
 * gives the agent of every task per column.  For each (k, j) the policy of
 * model (assign[k][j], j) is extracted from that column's final values (FP32
 * solves are first refined by FP64 value iteration of that model and column to
 * eps_vi), with the attractor tie rule on the tau-optimal action sets, then
 * evaluated per objective (Alg. 4, FP64 Jacobi from 0, eps_eval; with
 * opts->eval_start = 1 from the values the policy was chosen from: the
 * probability objective at 1, the cost objective at (V - w_p) / w_c with the
 * pair's weights scaled to sum 1 where w_c >= 1e-3; a proper policy's
 * evaluation reaches its values from any start, and the stop rule bounds the
 * error of the result alike).  r_out[K][d]: r[|I|+j] = completion probability of task j; r[i] = sum of the
 * cost values of the tasks assigned to i.  Each agent may receive at most
 * ceil(|J|/|I|) tasks.  On a team model (morap_load_team_model) assign is
 * ignored (may be NULL): the one policy of each column is evaluated on every
 * objective into r_out[K][d], and morap_get_policy(k, 0) returns it.
 * Errors: INVALID, STATE, IMPROPER, NOT_CONVERGED, HIP. */
int morap_evaluate(morap_ctx* ctx, const int32_t* assign, int K, const morap_vi_opts* opts,
                   double* r_out, morap_stats* stats);

/* Max-weight assignment of Alg. 2 on the host for each column:
 * c[K][|I|][|J|] -> assign_out[K][|J|], maximising sum_j c[k][f(j)][j] with at
 * most ceil(|J|/|I|) tasks per agent (Hungarian method, O(n^3)).
 * Errors: INVALID. */
int morap_assign(morap_ctx* ctx, const double* c, int K, int32_t* assign_out);

/* The team MDP of the decentralised model (Sec. 3.1, Def. teamMDP) for n
 * agents and n tasks (n_agents = n_tasks = n <= 16, else INVALID),
 * scalarised for one weight vector w[2n] and
 * laid out as one caller-built model for morap_load_models with one agent and
 * one task, to be solved with the weight row (1, 0): rew[r][0] = w . (the
 * objective vector of row r), rew[r][1] = 0.  A state is (agent, task, agent
 * state, task location, committed agents); its rows are the committed agent's
 * actions, the zero-reward switches that commit an agent or hand a task on at
 * its start and start the next task once one is done, or else one empty row
 * (value 0).  letters[i * n + j] as in morap_build_products.  Host only, no
 * context; two calls as morap_product_host (sizes_out = {S, R, N, init}).
 * Its optimum from the initial state is the best assignment's (Lemma
 * lem:ct-mdp-prop).  Errors: INVALID, UNSUPPORTED (the state count is
 * exponential in n), OOM. */
int morap_team_model_host(const morap_agent* agents, int n_agents, const morap_dfa* tasks,
                          int n_tasks, const int32_t* const* letters, const double* w,
                          int32_t* sizes_out, int32_t* state_row, int32_t* row_ptr, int32_t* col,
                          double* prob, double* rew, uint8_t* to_done);

/* The team MDP of Def. teamMDP for n agents and n tasks (n <= 16) with its
 * d = 2n objectives, as one caller-built model for morap_load_team_model
 * (host only, no context; two calls as morap_product_host, sizes_out = {S,
 * R, N, init}): rew[r] = (-cost, mass entering acceptance) of agent i acting
 * on task j, obj[r] = (i, n + j), the objectives the two rewards belong to;
 * the zero-reward rows (commit, hand over, start the next task, empty) have
 * obj[r] = (0, n).  Errors: as morap_team_model_host. */
int morap_team_model_mo_host(const morap_agent* agents, int n_agents, const morap_dfa* tasks, int n_tasks,
                             const int32_t* const* letters, int32_t* sizes_out, int32_t* state_row,
                             int32_t* row_ptr, int32_t* col, double* prob, double* rew, int32_t* obj,
                             uint8_t* to_done);

/* Load a team MDP with d = n_agents + n_tasks objectives into the context
 * (Def. teamMDP; replaces any loaded models): one model in the layout of
 * morap_load_models (its agent and task fields 0) plus obj[R][2], the
 * objective in [0, d) each of a row's two rewards belongs to.  On such a
 * context morap_solve takes W[K][d] and scalarises every row with its own
 * objectives (w[obj[r][0]] rew[r][0] + w[obj[r][1]] rew[r][1]); c_out[K]
 * gets the value at the initial state; morap_support evaluates the policy of
 * every column per objective (Alg. 4 on the d objectives) into r_out[K][d]
 * (assign_out, if given, gets 0 per task); morap_query and morap_query_batch
 * run Alg. 1 on it.  Its optimum for w equals the decentralised
 * assignment's (Lemma lem:ct-mdp-prop).  Errors: INVALID (as
 * morap_load_models, objective out of range), OOM, UNSUPPORTED. */
int morap_load_team_model(morap_ctx* ctx, int n_agents, int n_tasks, const morap_model* model,
                          const int32_t* obj);

/* The same assignment without a context (host only, no device touched), for
 * c[K][n_agents][n_tasks] given by the caller: assign_out[K][n_tasks] holds
 * the agent of each task.  Caller-owned buffers.  Errors: INVALID (sizes,
 * NULL pointers, a non-finite value). */
int morap_assign_host(const double* c, int n_agents, int n_tasks, int K, int32_t* assign_out);

/* Alg. 2 whole, for K weight vectors: solve -> assignment -> evaluate.
 * After an FP32 solve the assignment is checked on FP64 values: the FP64
 * re-solve of the assigned pairs measures each column's FP32 error e; every
 * other pair whose slack against the assignment (from the optimal duals) is
 * at most 2e is re-solved in FP64 as well, the column is assigned again with
 * these values, and it takes the new assignment when its value rises (stats:
 * refine_pairs, refine_columns).  r_out[K][d], assign_out[K][|J|] (nullable;
 * the assignment evaluated), c_out[K][|I|][|J|] (nullable; the solve's
 * values).  Errors: as morap_solve and morap_evaluate. */
int morap_support(morap_ctx* ctx, const double* W, int K, const morap_vi_opts* opts,
                  double* r_out, int32_t* assign_out, double* c_out, morap_stats* stats);

/* Statistics accumulated by every solve / evaluate on the context since the
 * last reset (morap_query and morap_support included).  Errors: INVALID. */
int morap_get_stats(const morap_ctx* ctx, morap_stats* out);
int morap_reset_stats(morap_ctx* ctx);

/* Policy chosen for task j in column k by the last morap_evaluate: mu_out[S]
 * of model (assign[k][j], j), each entry the chosen row counted from the
 * state's first row.  Errors: INVALID, STATE. */
int morap_get_policy(const morap_ctx* ctx, int k, int j, int8_t* mu_out);

/* Final values of column k of model m from the last morap_solve, as FP64
 * x_out[S].  Errors: INVALID, STATE. */
int morap_get_values(const morap_ctx* ctx, int k, int m, double* x_out);

/* ---------------------------------------------------------------------------
 * Point-oriented Pareto computation (Alg. 1)
 * ------------------------------------------------------------------------- */

typedef struct {
    double  eps;             /* Alg. 1 loop tolerance on ||t_down - t_up||_M        */
    int32_t max_iter;        /* Alg. 2 calls per query                              */
    int32_t verification_only; /* stop once t is separated (Sec. 5, Experiment 2) */
    int32_t use_proposer;    /* 1 = learned proposer gives the first weight vector  */
    int32_t keep_trace;      /* 1 = fill the trace arrays of the result             */
    int32_t warm_start;      /* 1 = after the first pass, each FP32 solve starts a
                                query's column from its values of the previous
                                pass (pairs with a zero cost weight from 0)     */
    int32_t proposer_passes; /* with use_proposer: the proposer gives the weight
                                vector of the first max(1, proposer_passes)
                                passes; after the first its input is t_down (the
                                closest point to t that the separating hyperplanes
                                found so far allow) in place of t.  A later
                                proposal is kept only if it is finite, on the
                                simplex, unlike every earlier weight vector of
                                the query, and the previous learned pass shrank
                                the gap by 1 %; otherwise that query takes Alg.
                                1's own update from then on (fallback = 2)     */
    morap_vi_opts vi;
} morap_query_opts;

/* Result of one query.  t_up / t_down / lam and the trace arrays are
 * caller-owned and may be NULL:
 *   t_up[d], t_down[d]              final inner / outer closest points;
 *   lam[max_iter]                   convex weights of the points of Phi whose
 *                                   combination dominates t_up;
 *   trace_w / trace_r [max_iter][d] weight vector and point of every pass;
 *   trace_f [max_iter][|J|]         assignment of every pass (the agent of
 *                                   each task), for morap_synthesize. */
typedef struct {
    int32_t verdict;         /* MORAP_FEASIBLE, MORAP_INFEASIBLE, MORAP_UNDECIDED */
    int32_t iterations;      /* Alg. 2 calls                                      */
    int32_t fallback;        /* 1 = the proposer's weight was rejected            */
    int32_t reserved;
    double  gap;             /* ||t_down - t_up||_M at exit                        */
    double  ms;              /* wall time (in a batch: its share of every pass it
                                took part in)                                   */
    int64_t backups;
    double* t_up;
    double* t_down;
    double* lam;
    double* trace_w;
    double* trace_r;
    int32_t* trace_f;
    double  latency_ms;      /* wall time from the start of the call to the end
                                of the Alg. 2 pass in which the query stopped
                                (batches: queries run in lockstep)             */
} morap_query_result;

/* Alg. 1 for threshold t[d] with norm matrix M[d][d] (symmetric positive
 * definite; NULL = identity).  Loop: r = Alg. 2(w); add r to Phi and (w, r)
 * to Lambda; if w.r < w.t_down, t_down = argmin ||t - z||_M s.t. w'.z <= w'.r'
 * for all of Lambda; t_up = argmin over x in down(Phi) of ||t - x||_M; stop if
 * ||t_down - t_up||_M <= eps; else w = M(t - t_up)/||M(t - t_up)||_1.
 * Verdict: FEASIBLE iff t in down(Phi), INFEASIBLE iff some (w', r') has
 * w'.r' < w'.t, else UNDECIDED.  Errors: INVALID, STATE, and those of
 * morap_support. */
int morap_query(morap_ctx* ctx, const double* t, const double* M,
                const morap_query_opts* opts, morap_query_result* result);

/* Q queries T[Q][d] advanced in lockstep: every Alg. 1 pass solves the weight
 * vectors of all unfinished queries as the columns of one morap_support call
 * (at most 64 columns per call; larger Q runs in groups of 64, each group to
 * its end before the next starts).
 * W0[Q][d] (nullable) replaces each query's first weight vector (rows >= 0,
 * summing to 1); NULL means (1, 0, ..., 0) or the learned proposer's output.
 * results[Q].  Errors: as morap_query. */
int morap_query_batch(morap_ctx* ctx, const double* T, const double* W0, int Q, const double* M,
                      const morap_query_opts* opts, morap_query_result* results);

/* Synthesis after Alg. 1 (Sec. 3.3, the random assignment and schedulers
 * extracted from the loop): with v a convex weighting of the passes' points
 * that dominates t_up (the query's lam), the random assignment picks the
 * assignment f of pass i with probability v[i] and then runs, for every task
 * j, the scheduler that pass computed for model (f(j), j).
 * Inputs (host, caller-owned): the n passes' weight vectors W[n][d], their
 * assignments F[n][|J|] (a query's trace_w, trace_f) and v[n] >= 0.  The
 * passes with v > 0 are re-solved and their recorded assignments evaluated
 * (morap_solve and morap_evaluate on exactly those columns), which reproduces
 * their points and schedulers.  Outputs: n_picked, picked_out[n] (indices of
 * the passes with v > 0, in order), r_out[n][d] (their points, first n_picked
 * rows), matrix_out[|I|][|J|] (nullable): the probability that agent i
 * serves task j, sum of v[i] over the picked passes with f(j) = i, divided by
 * the sum of their v.  Afterwards morap_get_policy(q, j) returns the
 * scheduler of task j in the q-th picked pass.  Errors: INVALID (no v > 0,
 * an agent index out of range, negative v), UNSUPPORTED (a team model is
 * loaded), and those of morap_solve and morap_evaluate. */
int morap_synthesize(morap_ctx* ctx, const double* W, const int32_t* F, const double* v, int n,
                     const morap_vi_opts* opts, int32_t* n_picked, int32_t* picked_out, double* r_out,
                     double* matrix_out);

/* Projections of Alg. 1 on their own (host, FP64).  Inner: x_out[d] in
 * down(conv Phi[m][d]) closest to t in the M-norm, lam_out[m] (nullable) its
 * convex weights.  Outer: z_out[d] closest to t subject to
 * W[n][d] z <= rowwise W.R.  Errors: INVALID, NOT_CONVERGED. */
int morap_project_inner(const double* Phi, int m, int d, const double* t, const double* M,
                        double* x_out, double* lam_out);
int morap_project_outer(const double* W, const double* R, int n, int d, const double* t,
                        const double* M, double* z_out);

/* ---------------------------------------------------------------------------
 * Learned weight proposer (a small MLP in front of the weight update of
 * Alg. 1; not part of the paper)
 * ------------------------------------------------------------------------- */

/* Sizes: input n_in = d + n_feat, three hidden layers of 256, output d.
 * Weights are BF16 on the device with FP32 master copies; products accumulate
 * in FP32 (MFMA).  Parameter order for get/set: W1[256][n_in], b1[256],
 * W2[256][256], b2, W3[256][256], b3, W4[d][256], b4[d] (row-major, FP32). */
typedef struct {
    int32_t batch;           /* rows per step                                    */
    int32_t epochs;
    float   lr, beta1, beta2, adam_eps;
    uint64_t seed;           /* shuffling                                        */
} morap_train_opts;

/* Create (or re-create) the proposer for input width n_in and output width d
 * with He-uniform weights from a counter-based generator (SplitMix64 of seed)
 * and zero biases.  Errors: INVALID, OOM, HIP. */
int morap_proposer_init(morap_ctx* ctx, int n_in, int d, uint64_t seed);

/* Number of FP32 parameters; get / set copy all of them (order above). */
int64_t morap_proposer_num_params(const morap_ctx* ctx);
int morap_proposer_get_params(const morap_ctx* ctx, float* out);
int morap_proposer_set_params(morap_ctx* ctx, const float* in);

/* Input standardisation applied before the first layer: x -> (x - mu) / sd
 * per input column (mu[n_in], sd[n_in] > 0; the library copies them).  It is
 * not trained and is saved with the parameters; init sets mu = 0, sd = 1.
 * Errors: INVALID, STATE. */
int morap_proposer_set_input_norm(morap_ctx* ctx, const float* mu, const float* sd);

/* Forward pass: X[n][n_in] -> W_out[n][d] (softmax rows).  Errors: INVALID,
 * STATE (no proposer), HIP. */
int morap_proposer_infer(morap_ctx* ctx, const float* X, int n, float* W_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * forward pass of morap_proposer_infer on DEVICE buffers, with no allocation
 * of any kind.  X_dev[n][n_in] (FP32, device pointer, caller-owned) ->
 * W_out_dev[n][d] (FP32 softmax rows, device pointer, caller-owned).  The
 * work is enqueued on the context's stream and not waited for (synchronise
 * the device or the stream before reading W_out_dev).  The activations use a
 * fixed scratch of 8 MiB per device (held until the process ends, its address
 * taken when the first context on the device is created): n must satisfy
 * n * (2 n_in + 1536 + 4 d) bytes (each part rounded up to 256) <= 8 MiB,
 * e.g. at most 4,712 rows for n_in = 62, d = 30; larger n returns
 * UNSUPPORTED with the limit in the message and enqueues nothing.  Every call
 * on a device shares that scratch: calls that overlap on one device (from
 * several contexts or streams) race.  Errors: INVALID (NULL pointers,
 * n < 1), STATE (no proposer), UNSUPPORTED (too many rows), HIP. */
int morap_proposer_infer_noalloc(morap_ctx* ctx, const float* X_dev, int n, float* W_out_dev);

/* One forward + backward pass on X[n][n_in] with targets T[n][d] (rows on the
 * simplex), mean cross-entropy loss.  loss_out (nullable) gets the loss;
 * grads_out (nullable) gets the FP32 gradients in parameter order.  When
 * apply != 0 an Adam step (opts lr, betas, eps) follows.  Errors: INVALID,
 * STATE, HIP. */
int morap_proposer_step(morap_ctx* ctx, const float* X, const float* T, int n,
                        const morap_train_opts* opts, int apply, float* loss_out,
                        float* grads_out);

/* Train for opts->epochs over the n examples (shuffled per epoch from
 * opts->seed), in batches of opts->batch.  loss_out[epochs] (nullable) gets
 * the mean loss of every epoch.  Errors: INVALID, STATE, HIP. */
int morap_proposer_train(morap_ctx* ctx, const float* X, const float* T, int n,
                         const morap_train_opts* opts, float* loss_out);

/* Save / load the FP32 parameters and sizes to / from a binary file.
 * Errors: INVALID (I/O, size mismatch), STATE. */
int morap_proposer_save(const morap_ctx* ctx, const char* path);
int morap_proposer_load(morap_ctx* ctx, const char* path);

/* Training target of the proposer for one answered query (host only, no
 * context): for a threshold t[d] outside the achievable set (t_down != t),
 * the normal M (t - t_down) of the face of the outer approximation that holds
 * the closest point t_down[d]; for a threshold inside it, the last weight
 * vector w_last[d] the plain loop used.  Negative entries become 0 and the
 * result w_out[d] is normalised to sum 1 (the uniform vector if nothing is
 * left).  M = NULL means the identity.  Errors: INVALID (NULL arrays, d < 1,
 * non-finite input). */
int morap_proposer_target(const double* t, const double* t_down, const double* w_last, int d, const double* M,
                          double* w_out);

/* Instance feature vector phi[n_feat] used by morap_query when
 * use_proposer = 1: the proposer's input is [t; phi] (n_in = d + n_feat).
 * The library copies phi.  Errors: INVALID. */
int morap_set_features(morap_ctx* ctx, const double* phi, int n_feat);

#ifdef __cplusplus
}
#endif

#endif /* MORAP_H */
