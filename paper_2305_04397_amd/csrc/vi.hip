// Value-iteration kernels for gfx950 (wave64).
//
//  * bellman_sweep: one Jacobi sweep of scalarised max-backups (Alg. 3, the
//    maximisation over enabled actions of (w . rho)(s,q,a) + sum P x) for every
//    active (model, column) pair.  Values are stored [state][Kp] so that the
//    successor gather of one state for a run of columns is one contiguous,
//    coalesced line.  A workgroup streams one tile of consecutive states of a
//    model: the tile's rows and entries are staged in LDS with coalesced loads,
//    then each group of `LPS` lanes walks one state's entries from LDS and
//    issues its successor gathers in batches of 8 so several are in flight.
//    The grid is persistent over a compacted list of the tiles of models that
//    still have active columns; each XCD walks its own contiguous eighth of
//    that list so neighbouring tiles share its L2.  Per-(model, column)
//    residual max |y - x| and max |y| are reduced in FP64 (wave shuffles, then
//    LDS, then one atomic per column per tile).
//  * converge / compact: freeze pairs whose residual is within tolerance
//    (the stop test of Alg. 3), record their value at the initial state and
//    rebuild the active tile list.
//  * instance kernels: eps-optimal action masks, attractor ranks (BFS
//    distances by in-place relaxation) with the action choice, and
//    fixed-policy evaluation sweeps (Alg. 4) on (column, model) instances, one
//    thread per state.
#include "common.h"
#include "kern.h"

#include <cfloat>

namespace morap {
namespace k {

// LDS staging limits of one tile (host tiles respect them)
constexpr int TILE_STATES = 128;
constexpr int TILE_ROWS = 768;
constexpr int TILE_NNZ = 2048;

int sweep_lds_rows() { return TILE_ROWS; }
int sweep_lds_nnz() { return TILE_NNZ; }
int sweep_tile_states(const Variant&) { return TILE_STATES; }

// ---------------------------------------------------------------------------
// small fills
// ---------------------------------------------------------------------------
template <class T>
__global__ void fill_kernel(T* p, T v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

template <class T>
static void fill(hipStream_t s, T* p, T v, int64_t n) {
    if (n <= 0) return;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(fill_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, s, p, v, n);
    MORAP_HIP(hipGetLastError());
}
void fill_u8(hipStream_t s, uint8_t* p, uint8_t v, int64_t n) { fill(s, p, v, n); }
void fill_i32(hipStream_t s, int32_t* p, int32_t v, int64_t n) { fill(s, p, v, n); }
void fill_u64(hipStream_t s, uint64_t* p, uint64_t v, int64_t n) { fill(s, p, v, n); }
void fill_f32(hipStream_t s, float* p, float v, int64_t n) { fill(s, p, v, n); }
void fill_f64(hipStream_t s, double* p, double v, int64_t n) { fill(s, p, v, n); }
void fill_i64(hipStream_t s, int64_t* p, int64_t v, int64_t n) { fill(s, p, v, n); }

__global__ void to_f32_kernel(const double* in, float* out, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) out[i] = (float)in[i];
}
void to_f32(hipStream_t s, const double* in, float* out, int64_t n) {
    if (n <= 0) return;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(to_f32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, in, out, n);
    MORAP_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// batched Bellman sweep
// ---------------------------------------------------------------------------
// Per-(model, column) residual and |y| maxima accumulated by a workgroup over
// its tiles of one model, flushed with one atomic per column when the model
// changes (and at the end).
template <int CPL, int LPS, int NW, int KT>
__device__ __forceinline__ void flush_residuals(double (&res)[CPL], double (&ym)[CPL], double (*l_red)[NW][KT],
                                                int m, int Kp, unsigned long long* res_all,
                                                unsigned long long* ymax_all, bool want_ymax) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, gl = tid % LPS;
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        res[c] = group_max<LPS>(res[c]);
        ym[c] = group_max<LPS>(ym[c]);
    }
    if (lane < LPS) {
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            l_red[0][wave][gl * CPL + c] = res[c];
            l_red[1][wave][gl * CPL + c] = ym[c];
        }
    }
    __syncthreads();
    if (tid < KT) {
        double r = 0.0, y = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            r = fmax(r, l_red[0][w][tid]);
            y = fmax(y, l_red[1][w][tid]);
        }
        const int64_t idx = (int64_t)m * Kp + blockIdx.y * KT + tid;
        max_flush(&res_all[idx], r);
        if (want_ymax) max_flush(&ymax_all[idx], y);
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        res[c] = 0.0;
        ym[c] = 0.0;
    }
}

template <class T, class T2, int CPL, int LPS, int WG>
__global__ void __launch_bounds__(WG)
bellman_sweep(const Tile* __restrict__ tiles, const int32_t* __restrict__ tile_base,
              const int32_t* __restrict__ act_models, const int32_t* __restrict__ act_prefix,
              const int64_t* __restrict__ counters,
              const int32_t* __restrict__ state_row, const int32_t* __restrict__ row_ptr,
              const int32_t* __restrict__ col, const T* __restrict__ prob, const T2* __restrict__ rew,
              const T* __restrict__ wc_all, const T* __restrict__ wp_all,
              const uint8_t* __restrict__ active_all,
              const T* __restrict__ x_in, T* __restrict__ x_out,
              unsigned long long* __restrict__ res_all, unsigned long long* __restrict__ ymax_all,
              int Kp, const T* __restrict__ rewk) {
    // rewk (nullable): the scalarised reward of every (row, column), [R][Kp]
    // (team models, whose rows carry their own objectives), replacing
    // wc rew.x + wp rew.y
    constexpr int KT = CPL * LPS;          // columns per k-tile
    constexpr int G = WG / LPS;            // states processed at once
    constexpr int NW = WG / 64;            // waves
    constexpr bool want_ymax = sizeof(T) == 4;   // |y| only bounds the FP32 stop test
    __shared__ int32_t l_srow[TILE_STATES + 1];
    __shared__ int32_t l_rptr[TILE_ROWS + 1];
    __shared__ T2 l_rew[TILE_ROWS];
    __shared__ int32_t l_col[TILE_NNZ];
    __shared__ T l_prob[TILE_NNZ];
    __shared__ uint16_t l_erow[TILE_NNZ];
    __shared__ double l_red[2][NW][KT];

    const int tid = threadIdx.x;
    const int grp = tid / LPS;             // state slot within a pass
    const int gl = tid % LPS;              // lane within the group
    const int kc = blockIdx.y * KT + gl * CPL;   // first column of this lane

    // Each workgroup owns a contiguous block of the active tile list; the
    // workgroups of one XCD (blockIdx % 8) own consecutive blocks, so
    // neighbouring tiles (which share successors) stay in that XCD's L2.
    const int n_tiles = (int)counters[1];
    const int n_act = (int)counters[2];
    int t_begin, t_end;
    xcd_share(n_tiles, blockIdx.x & 7, blockIdx.x >> 3, gridDim.x >> 3, t_begin, t_end);
    if (t_begin >= t_end) return;

    // active model holding the first tile, then advanced tile by tile
    int lo = 0;
    {
        int hi = n_act;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (act_prefix[mid] <= t_begin) lo = mid; else hi = mid;
        }
    }
    int cur_m = -1;
    bool tile_on = false, any = false;
    T wc[CPL], wp[CPL];
    bool act[CPL];
    double res[CPL], ym[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        res[c] = 0.0;
        ym[c] = 0.0;
        wc[c] = wp[c] = 0;
        act[c] = false;
    }

    for (int t = t_begin; t < t_end; ++t) {
        while (act_prefix[lo + 1] <= t) ++lo;
        const int m = act_models[lo];
        if (m != cur_m) {
            if (cur_m >= 0)
                flush_residuals<CPL, LPS, NW, KT>(res, ym, l_red, cur_m, Kp, res_all, ymax_all, want_ymax);
            cur_m = m;
            any = false;
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                const int64_t k = (int64_t)m * Kp + kc + c;
                wc[c] = wc_all[k];
                wp[c] = wp_all[k];
                act[c] = active_all[k] != 0;
                any |= act[c];
            }
            // skip the model when no column of this k-tile is active
            tile_on = __syncthreads_or(any ? 1 : 0) != 0;
        }
        if (!tile_on) continue;
        const Tile tl = tiles[tile_base[m] + (t - act_prefix[lo])];
        const int s0 = tl.s_begin, s1 = tl.s_end, ns = s1 - s0;
        const int r0 = state_row[s0], r1 = state_row[s1];
        const int e0 = row_ptr[r0], e1 = row_ptr[r1];
        const int nr = r1 - r0, ne = e1 - e0;

        // stage the tile in LDS (coalesced)
        for (int i = tid; i <= ns; i += WG) l_srow[i] = state_row[s0 + i] - r0;
        for (int i = tid; i <= nr; i += WG) l_rptr[i] = row_ptr[r0 + i] - e0;
        for (int i = tid; i < nr; i += WG) l_rew[i] = rew[r0 + i];
        for (int i = tid; i < ne; i += WG) {
            l_col[i] = col[e0 + i];
            l_prob[i] = prob[e0 + i];
        }
        __syncthreads();
        for (int r = tid; r < nr; r += WG)
            for (int e = l_rptr[r]; e < l_rptr[r + 1]; ++e) l_erow[e] = (uint16_t)r;
        __syncthreads();

        if (any) {
            for (int ls = grp; ls < ns; ls += G) {
                const int lr0 = l_srow[ls], lr1 = l_srow[ls + 1];
                T best[CPL];
#pragma unroll
                for (int c = 0; c < CPL; ++c) best[c] = -INFINITY;
                // rows without live successors
                for (int r = lr0; r < lr1; ++r) {
                    if (l_rptr[r] == l_rptr[r + 1]) {
                        const T2 rw = l_rew[r];
#pragma unroll
                        for (int c = 0; c < CPL; ++c)
                            best[c] = fmax(best[c], rewk ? rewk[(int64_t)(r0 + r) * Kp + kc + c]
                                                         : wc[c] * rw.x + wp[c] * rw.y);
                    }
                }
                const int le0 = l_rptr[lr0], le1 = l_rptr[lr1];
                int cur = -1;
                T acc[CPL];
#pragma unroll
                for (int c = 0; c < CPL; ++c) acc[c] = 0;
                constexpr int B = CPL >= 4 ? 4 : 8;   // gathers in flight per lane
                for (int base = le0; base < le1; base += B) {
                    const int n = min(B, le1 - base);
                    int jj[B];
                    T pp[B];
                    int rr[B];
#pragma unroll
                    for (int u = 0; u < B; ++u) {
                        if (u < n) {
                            jj[u] = l_col[base + u];
                            pp[u] = l_prob[base + u];
                            rr[u] = l_erow[base + u];
                        }
                    }
                    Vec<T, CPL> xv[B];
#pragma unroll
                    for (int u = 0; u < B; ++u)
                        if (u < n) xv[u] = vload<T, CPL>(x_in + (int64_t)jj[u] * Kp + kc);
#pragma unroll
                    for (int u = 0; u < B; ++u) {
                        if (u < n) {
                            if (rr[u] != cur) {
                                if (cur >= 0) {
#pragma unroll
                                    for (int c = 0; c < CPL; ++c) best[c] = fmax(best[c], acc[c]);
                                }
                                cur = rr[u];
                                const T2 rw = l_rew[cur];
#pragma unroll
                                for (int c = 0; c < CPL; ++c)
                                    acc[c] = rewk ? rewk[(int64_t)(r0 + cur) * Kp + kc + c]
                                                  : wc[c] * rw.x + wp[c] * rw.y;
                            }
#pragma unroll
                            for (int c = 0; c < CPL; ++c) acc[c] = fma(pp[u], xv[u].v[c], acc[c]);
                        }
                    }
                }
                if (cur >= 0) {
#pragma unroll
                    for (int c = 0; c < CPL; ++c) best[c] = fmax(best[c], acc[c]);
                }
                const int64_t gs = s0 + ls;
                const Vec<T, CPL> old = vload<T, CPL>(x_in + gs * Kp + kc);
#pragma unroll
                for (int c = 0; c < CPL; ++c) {
                    if (act[c]) {
                        x_out[gs * Kp + kc + c] = best[c];
                        res[c] = fmax(res[c], (double)fabs(best[c] - old.v[c]));
                        if (want_ymax) ym[c] = fmax(ym[c], fabs((double)best[c]));
                    }
                }
            }
        }
        __syncthreads();   // the next tile reuses the staging area
    }
    if (cur_m >= 0) flush_residuals<CPL, LPS, NW, KT>(res, ym, l_red, cur_m, Kp, res_all, ymax_all, want_ymax);
}

// ---------------------------------------------------------------------------
// sweep dispatch: variant id -> template instance
// ---------------------------------------------------------------------------
template <class T, class T2, int CPL, int LPS>
static void launch_sweep(hipStream_t s, int grid, int ktiles, const SweepArgs& a) {
    constexpr int WG = (64 * LPS < 256) ? 64 * LPS : 256;
    hipLaunchKernelGGL((bellman_sweep<T, T2, CPL, LPS, WG>), dim3(grid, ktiles), dim3(WG), 0, s,
                       a.tiles, a.tile_base, a.act_models, a.act_prefix, a.counters, a.state_row,
                       a.row_ptr, a.col, (const T*)a.prob, (const T2*)a.rew, (const T*)a.wc,
                       (const T*)a.wp, a.active, (const T*)a.x_in, (T*)a.x_out, a.res, a.ymax, a.Kp,
                       (const T*)a.rewk);
}

template <class T, class T2>
static void sweep_t(hipStream_t s, const Variant& v, int grid, int ktiles, const SweepArgs& a) {
#define MORAP_V(C, L) \
    if (v.cpl == C && v.lps == L) { launch_sweep<T, T2, C, L>(s, grid, ktiles, a); return; }
    MORAP_V(1, 1) MORAP_V(1, 2) MORAP_V(2, 1) MORAP_V(1, 4) MORAP_V(2, 2) MORAP_V(4, 1)
    MORAP_V(1, 8) MORAP_V(2, 4) MORAP_V(4, 2) MORAP_V(1, 16) MORAP_V(2, 8) MORAP_V(4, 4)
    MORAP_V(1, 32) MORAP_V(2, 16) MORAP_V(4, 8) MORAP_V(1, 64) MORAP_V(2, 32) MORAP_V(4, 16)
#undef MORAP_V
    fail(MORAP_E_UNSUPPORTED, "no sweep kernel for this variant");
}

template <class T, class T2>
static const void* sweep_fn(const Variant& v) {
#define MORAP_F(C, L)                                                                                   \
    if (v.cpl == C && v.lps == L)                                                                       \
        return reinterpret_cast<const void*>(                                                           \
            &bellman_sweep<T, T2, C, L, ((64 * L < 256) ? 64 * L : 256)>);
    MORAP_F(1, 1) MORAP_F(1, 2) MORAP_F(2, 1) MORAP_F(1, 4) MORAP_F(2, 2) MORAP_F(4, 1)
    MORAP_F(1, 8) MORAP_F(2, 4) MORAP_F(4, 2) MORAP_F(1, 16) MORAP_F(2, 8) MORAP_F(4, 4)
    MORAP_F(1, 32) MORAP_F(2, 16) MORAP_F(4, 8) MORAP_F(1, 64) MORAP_F(2, 32) MORAP_F(4, 16)
#undef MORAP_F
    fail(MORAP_E_UNSUPPORTED, "no sweep kernel for this variant");
}

int sweep_resident(int prec, const Variant& v) {
    int n = 0;
    MORAP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &n, prec == MORAP_F32 ? sweep_fn<float, float2>(v) : sweep_fn<double, double2>(v), v.wg, 0));
    return n;
}

void sweep(hipStream_t s, int prec, const Variant& v, int grid, int ktiles, const SweepArgs& a) {
    if (prec == MORAP_F32) sweep_t<float, float2>(s, v, grid, ktiles, a);
    else sweep_t<double, double2>(s, v, grid, ktiles, a);
    MORAP_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// team models: the scalarised reward of every (row, column) from the row's
// own objectives, out[r][k] = W[k][obj[r][0]] rew[r][0] + W[k][obj[r][1]]
// rew[r][1] for k < K, 0 for the padding columns
// ---------------------------------------------------------------------------
__global__ void team_rewards_kernel(int64_t R, int K, int Kp, int d, const double* __restrict__ W,
                                    const int32_t* __restrict__ obj, const double* __restrict__ rew,
                                    double* __restrict__ out64, float* __restrict__ out32) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= R * Kp) return;
    const int64_t r = i / Kp;
    const int k = (int)(i % Kp);
    double v = 0.0;
    if (k < K) v = W[(int64_t)k * d + obj[2 * r]] * rew[2 * r] + W[(int64_t)k * d + obj[2 * r + 1]] * rew[2 * r + 1];
    out64[i] = v;
    out32[i] = (float)v;
}

__global__ void team_eval_kernel(int64_t S, int d, const int32_t* __restrict__ pi, const int32_t* __restrict__ row_ptr,
                                 const int32_t* __restrict__ col, const double* __restrict__ prob,
                                 const double* __restrict__ rew, const int32_t* __restrict__ obj,
                                 const double* __restrict__ E_in, double* __restrict__ E_out,
                                 unsigned long long* __restrict__ res) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double change = 0.0;
    if (i < S * d) {
        const int64_t s = i / d;
        const int o = (int)(i % d);
        const int row = pi[s];
        double v = (obj[2 * row] == o ? rew[2 * row] : 0.0) + (obj[2 * row + 1] == o ? rew[2 * row + 1] : 0.0);
        for (int e = row_ptr[row]; e < row_ptr[row + 1]; ++e) v = fma(prob[e], E_in[(int64_t)col[e] * d + o], v);
        E_out[i] = v;
        change = fabs(v - E_in[i]);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) change = fmax(change, __shfl_xor(change, off, 64));
    if (res && (threadIdx.x & 63) == 0 && change > 0.0)
        atomicMax(res, (unsigned long long)__double_as_longlong(change));
}

void team_eval_sweep(hipStream_t s, int64_t S, int d, const int32_t* pi, const int32_t* row_ptr, const int32_t* col,
                     const double* prob, const double* rew, const int32_t* obj, const double* E_in, double* E_out,
                     unsigned long long* res) {
    const int64_t n = S * d;
    if (n <= 0) return;
    hipLaunchKernelGGL(team_eval_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, S, d, pi, row_ptr, col,
                       prob, rew, obj, E_in, E_out, res);
    MORAP_HIP(hipGetLastError());
}

// The start lies below the optimum over proper policies (the fixed policy is
// one); the margin covers the evaluation's stop and rounding.
template <class T>
__global__ void team_start_kernel(int64_t S, int K, int Kp, int d, const double* __restrict__ W,
                                  const double* __restrict__ E, T* __restrict__ x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S * Kp) return;
    const int64_t s = i / Kp;
    const int k = (int)(i % Kp);
    double v = 0.0;
    if (k < K) {
        for (int o = 0; o < d; ++o) v = fma(W[(int64_t)k * d + o], E[s * d + o], v);
        v -= 1e-9 * (1.0 + fabs(v));
    }
    x[i] = (T)v;
}

void team_start(hipStream_t s, int64_t S, int K, int Kp, int d, const double* W, const double* E, int prec, void* x) {
    const int64_t n = S * Kp;
    if (n <= 0) return;
    const dim3 g((unsigned)((n + 255) / 256));
    if (prec == MORAP_F32)
        hipLaunchKernelGGL(team_start_kernel<float>, g, dim3(256), 0, s, S, K, Kp, d, W, E, (float*)x);
    else
        hipLaunchKernelGGL(team_start_kernel<double>, g, dim3(256), 0, s, S, K, Kp, d, W, E, (double*)x);
    MORAP_HIP(hipGetLastError());
}

void team_rewards(hipStream_t s, int64_t R, int K, int Kp, int d, const double* W, const int32_t* obj,
                  const double* rew, double* out64, float* out32) {
    const int64_t n = R * Kp;
    if (n <= 0) return;
    hipLaunchKernelGGL(team_rewards_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, R, K, Kp, d, W, obj,
                       rew, out64, out32);
    MORAP_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// convergence of (model, column) pairs and compaction of the active tiles
// ---------------------------------------------------------------------------
// Threads stride over the (model, column) pairs of the models active in the
// sweep just done.  counters: [0] active pairs (accumulating), [1] active
// tiles, [2] active models, [3] active pairs after the last sweep, [4]
// backups done, [5] sweeps done, [6] CSR bytes streamed, [7] state-columns
// updated (each one value read and one written), [8] pairs stopped at the
// FP32 rounding floor.  The three sums are reduced
// in the workgroup and added with one atomic each: thousands of atomics on
// the same counters would serialise in L2.
constexpr int kConvergeBlocks = 256;
template <class T>
__global__ void __launch_bounds__(256) converge_kernel(ConvergeArgs a) {
    const int64_t n = a.counters[2] * a.Kp;
    const int32_t next_sweep = (int32_t)(a.counters[5] + 1);
    unsigned long long bk = 0, sc = 0, cnt = 0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const int m = a.act_models[t / a.Kp];
        const int k = (int)(t % a.Kp);
        const int64_t i = (int64_t)m * a.Kp + k;
        bool still = false;
        if (a.active[i]) {
            const double r = __longlong_as_double((long long)a.res[i]);
            const double y = __longlong_as_double((long long)a.ymax[i]);
            const double tol = fmax(a.eps, a.unit * y);
            // Jacobi sweeps in FP32 can settle into a cycle: the values of
            // alternate sweeps form two chains (a state's new value reads its
            // neighbours' old ones) that can come to rest on two different
            // fixed points of the rounded backup, as far apart as a rounding
            // error amplified by the expected number of visits.  The change
            // then stays constant; such a pair stops at that floor.
            bool floor_stop = false;
            if (a.stall_sweeps > 0 && r > tol) {
                if (r < a.best_res[i]) {
                    a.best_res[i] = r;
                    a.stall[i] = 0;
                } else if (++a.stall[i] >= a.stall_sweeps && r <= a.floor * y) {
                    floor_stop = true;
                    atomicAdd((unsigned long long*)&a.counters[8], 1ull);
                }
            }
            if (r <= tol || floor_stop) {
                a.active[i] = 0;
                a.final_par[i] = (uint8_t)a.out_par;
                a.pair_sweeps[i] = next_sweep;
                const int32_t s0 = a.init[m];
                a.c[(int64_t)k * a.M + m] =
                    s0 >= 0 ? (double)((const T*)a.x_out)[(int64_t)s0 * a.Kp + k] : 0.0;
            } else {
                still = true;
                a.model_active[m] = 1;
            }
            a.res[i] = 0ull;
            a.ymax[i] = 0ull;
        }
        // backups of this sweep: rows of the model for every pair that was active
        if (still || a.pair_sweeps[i] == next_sweep) {
            bk += (unsigned long long)a.rows_per_model[m];
            sc += (unsigned long long)a.states_per_model[m];
        }
        cnt += still ? 1ull : 0ull;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        bk += __shfl_xor(bk, o, 64);
        sc += __shfl_xor(sc, o, 64);
        cnt += __shfl_xor(cnt, o, 64);
    }
    __shared__ unsigned long long part[3][4];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        part[0][w] = cnt;
        part[1][w] = bk;
        part[2][w] = sc;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const unsigned long long v = part[threadIdx.x][0] + part[threadIdx.x][1] + part[threadIdx.x][2] +
                                     part[threadIdx.x][3];
        const int slot = threadIdx.x == 0 ? 0 : (threadIdx.x == 1 ? 4 : 7);
        if (v) atomicAdd((unsigned long long*)&a.counters[slot], v);
    }
}

void converge(hipStream_t s, const ConvergeArgs& a) {
    const int64_t n = (int64_t)a.M * a.Kp;
    const unsigned blocks = (unsigned)std::min<int64_t>(kConvergeBlocks, std::max<int64_t>(1, (n + 255) / 256));
    if (a.prec == MORAP_F32)
        hipLaunchKernelGGL(converge_kernel<float>, dim3(blocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(converge_kernel<double>, dim3(blocks), dim3(256), 0, s, a);
    MORAP_HIP(hipGetLastError());
}

// Single workgroup: ordered list of active models with the exclusive prefix of
// their tile counts; publishes the pair count and advances the sweep counter.
__global__ void __launch_bounds__(1024) compact_kernel(ConvergeArgs a) {
    __shared__ int32_t part[1024];
    __shared__ int32_t partm[1024];
    const int tid = threadIdx.x;
    const int per = (a.M + 1023) / 1024;
    const int b = tid * per, e = min(a.M, b + per);
    int sum = 0, cnt = 0;
    unsigned long long bytes = 0;
    for (int m = b; m < e; ++m)
        if (a.model_active[m]) {
            sum += a.tile_base[m + 1] - a.tile_base[m];
            ++cnt;
            bytes += (unsigned long long)a.csr_bytes[m];
        }
    part[tid] = sum;
    partm[tid] = cnt;
    if (bytes && !a.relist) atomicAdd((unsigned long long*)&a.counters[6], bytes);
    __syncthreads();
    // inclusive scan (Hillis-Steele)
    for (int o = 1; o < 1024; o <<= 1) {
        int v = tid >= o ? part[tid - o] : 0;
        int w = tid >= o ? partm[tid - o] : 0;
        __syncthreads();
        part[tid] += v;
        partm[tid] += w;
        __syncthreads();
    }
    int off = tid ? part[tid - 1] : 0;
    int offm = tid ? partm[tid - 1] : 0;
    for (int m = b; m < e; ++m) {
        if (a.model_active[m]) {
            a.act_models[offm] = m;
            a.act_prefix[offm] = off;
            off += a.tile_base[m + 1] - a.tile_base[m];
            ++offm;
        }
        a.model_active[m] = 0;
    }
    if (tid == 1023) {
        a.act_prefix[offm] = off;
        a.counters[1] = off;
        a.counters[2] = offm;
        if (!a.relist) {
            a.counters[3] = a.counters[0];
            a.counters[0] = 0;
            a.counters[5] += 1;
        }
    }
}

// The active models' tiles as one ordered list (one workgroup per active
// model), so a sweep finds the tile of any position with one load.
__global__ void __launch_bounds__(64) expand_kernel(ConvergeArgs a) {
    const int b = blockIdx.x;
    if (b >= (int)a.counters[2]) return;
    const int m = a.act_models[b];
    const int base = a.act_prefix[b];
    const int t0 = a.tile_base[m], nt = a.tile_base[m + 1] - t0;
    for (int i = threadIdx.x; i < nt; i += 64) a.act_tiles[base + i] = t0 + i;
}

// the active models of the current lists, flagged again (for relist)
__global__ void remark_kernel(ConvergeArgs a) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < (int)a.counters[2]) a.model_active[a.act_models[b]] = 1;
}

void relist(hipStream_t s, ConvergeArgs a) {
    hipLaunchKernelGGL(remark_kernel, dim3((unsigned)((a.M + 255) / 256)), dim3(256), 0, s, a);
    MORAP_HIP(hipGetLastError());
    a.relist = 1;
    compact(s, a);
}

void compact(hipStream_t s, const ConvergeArgs& a) {
    hipLaunchKernelGGL(compact_kernel, dim3(1), dim3(1024), 0, s, a);
    MORAP_HIP(hipGetLastError());
    if (a.M > 0) hipLaunchKernelGGL(expand_kernel, dim3(a.M), dim3(64), 0, s, a);
    MORAP_HIP(hipGetLastError());
}

// start of a solve: columns k < K of models with a live initial state are
// active; everything else is cleared.
__global__ void init_solve_kernel(ConvergeArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = (int64_t)a.M * a.Kp;
    if (i < n) {
        const int m = (int)(i / a.Kp);
        const int k = (int)(i % a.Kp);
        const bool on = k < a.K && a.init[m] >= 0 && (a.mask == nullptr || a.mask[i] != 0);
        a.active[i] = on ? 1 : 0;
        a.final_par[i] = 0;
        a.pair_sweeps[i] = 0;
        a.res[i] = 0ull;
        a.ymax[i] = 0ull;
        a.best_res[i] = INFINITY;
        a.stall[i] = 0;
        if (on) a.model_active[m] = 1;
        if (k < a.K) a.c[(int64_t)k * a.M + m] = 0.0;
    }
    // the compaction that follows counts as no sweep: start the counter at -1
    if (i < 9) a.counters[i] = (i == 5) ? -1 : 0;
}

void init_solve(hipStream_t s, const ConvergeArgs& a) {
    const int64_t n = (int64_t)a.M * a.Kp;
    fill_u8(s, a.model_active, 0, a.M);
    hipLaunchKernelGGL(init_solve_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
    MORAP_HIP(hipGetLastError());
    compact(s, a);
}

// ---------------------------------------------------------------------------
// instances: (column, model) pairs, one thread per state
// ---------------------------------------------------------------------------
struct InstLoc {
    int inst, m, ls, S;
    int64_t is;      // instance state index
    int32_t gs;      // global state
    int32_t sb;      // model's first global state
};

__device__ __forceinline__ bool inst_locate(const InstArgs& a, InstLoc& L) {
    const int t = blockIdx.x;
    if (t >= a.n_tiles) return false;
    L.inst = a.inst_tiles[2 * t];
    L.ls = a.inst_tiles[2 * t + 1] + threadIdx.x;
    L.m = a.inst_model[L.inst];
    L.sb = a.state_base[L.m];
    L.S = a.state_base[L.m + 1] - L.sb;
    if (L.ls >= L.S) return false;
    L.is = a.inst_base[L.inst] + L.ls;
    L.gs = L.sb + L.ls;
    return true;
}

template <class T>
__global__ void gather_kernel(InstArgs a, const T* x0, const T* x1, const uint8_t* par, int Kp,
                              double* xi) {
    InstLoc L;
    if (!inst_locate(a, L)) return;
    const int k = a.inst_k[L.inst];
    const T* x = par[(int64_t)L.m * Kp + k] ? x1 : x0;
    xi[L.is] = (double)x[(int64_t)L.gs * Kp + k];
}

// Start of an FP32 solve from the previous solve's final values (the next
// pass of the same queries: their weights moved a little): out[s][k] =
// a[m][k] x_prev[s][map[k]] + b[m][k] from the buffer the pair froze in, 0
// where map[k] < 0 or a[m][k] = 0, and on the zero row.  The host picks a
// and b (see solve); ab holds the pairs (a, b).
__global__ void warm_columns_kernel(int64_t n, int Kp, int K, const int32_t* __restrict__ map,
                                    const int32_t* __restrict__ state_model, int64_t S,
                                    const float2* __restrict__ ab, const float* __restrict__ x0,
                                    const float* __restrict__ x1, const uint8_t* __restrict__ par, int Kp_old,
                                    float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t s = i / Kp;
    const int k = (int)(i % Kp);
    float v = 0.f;
    if (s < S && k < K) {
        const int ko = map[k];
        if (ko >= 0) {
            const int m = state_model[s];
            const float2 f = ab[(int64_t)m * Kp + k];
            if (f.x != 0.f) {
                const float* x = par[(int64_t)m * Kp_old + ko] ? x1 : x0;
                v = fmaf(f.x, x[s * Kp_old + ko], f.y);
            }
        }
    }
    out[i] = v;
}

void warm_columns(hipStream_t s, int64_t S, int Kp, int K, const int32_t* map, const int32_t* state_model,
                  const float* ab, const float* x0, const float* x1, const uint8_t* final_par, int Kp_old,
                  float* out) {
    const int64_t n = (S + 1) * Kp;
    hipLaunchKernelGGL(warm_columns_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, Kp, K, map,
                       state_model, S, reinterpret_cast<const float2*>(ab), x0, x1, final_par, Kp_old, out);
    MORAP_HIP(hipGetLastError());
}

// Start of the FP64 re-solve of an instance from the FP32 solve's values of
// its pair: the optimal values of the model scale with its two weights, so
// x = x32 / (w_i + w_j) (scale[inst] = 1 / (w_i + w_j)).  Only instances
// whose scaled cost weight is positive start there: every improper policy
// then loses without bound and the Bellman operator has one fixed point,
// reached from any start.  With a zero cost weight zero-reward loops admit
// larger fixed points, and those instances start from 0 as Alg. 3 does.
__global__ void warm_kernel(InstArgs a, const float* x0, const float* x1, const uint8_t* par, int Kp,
                            const double* scale, const double* iwc, double* xi) {
    InstLoc L;
    if (!inst_locate(a, L)) return;
    double v = 0.0;
    if (iwc[L.inst] > 0.0) {
        const int k = a.inst_k[L.inst];
        const float* x = par[(int64_t)L.m * Kp + k] ? x1 : x0;
        v = (double)x[(int64_t)L.gs * Kp + k] * scale[L.inst];
    }
    xi[L.is] = v;
}

void warm_start(hipStream_t s, const InstArgs& a, const void* x0, const void* x1, const uint8_t* final_par, int Kp,
                const double* scale, const double* iwc, double* xi) {
    if (a.n_tiles <= 0) return;
    hipLaunchKernelGGL(warm_kernel, dim3(a.n_tiles), dim3(256), 0, s, a, (const float*)x0, (const float*)x1,
                       final_par, Kp, scale, iwc, xi);
    MORAP_HIP(hipGetLastError());
}

void gather_columns(hipStream_t s, const InstArgs& a, int prec, const void* x0, const void* x1,
                    const uint8_t* final_par, int Kp, double* xi) {
    if (a.n_tiles <= 0) return;
    if (prec == MORAP_F32)
        hipLaunchKernelGGL(gather_kernel<float>, dim3(a.n_tiles), dim3(256), 0, s, a, (const float*)x0,
                           (const float*)x1, final_par, Kp, xi);
    else
        hipLaunchKernelGGL(gather_kernel<double>, dim3(a.n_tiles), dim3(256), 0, s, a, (const double*)x0,
                           (const double*)x1, final_par, Kp, xi);
    MORAP_HIP(hipGetLastError());
}

// One workgroup: the stop test of every entry (entry i stops when res[i] <=
// eps; its final buffer parity is recorded), residuals cleared, and the
// number still running written to *counter (no separate clearing launch).
__global__ void __launch_bounds__(1024) inst_converge_kernel(int n, unsigned long long* res, uint8_t* active,
                                                             uint8_t* par, int out_par, double eps,
                                                             int64_t* counter, const double* eps_i) {
    unsigned long long still = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        if (!active[i]) continue;
        const double r = __longlong_as_double((long long)res[i]);
        if (r <= (eps_i ? eps_i[i] : eps)) {
            active[i] = 0;
            par[i] = (uint8_t)out_par;
        } else {
            ++still;
        }
        res[i] = 0ull;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) still += __shfl_xor(still, o, 64);
    __shared__ unsigned long long part[16];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = still;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long total = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) total += part[w];
        *counter = (int64_t)total;
    }
}

void inst_converge(hipStream_t s, int n, unsigned long long* res, uint8_t* active, uint8_t* par,
                   int out_par, double eps, int64_t* counter, const double* eps_i) {
    if (n <= 0) {
        fill_i64(s, counter, 0, 1);
        return;
    }
    hipLaunchKernelGGL(inst_converge_kernel, dim3(1), dim3(1024), 0, s, n, res, active, par, out_par, eps,
                       counter, eps_i);
    MORAP_HIP(hipGetLastError());
}

// eps-optimal rows of every state: bit r of mask = row r (local) has
// Q(s, r) >= max_a Q(s, a) - tau, with Q in FP64 at the final values.
// With `only_unranked` the masks of ranked states are kept and only unranked
// states get the (wider) tolerance; otherwise every state starts unranked.
__global__ void __launch_bounds__(256) opt_mask_kernel(InstArgs a, const double* wc, const double* wp,
                                                       const double* x, double tau, uint32_t* mask,
                                                       int32_t* rank, int8_t* mu, int only_unranked) {
    InstLoc L;
    if (!inst_locate(a, L)) return;
    if (only_unranked && rank[L.is] >= 0) return;
    const int64_t ib = a.inst_base[L.inst];
    const double w0 = wc[L.inst], w1 = wp[L.inst];
    const int rb = a.state_row[L.gs], re = a.state_row[L.gs + 1];
    const int kk = a.inst_k[L.inst];
    // a row's scalarised reward: the instance's two weights, or for a team
    // model the row's own objectives (rewk)
    auto reward = [&](int row) {
        return a.rewk ? a.rewk[(int64_t)row * a.rewk_ld + kk] : w0 * a.rew[2 * row] + w1 * a.rew[2 * row + 1];
    };
    // two passes (max, then the tolerance test) keep Q out of scratch memory
    double qmax = -INFINITY;
    for (int row = rb; row < re; ++row) {
        double acc = reward(row);
        for (int e = a.row_ptr[row]; e < a.row_ptr[row + 1]; ++e)
            acc = fma(a.prob[e], x[ib + (a.col[e] - L.sb)], acc);
        qmax = fmax(qmax, acc);
    }
    uint32_t bits = 0;
    for (int row = rb; row < re; ++row) {
        double acc = reward(row);
        for (int e = a.row_ptr[row]; e < a.row_ptr[row + 1]; ++e)
            acc = fma(a.prob[e], x[ib + (a.col[e] - L.sb)], acc);
        if (acc >= qmax - tau) bits |= 1u << (row - rb);
    }
    mask[L.is] = bits;
    if (!only_unranked) {
        rank[L.is] = -1;
        mu[L.is] = -1;
    }
}

void opt_mask(hipStream_t s, const InstArgs& a, const double* wc, const double* wp, const double* x,
              double tau, uint32_t* mask, int32_t* rank, int8_t* mu, bool only_unranked) {
    if (a.n_tiles <= 0) return;
    hipLaunchKernelGGL(opt_mask_kernel, dim3(a.n_tiles), dim3(256), 0, s, a, wc, wp, x, tau, mask, rank, mu,
                       only_unranked ? 1 : 0);
    MORAP_HIP(hipGetLastError());
}

// Instance state of thread threadIdx.x in tile t (as inst_locate).
__device__ __forceinline__ bool inst_locate_tile(const InstArgs& a, int t, InstLoc& L) {
    L.inst = a.inst_tiles[2 * t];
    L.ls = a.inst_tiles[2 * t + 1] + threadIdx.x;
    L.m = a.inst_model[L.inst];
    L.sb = a.state_base[L.m];
    L.S = a.state_base[L.m + 1] - L.sb;
    if (L.ls >= L.S) return false;
    L.is = a.inst_base[L.inst] + L.ls;
    L.gs = L.sb + L.ls;
    return true;
}

// Attractor ranks as BFS distances.  The rank of a state is its distance to
// done in the graph whose edges are the successors of its tau-optimal rows
// (done at 0), which is the round in which the level-synchronous attractor
// ranks it.  States ranked in an earlier phase (rank <= base) are sources
// at distance base.  The relaxation runs in place: a tile's states are
// relaxed up to `local` times per launch (neighbours inside the tile
// propagate within one launch) and read other tiles' current ranks; ranks
// only decrease, so the fixed point is the exact distance in any order.
// rank < 0 means not (yet) ranked.
__global__ void __launch_bounds__(256) relax_kernel(InstArgs a, const uint32_t* mask, int32_t* rank, int base,
                                                    int reverse, int local, int64_t* changed,
                                                    uint8_t* inst_changed) {
    const int t = reverse ? a.n_tiles - 1 - (int)blockIdx.x : (int)blockIdx.x;
    InstLoc L;
    const bool ok = inst_locate_tile(a, t, L);
    const bool mine = ok && (rank[L.is] < 0 || rank[L.is] > base);
    int64_t ib = 0;
    int rb = 0;
    uint32_t bits0 = 0;
    if (mine) {
        ib = a.inst_base[L.inst];
        rb = a.state_row[L.gs];
        bits0 = mask[L.is];
    }
    unsigned long long n_upd = 0;
    for (int it = 0; it < local; ++it) {
        int upd = 0;
        if (mine) {
            const int cur = rank[L.is];
            int cand = 0x7FFFFFFF;
            uint32_t bits = bits0;
            while (bits) {
                const int row = rb + __builtin_ctz(bits);
                bits &= bits - 1;
                if (a.to_done[row]) cand = min(cand, base + 1);
                for (int e = a.row_ptr[row]; e < a.row_ptr[row + 1]; ++e) {
                    const int32_t d = rank[ib + (a.col[e] - L.sb)];
                    if (d >= 0) cand = min(cand, max(d, base) + 1);
                }
            }
            if (cand != 0x7FFFFFFF && (cur < 0 || cand < cur)) {
                rank[L.is] = cand;
                upd = 1;
            }
        }
        n_upd += upd;
        if (!__syncthreads_or(upd)) break;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) n_upd += __shfl_xor(n_upd, o, 64);
    if ((threadIdx.x & 63) == 0 && n_upd) {
        atomicAdd((unsigned long long*)changed, n_upd);
        // the instance is not at its fixed point yet (ranks spread only
        // inside an instance, so one without updates for a whole round is)
        inst_changed[a.inst_tiles[2 * t]] = 1;
    }
}

void relax_ranks(hipStream_t s, const InstArgs& a, const uint32_t* mask, int32_t* rank, int base, bool reverse,
                 int local, int64_t* changed, uint8_t* inst_changed) {
    if (a.n_tiles <= 0) return;
    hipLaunchKernelGGL(relax_kernel, dim3(a.n_tiles), dim3(256), 0, s, a, mask, rank, base, reverse ? 1 : 0,
                       local, changed, inst_changed);
    MORAP_HIP(hipGetLastError());
}

// The action of every state ranked above `base`: among its tau-optimal rows
// that move mass into done or into states of lower rank, the one moving the
// most mass there (masses within 1e-12 are equal; then the lowest row).
// Also records the largest rank in counter[0].
__global__ void __launch_bounds__(256) choose_kernel(InstArgs a, const uint32_t* mask, const int32_t* rank,
                                                     int8_t* mu, int base, int64_t* max_rank) {
    InstLoc L;
    int top = 0;
    if (inst_locate(a, L) && rank[L.is] > base) {
        const int level = rank[L.is];
        top = level;
        const int64_t ib = a.inst_base[L.inst];
        const int rb = a.state_row[L.gs];
        uint32_t bits = mask[L.is];
        int best_lr = -1;
        double best_m = -1.0;
        while (bits) {
            const int lr = __builtin_ctz(bits);
            bits &= bits - 1;
            const int row = rb + lr;
            const int e0 = a.row_ptr[row], e1 = a.row_ptr[row + 1];
            bool hit = a.to_done[row] != 0;
            double m = 0.0;
            if (hit) {
                double live = 0.0;
                for (int e = e0; e < e1; ++e) live += a.prob[e];
                m = 1.0 - live;
            }
            for (int e = e0; e < e1; ++e) {
                const int32_t rk = rank[ib + (a.col[e] - L.sb)];
                if (rk >= 0 && rk < level) {
                    hit = true;
                    m += a.prob[e];
                }
            }
            if (hit && m > best_m + 1e-12) {
                best_m = m;
                best_lr = lr;
            }
        }
        mu[L.is] = (int8_t)best_lr;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) top = max(top, __shfl_xor(top, o, 64));
    if ((threadIdx.x & 63) == 0 && top) atomicMax((unsigned long long*)max_rank, (unsigned long long)top);
}

void choose_actions(hipStream_t s, const InstArgs& a, const uint32_t* mask, const int32_t* rank, int8_t* mu,
                    int base, int64_t* max_rank) {
    if (a.n_tiles <= 0) return;
    hipLaunchKernelGGL(choose_kernel, dim3(a.n_tiles), dim3(256), 0, s, a, mask, rank, mu, base, max_rank);
    MORAP_HIP(hipGetLastError());
}

__global__ void count_unranked_kernel(InstArgs a, const int32_t* rank, int64_t* counter) {
    InstLoc L;
    unsigned long long bad = 0;
    if (inst_locate(a, L) && rank[L.is] < 0) bad = 1;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) bad += __shfl_xor(bad, o, 64);
    if ((threadIdx.x & 63) == 0 && bad) atomicAdd((unsigned long long*)counter, bad);
}

void count_unranked(hipStream_t s, const InstArgs& a, const int32_t* rank, int64_t* counter) {
    if (a.n_tiles <= 0) return;
    hipLaunchKernelGGL(count_unranked_kernel, dim3(a.n_tiles), dim3(256), 0, s, a, rank, counter);
    MORAP_HIP(hipGetLastError());
}

// Alg. 4: fixed-policy Jacobi sweep for both objectives (cost, probability);
// x is [instance state][2]; active / res are per (instance, objective).
__global__ void __launch_bounds__(256) eval_kernel(InstArgs a, const int8_t* mu, const uint8_t* active,
                                                   const double* x_in, double* x_out,
                                                   unsigned long long* res) {
    InstLoc L;
    const bool ok = inst_locate(a, L);
    double r0 = 0.0, r1 = 0.0;
    if (ok) {
        const bool a0 = active[2 * L.inst] != 0, a1 = active[2 * L.inst + 1] != 0;
        if (a0 || a1) {
            const int64_t ib = a.inst_base[L.inst];
            const int row = a.state_row[L.gs] + mu[L.is];
            double c0 = a.rew[2 * row], c1 = a.rew[2 * row + 1];
            if (a.row_obj) {
                // team model: the instance evaluates objectives o0 and o1;
                // each of the row's rewards counts for the objective it
                // belongs to
                const int o0 = a.inst_obj[2 * L.inst], o1 = a.inst_obj[2 * L.inst + 1];
                const int oc = a.row_obj[2 * row], op = a.row_obj[2 * row + 1];
                const double rc = a.rew[2 * row], rp = a.rew[2 * row + 1];
                c0 = (oc == o0 ? rc : 0.0) + (op == o0 ? rp : 0.0);
                c1 = (oc == o1 ? rc : 0.0) + (op == o1 ? rp : 0.0);
            }
            for (int e = a.row_ptr[row]; e < a.row_ptr[row + 1]; ++e) {
                const int64_t j = ib + (a.col[e] - L.sb);
                const double2 v = reinterpret_cast<const double2*>(x_in)[j];
                c0 = fma(a.prob[e], v.x, c0);
                c1 = fma(a.prob[e], v.y, c1);
            }
            const double2 old = reinterpret_cast<const double2*>(x_in)[L.is];
            if (a0) { x_out[2 * L.is] = c0; r0 = fabs(c0 - old.x); }
            if (a1) { x_out[2 * L.is + 1] = c1; r1 = fabs(c1 - old.y); }
        }
    }
    r0 = wave_max(r0);
    r1 = wave_max(r1);
    if ((threadIdx.x & 63) == 0) {
        const int i0 = a.inst_tiles[2 * blockIdx.x];
        if (r0 > 0.0) atomicMax(&res[2 * i0], (unsigned long long)__double_as_longlong(r0));
        if (r1 > 0.0) atomicMax(&res[2 * i0 + 1], (unsigned long long)__double_as_longlong(r1));
    }
}

void eval_sweep(hipStream_t s, const InstArgs& a, const int8_t* mu, const uint8_t* active,
                const double* x_in, double* x_out, unsigned long long* res) {
    if (a.n_tiles <= 0) return;
    hipLaunchKernelGGL(eval_kernel, dim3(a.n_tiles), dim3(256), 0, s, a, mu, active, x_in, x_out, res);
    MORAP_HIP(hipGetLastError());
}

__global__ void set_active_kernel(int n, k::InstArgs a, uint8_t* active, unsigned long long* res,
                                  uint8_t* par, int width) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * width) return;
    const int m = a.inst_model[i / width];
    active[i] = a.init[m] >= 0 ? 1 : 0;
    res[i] = 0ull;
    par[i] = 0;
}

void set_active(hipStream_t s, int n, const InstArgs& a, uint8_t* active, unsigned long long* res,
                uint8_t* par, int width) {
    if (n <= 0) return;
    hipLaunchKernelGGL(set_active_kernel, dim3((n * width + 255) / 256), dim3(256), 0, s, n, a, active, res,
                       par, width);
    MORAP_HIP(hipGetLastError());
}

__global__ void select_final_kernel(InstArgs a, double* x0, const double* x1, const uint8_t* par, int width) {
    InstLoc L;
    if (!inst_locate(a, L)) return;
    for (int o = 0; o < width; ++o)
        if (par[(int64_t)L.inst * width + o]) x0[L.is * width + o] = x1[L.is * width + o];
}

// runs (dst, src, length) of instance states: x[dst + i][2] = prev[src + i][2]
__global__ void copy_runs_kernel(const int64_t* __restrict__ runs, int n_runs, const double* __restrict__ prev,
                                 double* __restrict__ x) {
    const int r = blockIdx.x;
    if (r >= n_runs) return;
    const int64_t dst = runs[3 * r], src = runs[3 * r + 1], len = runs[3 * r + 2];
    for (int64_t i = threadIdx.x; i < 2 * len; i += blockDim.x) x[2 * dst + i] = prev[2 * src + i];
}

void copy_runs(hipStream_t s, const int64_t* runs, int n_runs, const double* prev, double* x) {
    if (n_runs <= 0) return;
    hipLaunchKernelGGL(copy_runs_kernel, dim3(n_runs), dim3(256), 0, s, runs, n_runs, prev, x);
    MORAP_HIP(hipGetLastError());
}

// Start of the per-objective evaluation from the instance's scalarised
// values V = w_c C + w_p P (weights scaled to sum 1, the values its policy
// was chosen from): the probability objective at its warm value where the
// instance was warm-started, else 1 (its value under any proper policy of a
// task without a trap); the cost objective at (V - w_p P0) / w_c where
// w_c >= 1e-3 (below, the division would magnify V's own error), else as it
// was.  For a policy greedy for V the start is its value up to V's error.
__global__ void eval_start_kernel(InstArgs a, const double* __restrict__ xi, const double* __restrict__ iwc,
                                  const double* __restrict__ iwp, const uint8_t* __restrict__ iwarm,
                                  double* __restrict__ xe) {
    InstLoc L;
    if (!inst_locate(a, L)) return;
    const double wc = iwc[L.inst], wp = iwp[L.inst];
    const double p0 = iwarm[L.inst] ? xe[2 * L.is + 1] : 1.0;
    xe[2 * L.is + 1] = p0;
    if (wc >= 1e-3) xe[2 * L.is] = (xi[L.is] - wp * p0) / wc;
}

void eval_start(hipStream_t s, const InstArgs& a, const double* xi, const double* iwc, const double* iwp,
                const uint8_t* iwarm, double* xe) {
    if (a.n_tiles <= 0) return;
    hipLaunchKernelGGL(eval_start_kernel, dim3(a.n_tiles), dim3(256), 0, s, a, xi, iwc, iwp, iwarm, xe);
    MORAP_HIP(hipGetLastError());
}

void select_final(hipStream_t s, const InstArgs& a, double* x0, const double* x1, const uint8_t* par,
                  int width) {
    if (a.n_tiles <= 0) return;
    hipLaunchKernelGGL(select_final_kernel, dim3(a.n_tiles), dim3(256), 0, s, a, x0, x1, par, width);
    MORAP_HIP(hipGetLastError());
}

__global__ void mark_pairs_kernel(InstArgs a, int Kp, uint8_t* mask) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= a.n_inst) return;
    mask[(int64_t)a.inst_model[q] * Kp + a.inst_k[q]] = 1;
}

void mark_pairs(hipStream_t s, const InstArgs& a, int Kp, uint8_t* mask) {
    if (a.n_inst <= 0) return;
    hipLaunchKernelGGL(mark_pairs_kernel, dim3((a.n_inst + 255) / 256), dim3(256), 0, s, a, Kp, mask);
    MORAP_HIP(hipGetLastError());
}

__global__ void gather_init_kernel(int n, const int64_t* idx, const double* x, double* out) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int64_t i = idx[q];
    out[2 * q] = i >= 0 ? x[2 * i] : 0.0;
    out[2 * q + 1] = i >= 0 ? x[2 * i + 1] : 0.0;
}

void gather_init(hipStream_t s, int n, const int64_t* idx, const double* x, double* out) {
    if (n <= 0) return;
    hipLaunchKernelGGL(gather_init_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, idx, x, out);
    MORAP_HIP(hipGetLastError());
}

}  // namespace k
}  // namespace morap
