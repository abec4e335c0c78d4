// Batched Bellman sweep over the neighbourhood-block form of the products
// (Alg. 3, one Jacobi sweep of scalarised max-backups for every active
// (model, column) pair).
//
// In a product M_i (x) A_j the transition probabilities of (s, q) under an
// action are those of the agent state s (Sec. 2, "Product MDP"); only which
// product state each agent successor lands in, and whether it is done,
// depends on q.  When every agent state has at most 5 actions and at most 5
// distinct successors (the state itself counted), one product state is fully
// described by
//   * a 32-byte record: the global product state of each of the 5 agent
//     successor slots (the zero row when the slot is unused or its successor
//     is done), the index of its agent state's block, the slots that enter an
//     accepting location, the enabled actions and the state itself (records
//     are stored in the order a tile is walked: column by column on grids);
//   * its agent state's block: P[a][d] over (action, slot) and -cost[a] (a
//     disabled action repeats the first enabled one),
//     shared by every location and every task of that agent.
// A backup then reads the record, the (cached) agent block and 5 successor
// value rows; the probability-reward column is the mass the action puts on
// accepting slots.  There is no barrier: each XCD takes a contiguous eighth
// of the active tiles and its waves take every n-th of them, so neighbouring
// tiles (which share successor rows) are processed at the same time and their
// rows meet in that XCD's L2; a wave walks its tile's states `U` at a time
// with all successor gathers of those states in flight, and lanes map to
// columns.  With 64 lanes per state the record, the block and every branch are
// wave-uniform (scalar loads and branches).
#include "common.h"
#include "kern.h"

#include <cfloat>
#include <type_traits>

namespace morap {
namespace k {

constexpr int NSLOT = 5;
constexpr int BLK = 32;   // values per agent block

// Sparsity patterns of the blocks (bit 5a + d = entry P[a][d] may be nonzero):
// every entry, or the grid pattern of the host's slot order (slot 0 = stay,
// 1 + a = the cell move a aims at; the N/S moves slip E/W and vice versa).
constexpr uint32_t PAT_DENSE = (1u << 25) - 1;
constexpr uint32_t PAT_GRID = (1u << 0) | (1u << 1) | (1u << 3) | (1u << 4) |        // N: stay, N, E, W
                              (1u << 5) | (1u << 7) | (1u << 8) | (1u << 9) |        // S: stay, S, E, W
                              (1u << 10) | (1u << 11) | (1u << 12) | (1u << 13) |    // E: stay, N, S, E
                              (1u << 15) | (1u << 16) | (1u << 17) | (1u << 19) |    // W: stay, N, S, W
                              (1u << 20);                                            // stay
template <uint32_t PAT>
__device__ __forceinline__ constexpr bool nz(int a, int d) { return (PAT >> (a * NSLOT + d)) & 1u; }

static uint32_t pattern_for(uint32_t union_pattern) {
    return (union_pattern & ~PAT_GRID) == 0 ? PAT_GRID : PAT_DENSE;
}

template <class T, int CPL, int LPS, int U, int WG, uint32_t PAT>
__global__ void __launch_bounds__(WG)
bellman_block(const Tile* __restrict__ tiles,
              const int32_t* __restrict__ act_tiles, const int64_t* __restrict__ counters,
              const int32_t* __restrict__ rec,
              const T* __restrict__ ablk, const T* __restrict__ wc_all, const T* __restrict__ wp_all,
              const uint8_t* __restrict__ active_all, const T* __restrict__ x_in, T* __restrict__ x_out,
              unsigned long long* __restrict__ res_all, unsigned long long* __restrict__ ymax_all, int Kp,
              int32_t zero_row) {
    constexpr int SPW = 64 / LPS;          // states per wave step
    constexpr int KT = CPL * LPS;          // columns per k-tile
    constexpr int NW = WG / 64;
    constexpr bool want_ymax = sizeof(T) == 4;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int g = lane / LPS;              // state slot within a step
    const int gl = lane % LPS;
    const int kc = blockIdx.y * KT + gl * CPL;

    // work units: active tiles, split in `sub` parts when there are fewer
    // tiles than waves
    const int n_tiles = (int)counters[1];
    const int n_waves = gridDim.x * NW;
    const int sub = n_tiles * 4 <= n_waves ? 4 : (n_tiles * 2 <= n_waves ? 2 : 1);
    const int n_units = n_tiles * sub;
    // XCD x takes the units [xb, xe); its waves take every count-th unit of
    // it, so neighbouring units (which share successor rows) are in flight
    // together and their rows meet in the XCD's L2
    const int count = (gridDim.x >> 3) * NW;
    const int xb = (int)((int64_t)n_units * (blockIdx.x & 7) / 8);
    const int xe = (int)((int64_t)n_units * ((blockIdx.x & 7) + 1) / 8);
    const int u_begin = xb + (int)(blockIdx.x >> 3) * NW + wave;
    if (u_begin >= xe) return;
    int cur_m = -1;
    bool on = false;
    T wc[CPL], wp[CPL];
    bool act[CPL];
    double res[CPL], ym[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        res[c] = ym[c] = 0.0;
        wc[c] = wp[c] = 0;
        act[c] = false;
    }

    auto flush = [&](int m) {
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            res[c] = group_max<LPS>(res[c]);
            if (want_ymax) ym[c] = group_max<LPS>(ym[c]);
        }
        if (lane < LPS) {
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                const int64_t idx = (int64_t)m * Kp + kc + c;
                max_flush(&res_all[idx], res[c]);
                if (want_ymax) max_flush(&ymax_all[idx], ym[c]);
            }
        }
#pragma unroll
        for (int c = 0; c < CPL; ++c) res[c] = ym[c] = 0.0;
    };

    for (int u = u_begin; u < xe; u += count) {
        const int t = u / sub, part = u - t * sub;
        const Tile tl = tiles[act_tiles[t]];
        const int m = tl.model;
        if (m != cur_m) {
            if (cur_m >= 0) flush(cur_m);
            cur_m = m;
            bool any = false;
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                const int64_t kk = (int64_t)m * Kp + kc + c;
                wc[c] = wc_all[kk];
                wp[c] = wp_all[kk];
                act[c] = active_all[kk] != 0;
                any |= act[c];
            }
            on = __ballot(any) != 0;
        }
        if (!on) continue;
        const int len = tl.s_end - tl.s_begin;
        const int sb = tl.s_begin + (len * part) / sub;
        const int se = tl.s_begin + (len * (part + 1)) / sub;

        for (int s = sb; s < se; s += U * SPW) {
            int gs[U];
            bool ok[U];
            int32_t sc[U][NSLOT], bi[U], fl[U];
#pragma unroll
            for (int q = 0; q < U; ++q) {
                const int pos = s + q * SPW + g;   // record position; the record names its state
                ok[q] = pos < se;
                gs[q] = 0;
                if (ok[q]) {
                    const int32_t* r = rec + (int64_t)pos * 8;
                    const int4 r0 = *reinterpret_cast<const int4*>(r);
                    const int4 r1 = *reinterpret_cast<const int4*>(r + 4);
                    sc[q][0] = r0.x; sc[q][1] = r0.y; sc[q][2] = r0.z; sc[q][3] = r0.w;
                    sc[q][4] = r1.x; bi[q] = r1.y; fl[q] = r1.z;
                    gs[q] = r1.w;
                } else {
#pragma unroll
                    for (int d = 0; d < NSLOT; ++d) sc[q][d] = zero_row;
                    bi[q] = 0;
                    fl[q] = 0;
                }
            }
            // every successor gather of the U states in flight together
            Vec<T, CPL> xv[U][NSLOT];
#pragma unroll
            for (int q = 0; q < U; ++q)
#pragma unroll
                for (int d = 0; d < NSLOT; ++d) {
                    const T* row = x_in + (int64_t)sc[q][d] * Kp;
                    xv[q][d] = vload<T, CPL>(row + kc);
                }
#pragma unroll
            for (int q = 0; q < U; ++q) {
                if (!ok[q]) continue;
                // the agent block: P[a][d] (25 values), then -cost[a] (5)
                T B[BLK];
                {
                    using V4 = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
                    constexpr int PER = sizeof(V4) / sizeof(T);
                    const V4* src = reinterpret_cast<const V4*>(ablk + (int64_t)bi[q] * BLK);
#pragma unroll
                    for (int i = 0; i < BLK / PER; ++i) {
                        const V4 v = src[i];
                        if constexpr (PER == 4) {
                            B[4 * i] = v.x; B[4 * i + 1] = v.y; B[4 * i + 2] = v.z; B[4 * i + 3] = v.w;
                        } else {
                            B[2 * i] = v.x; B[2 * i + 1] = v.y;
                        }
                    }
                }
                const int accm = fl[q] & 31;
                // the state's own value (slot 0 unless its self-successor
                // changes location or is done)
                Vec<T, CPL> old = xv[q][0];
                if (sc[q][0] != gs[q]) old = vload<T, CPL>(x_in + (int64_t)gs[q] * Kp + kc);
                T best[CPL];
#pragma unroll
                for (int c = 0; c < CPL; ++c) best[c] = -INFINITY;
#pragma unroll
                for (int a = 0; a < 5; ++a) {
                    // probability reward: the action's mass on accepting slots
                    T rp = 0;
                    if (accm) {
#pragma unroll
                        for (int d = 0; d < NSLOT; ++d)
                            if (nz<PAT>(a, d) && ((accm >> d) & 1)) rp += B[a * NSLOT + d];
                    }
#pragma unroll
                    for (int c = 0; c < CPL; ++c) {
                        T acc = wc[c] * B[25 + a];
                        if (accm) acc = fma(wp[c], rp, acc);
#pragma unroll
                        for (int d = 0; d < NSLOT; ++d)
                            if (nz<PAT>(a, d)) acc = fma(B[a * NSLOT + d], xv[q][d].v[c], acc);
                        best[c] = fmax(best[c], acc);
                    }
                }
                const int64_t o = (int64_t)gs[q] * Kp + kc;
#pragma unroll
                for (int c = 0; c < CPL; ++c) {
                    if (act[c]) {
                        x_out[o + c] = best[c];
                        res[c] = fmax(res[c], (double)fabs(best[c] - old.v[c]));
                        if (want_ymax) ym[c] = fmax(ym[c], fabs((double)best[c]));
                    }
                }
            }
        }
    }
    if (cur_m >= 0) flush(cur_m);
}

// One state per wave step, lane = column (64 columns per k-tile): the
// record fields, the agent block and every branch are wave-uniform, so the
// block sits in scalar registers and the vector unit only does the backup
// arithmetic.  A work unit's records are staged with one coalesced load per
// lane (lane i holds the record of the unit's i-th state) and the next unit's
// records are fetched while the current one is processed; U states have their
// successor gathers in flight together.
struct UnitDesc {
    int m, sb, se;
};

template <class T, int U, int WG, uint32_t PAT>
__global__ void __launch_bounds__(WG)
bellman_block_wave(const Tile* __restrict__ tiles,
                   const int32_t* __restrict__ act_tiles, const int64_t* __restrict__ counters,
                   const int32_t* __restrict__ rec,
                   const T* __restrict__ ablk, const T* __restrict__ wc_all, const T* __restrict__ wp_all,
                   const uint8_t* __restrict__ active_all, const T* __restrict__ x_in, T* __restrict__ x_out,
                   unsigned long long* __restrict__ res_all, unsigned long long* __restrict__ ymax_all, int Kp,
                   int32_t zero_row) {
    constexpr int NW = WG / 64;
    constexpr bool want_ymax = sizeof(T) == 4;
    // each wave's records of its current unit (lane i wrote records i and
    // 64 + i); a unit is at most one tile of 128 states
    constexpr int RPL = 2;
    __shared__ int4 l_rec[NW][64 * RPL][2];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const unsigned kc = blockIdx.y * 64u + (unsigned)lane;

    const int n_tiles = (int)counters[1];
    const int n_waves = gridDim.x * NW;
    const int sub = n_tiles * 4 <= n_waves ? 4 : (n_tiles * 2 <= n_waves ? 2 : 1);
    const int n_units = n_tiles * sub;
    // XCD x takes the units [xb, xe); its waves take every count-th unit of
    // it, so neighbouring units (which share successor rows) are in flight
    // together and their rows meet in the XCD's L2
    const int count = (gridDim.x >> 3) * NW;
    const int xb = (int)((int64_t)n_units * (blockIdx.x & 7) / 8);
    const int xe = (int)((int64_t)n_units * ((blockIdx.x & 7) + 1) / 8);
    const int u_begin = xb + (int)(blockIdx.x >> 3) * NW + wave;
    if (u_begin >= xe) return;

    // unit -> (model, state range)
    auto describe = [&](int u) {
        const int t = u / sub, part = u - t * sub;
        const Tile tl = tiles[act_tiles[t]];
        const int len = tl.s_end - tl.s_begin;
        return UnitDesc{tl.model, tl.s_begin + (len * part) / sub, tl.s_begin + (len * (part + 1)) / sub};
    };
    // records are read once per sweep: streaming loads keep them from
    // displacing value rows in the caches
    auto stage = [&](const UnitDesc& d, int4 (&rr)[RPL][2]) {
#pragma unroll
        for (int h = 0; h < RPL; ++h) {
            if (64 * h + lane < d.se - d.sb) {
                typedef int i32x4 __attribute__((ext_vector_type(4)));
                const i32x4* r = reinterpret_cast<const i32x4*>(rec + (int64_t)(d.sb + 64 * h + lane) * 8);
                const i32x4 v0 = __builtin_nontemporal_load(r), v1 = __builtin_nontemporal_load(r + 1);
                rr[h][0] = make_int4(v0.x, v0.y, v0.z, v0.w);
                rr[h][1] = make_int4(v1.x, v1.y, v1.z, v1.w);
            }
        }
    };

    int cur_m = -1;
    bool on = false, act = false;
    T wc = 0, wp = 0;
    // the change |y - x| in T: for FP32 exact whenever y and x are within a
    // factor of two of each other (Sterbenz), as near the stop test
    T res = 0, ym = 0;
    auto flush = [&](int m) {
        const int64_t idx = (int64_t)m * Kp + kc;
        max_flush(&res_all[idx], (double)res);
        if (want_ymax) max_flush(&ymax_all[idx], (double)ym);
        res = ym = 0;
    };

    UnitDesc nd = describe(u_begin);
    int4 nr[RPL][2];
#pragma unroll
    for (int h = 0; h < RPL; ++h) nr[h][0] = nr[h][1] = make_int4(0, 0, 0, 0);
    stage(nd, nr);
    for (int u = u_begin; u < xe; u += count) {
        const UnitDesc d = nd;
        // publish this unit's records to the wave's LDS slots (same-wave
        // LDS accesses are ordered: no barrier), then fetch the next unit's
#pragma unroll
        for (int h = 0; h < RPL; ++h) {
            l_rec[wave][64 * h + lane][0] = nr[h][0];
            l_rec[wave][64 * h + lane][1] = nr[h][1];
        }
        if (u + count < xe) {
            nd = describe(u + count);
            stage(nd, nr);
        }
        if (d.m != cur_m) {
            if (cur_m >= 0) flush(cur_m);
            cur_m = d.m;
            const int64_t kk = (int64_t)d.m * Kp + kc;
            wc = wc_all[kk];
            wp = wp_all[kk];
            act = active_all[kk] != 0;
            on = __ballot(act) != 0;
        }
        if (!on) continue;
        const int n = d.se - d.sb;
        for (int i = 0; i < n; i += U) {
            int32_t sc[U][NSLOT], bi[U], fl[U], gs[U];
#pragma unroll
            for (int q = 0; q < U; ++q) {
                const int j = min(i + q, n - 1);   // past the end: repeat the last state, not stored
                const int4 a0 = l_rec[wave][j][0], a1 = l_rec[wave][j][1];
                sc[q][0] = __builtin_amdgcn_readfirstlane(a0.x);
                sc[q][1] = __builtin_amdgcn_readfirstlane(a0.y);
                sc[q][2] = __builtin_amdgcn_readfirstlane(a0.z);
                sc[q][3] = __builtin_amdgcn_readfirstlane(a0.w);
                sc[q][4] = __builtin_amdgcn_readfirstlane(a1.x);
                bi[q] = __builtin_amdgcn_readfirstlane(a1.y);
                fl[q] = __builtin_amdgcn_readfirstlane(a1.z);
                gs[q] = __builtin_amdgcn_readfirstlane(a1.w);   // the record's state
            }
            // successor rows and the state's own row (usually slot 0 again:
            // an L1 hit), all loads unconditional so they retire in order
            T xv[U][NSLOT], xo[U];
#pragma unroll
            for (int q = 0; q < U; ++q) {
#pragma unroll
                for (int dd = 0; dd < NSLOT; ++dd) {
                    const T* row = x_in + (int64_t)sc[q][dd] * Kp;
                    xv[q][dd] = row[kc];
                }
                xo[q] = (x_in + (int64_t)gs[q] * Kp)[kc];
            }
#pragma unroll
            for (int q = 0; q < U; ++q) {
                if (i + q >= n) break;
                T B[BLK];
                {
                    using V4 = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
                    constexpr int PER = sizeof(V4) / sizeof(T);
                    const V4* src = reinterpret_cast<const V4*>(ablk + (int64_t)bi[q] * BLK);
#pragma unroll
                    for (int k = 0; k < 32 / PER; ++k) {
                        const V4 v = src[k];
                        if constexpr (PER == 4) {
                            B[4 * k] = v.x; B[4 * k + 1] = v.y; B[4 * k + 2] = v.z; B[4 * k + 3] = v.w;
                        } else {
                            B[2 * k] = v.x; B[2 * k + 1] = v.y;
                        }
                    }
                }
                const int accm = fl[q] & 31;
                const T old = xo[q];
                T best = -INFINITY;
#pragma unroll
                for (int a = 0; a < 5; ++a) {
                    T acc = wc * B[25 + a];
                    if (accm) {
                        T rp = 0;
#pragma unroll
                        for (int dd = 0; dd < NSLOT; ++dd)
                            if (nz<PAT>(a, dd) && ((accm >> dd) & 1)) rp += B[a * NSLOT + dd];
                        acc = fma(wp, rp, acc);
                    }
#pragma unroll
                    for (int dd = 0; dd < NSLOT; ++dd)
                        if (nz<PAT>(a, dd)) acc = fma(B[a * NSLOT + dd], xv[q][dd], acc);
                    best = fmax(best, acc);
                }
                if (act) {
                    // the new values are read only by the next sweep: stream them out
                    __builtin_nontemporal_store(best, (x_out + (int64_t)gs[q] * Kp) + kc);
                    res = fmax(res, fabs(best - old));
                    if (want_ymax) ym = fmax(ym, fabs(best));
                }
            }
        }
    }
    if (cur_m >= 0) flush(cur_m);
}

// Value iteration of (column, model) instances over the neighbourhood
// blocks, FP64, one thread per instance state (instance-major values, one
// column each), with the summation order of the batched block sweep.  Used to
// re-solve only the assigned pairs: each instance's weights, its own
// residual (max over its states, one atomic per tile).
template <uint32_t PAT>
__global__ void __launch_bounds__(256) inst_vi_kernel(InstArgs a, const int32_t* __restrict__ rec,
                                                      const double* __restrict__ ablk, const double* wc,
                                                      const double* wp, const uint8_t* active,
                                                      const double* __restrict__ x_in, double* __restrict__ x_out,
                                                      unsigned long long* res, int32_t zero_row) {
    const int t = blockIdx.x;
    if (t >= a.n_tiles) return;
    const int inst = a.inst_tiles[2 * t];
    double r = 0.0;
    if (active[inst]) {
        const int ls = a.inst_tiles[2 * t + 1] + threadIdx.x;
        const int m = a.inst_model[inst];
        const int sb = a.state_base[m];
        if (ls < a.state_base[m + 1] - sb) {
            const int64_t ib = a.inst_base[inst];
            // the record at position sb + ls names its state
            const int4 r0 = *reinterpret_cast<const int4*>(rec + (int64_t)(sb + ls) * 8);
            const int4 r1 = *reinterpret_cast<const int4*>(rec + (int64_t)(sb + ls) * 8 + 4);
            const int own = r1.w - sb;
            const int sc[NSLOT] = {r0.x, r0.y, r0.z, r0.w, r1.x};
            double xv[NSLOT];
#pragma unroll
            for (int d = 0; d < NSLOT; ++d) xv[d] = sc[d] == zero_row ? 0.0 : x_in[ib + (sc[d] - sb)];
            const double* B = ablk + (int64_t)r1.y * BLK;
            const int accm = r1.z & 31;
            const double w0 = wc[inst], w1 = wp[inst];
            double best = -INFINITY;
#pragma unroll
            for (int act = 0; act < 5; ++act) {
                double rp = 0;
                if (accm) {
#pragma unroll
                    for (int d = 0; d < NSLOT; ++d)
                        if (nz<PAT>(act, d) && ((accm >> d) & 1)) rp += B[act * NSLOT + d];
                }
                double acc = w0 * B[25 + act];
                if (accm) acc = fma(w1, rp, acc);
#pragma unroll
                for (int d = 0; d < NSLOT; ++d)
                    if (nz<PAT>(act, d)) acc = fma(B[act * NSLOT + d], xv[d], acc);
                best = fmax(best, acc);
            }
            const double old = x_in[ib + own];
            x_out[ib + own] = best;
            r = fabs(best - old);
        }
    }
    r = wave_max(r);
    __shared__ double l_r[4];
    if ((threadIdx.x & 63) == 0) l_r[threadIdx.x >> 6] = r;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double m4 = fmax(fmax(l_r[0], l_r[1]), fmax(l_r[2], l_r[3]));
        if (m4 > 0.0) atomicMax(&res[inst], (unsigned long long)__double_as_longlong(m4));
    }
}

void inst_vi_sweep(hipStream_t s, const InstArgs& a, const int32_t* rec, const double* ablk, const double* wc,
                   const double* wp, const uint8_t* active, const double* x_in, double* x_out,
                   unsigned long long* res, int32_t zero_row, uint32_t pattern) {
    if (a.n_tiles <= 0) return;
    if (pattern_for(pattern) == PAT_GRID)
        hipLaunchKernelGGL(inst_vi_kernel<PAT_GRID>, dim3(a.n_tiles), dim3(256), 0, s, a, rec, ablk, wc, wp, active,
                           x_in, x_out, res, zero_row);
    else
        hipLaunchKernelGGL(inst_vi_kernel<PAT_DENSE>, dim3(a.n_tiles), dim3(256), 0, s, a, rec, ablk, wc, wp,
                           active, x_in, x_out, res, zero_row);
    MORAP_HIP(hipGetLastError());
}

// Alg. 4 over the neighbourhood blocks: one fixed-policy Jacobi sweep of both
// objectives (cost, probability) of (column, model) instances, FP64, one
// thread per instance state; x is [instance state][2], the policy mu the
// chosen row among the state's enabled actions.
template <uint32_t PAT>
__global__ void __launch_bounds__(256) eval_block_kernel(InstArgs a, const int32_t* __restrict__ rec,
                                                         const double* __restrict__ ablk, const int8_t* mu,
                                                         const uint8_t* active, const double* __restrict__ x_in,
                                                         double* __restrict__ x_out, unsigned long long* res,
                                                         int32_t zero_row) {
    // each wave walks a contiguous run of quarter tiles (64 states of one
    // instance) in a grid of resident size: one short-lived workgroup per
    // tile would leave most of each CU idle behind the workgroup dispatcher.
    // Residuals are kept per instance and flushed when the instance changes.
    const int n_units = a.n_tiles * 4;
    const int n_waves = gridDim.x * 4;
    const int per = (n_units + n_waves - 1) / n_waves;
    const int u0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * per;
    const int u1 = min(n_units, u0 + per);
    // the instance's descriptor (model, state range, value base, active
    // entries) is loaded when the instance changes, not per unit: consecutive
    // units mostly share it, and its loads form a dependent chain
    int cur = -1, sb = 0, n_st = 0;
    int64_t ib = 0;
    bool a0 = false, a1 = false;
    double m0 = 0.0, m1 = 0.0;
    for (int u = u0; u < u1; ++u) {
        const int t = u >> 2;
        const int inst = a.inst_tiles[2 * t];
        if (inst != cur) {
            if (cur >= 0 && (threadIdx.x & 63) == 0) {
                max_flush(&res[2 * cur], m0);
                max_flush(&res[2 * cur + 1], m1);
            }
            cur = inst;
            m0 = m1 = 0.0;
            const int m = a.inst_model[inst];
            sb = a.state_base[m];
            n_st = a.state_base[m + 1] - sb;
            ib = a.inst_base[inst];
            a0 = active[2 * inst] != 0;
            a1 = active[2 * inst + 1] != 0;
        }
        double r0 = 0.0, r1 = 0.0;
        if (a0 || a1) {
            const int ls = a.inst_tiles[2 * t + 1] + (u & 3) * 64 + (threadIdx.x & 63);
            if (ls < n_st) {
                const int4 q0 = *reinterpret_cast<const int4*>(rec + (int64_t)(sb + ls) * 8);
                const int4 q1 = *reinterpret_cast<const int4*>(rec + (int64_t)(sb + ls) * 8 + 4);
                const int own = q1.w - sb;
                // the chosen row is the mu-th enabled action
                uint32_t am = (uint32_t)(q1.z >> 8) & 31u;
                for (int k = mu[ib + own]; k > 0; --k) am &= am - 1;
                const int act = __builtin_ctz(am);
                const double* B = ablk + (int64_t)q1.y * BLK;
                const int accm = q1.z & 31;
                const int sc[NSLOT] = {q0.x, q0.y, q0.z, q0.w, q1.x};
                double c0 = B[25 + act], c1 = 0.0;
#pragma unroll
                for (int d = 0; d < NSLOT; ++d)
                    if (nz<PAT>(0, d) || nz<PAT>(1, d) || nz<PAT>(2, d) || nz<PAT>(3, d) || nz<PAT>(4, d))
                        if ((accm >> d) & 1) c1 += B[act * NSLOT + d];
#pragma unroll
                for (int d = 0; d < NSLOT; ++d) {
                    const double p = B[act * NSLOT + d];
                    if (sc[d] != zero_row) {
                        const double2 v = reinterpret_cast<const double2*>(x_in)[ib + (sc[d] - sb)];
                        c0 = fma(p, v.x, c0);
                        c1 = fma(p, v.y, c1);
                    }
                }
                const double2 old = reinterpret_cast<const double2*>(x_in)[ib + own];
                if (a0) { x_out[2 * (ib + own)] = c0; r0 = fabs(c0 - old.x); }
                if (a1) { x_out[2 * (ib + own) + 1] = c1; r1 = fabs(c1 - old.y); }
            }
        }
        m0 = fmax(m0, wave_max(r0));
        m1 = fmax(m1, wave_max(r1));
    }
    if (cur >= 0 && (threadIdx.x & 63) == 0) {
        max_flush(&res[2 * cur], m0);
        max_flush(&res[2 * cur + 1], m1);
    }
}

// Workgroups of 256 threads that stay resident per CU (occupancy API, once
// per kernel): the striding evaluation kernel is launched with exactly as
// many as fit, so no workgroup waits for a second round.
template <class F>
static int resident_per_cu(F* kern) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, 256, 0) != hipSuccess) n = 1;
    return std::max(1, n);
}
template <uint32_t PAT>
static int eval_groups(const InstArgs& a) {
    static const int per_cu = resident_per_cu(eval_block_kernel<PAT>);
    return std::min(a.n_tiles, std::max(1, a.cus) * per_cu);
}

void eval_block_sweep(hipStream_t s, const InstArgs& a, const int32_t* rec, const double* ablk, const int8_t* mu,
                      const uint8_t* active, const double* x_in, double* x_out, unsigned long long* res,
                      int32_t zero_row, uint32_t pattern) {
    if (a.n_tiles <= 0) return;
    if (pattern_for(pattern) == PAT_GRID)
        hipLaunchKernelGGL(eval_block_kernel<PAT_GRID>, dim3(eval_groups<PAT_GRID>(a)), dim3(256), 0, s, a, rec,
                           ablk, mu, active, x_in, x_out, res, zero_row);
    else
        hipLaunchKernelGGL(eval_block_kernel<PAT_DENSE>, dim3(eval_groups<PAT_DENSE>(a)), dim3(256), 0, s, a, rec,
                           ablk, mu, active, x_in, x_out, res, zero_row);
    MORAP_HIP(hipGetLastError());
}

template <class T, int U, uint32_t PAT>
static void launch_block_wave_p(hipStream_t s, int grid, int ktiles, const SweepArgs& a) {
    constexpr int WG = 256;
    hipLaunchKernelGGL((bellman_block_wave<T, U, WG, PAT>), dim3(grid, ktiles), dim3(WG), 0, s, a.tiles,
                       a.act_tiles, a.counters, a.rec, (const T*)a.ablk,
                       (const T*)a.wc, (const T*)a.wp, a.active, (const T*)a.x_in, (T*)a.x_out, a.res, a.ymax,
                       a.Kp, a.zero_row);
}

template <class T, int U>
static void launch_block_wave(hipStream_t s, int grid, int ktiles, const SweepArgs& a) {
    if (pattern_for(a.pattern) == PAT_GRID) launch_block_wave_p<T, U, PAT_GRID>(s, grid, ktiles, a);
    else launch_block_wave_p<T, U, PAT_DENSE>(s, grid, ktiles, a);
}

template <class T, int CPL, int LPS, int U, uint32_t PAT>
static void launch_block_p(hipStream_t s, int grid, int ktiles, const SweepArgs& a) {
    constexpr int WG = 256;
    hipLaunchKernelGGL((bellman_block<T, CPL, LPS, U, WG, PAT>), dim3(grid, ktiles), dim3(WG), 0, s, a.tiles,
                       a.act_tiles, a.counters, a.rec, (const T*)a.ablk,
                       (const T*)a.wc, (const T*)a.wp, a.active, (const T*)a.x_in, (T*)a.x_out, a.res, a.ymax,
                       a.Kp, a.zero_row);
}

template <class T, int CPL, int LPS, int U>
static void launch_block(hipStream_t s, int grid, int ktiles, const SweepArgs& a) {
    if (pattern_for(a.pattern) == PAT_GRID) launch_block_p<T, CPL, LPS, U, PAT_GRID>(s, grid, ktiles, a);
    else launch_block_p<T, CPL, LPS, U, PAT_DENSE>(s, grid, ktiles, a);
}

template <class T>
static void block_t(hipStream_t s, const Variant& v, int grid, int ktiles, const SweepArgs& a) {
#define MORAP_B(C, L) \
    if (v.cpl == C && v.lps == L) { launch_block<T, C, L, 2>(s, grid, ktiles, a); return; }
    MORAP_B(1, 1) MORAP_B(1, 2) MORAP_B(2, 1) MORAP_B(1, 4) MORAP_B(2, 2) MORAP_B(4, 1)
    MORAP_B(1, 8) MORAP_B(2, 4) MORAP_B(4, 2) MORAP_B(1, 16) MORAP_B(2, 8) MORAP_B(4, 4)
    MORAP_B(1, 32) MORAP_B(2, 16) MORAP_B(4, 8) MORAP_B(2, 32) MORAP_B(4, 16)
    if (v.cpl == 1 && v.lps == 64) {
        if (v.unroll == 2) launch_block_wave<T, 2>(s, grid, ktiles, a);
        else if (v.unroll == 8) launch_block_wave<T, 8>(s, grid, ktiles, a);
        else launch_block_wave<T, 4>(s, grid, ktiles, a);
        return;
    }
#undef MORAP_B
    fail(MORAP_E_UNSUPPORTED, "no block sweep kernel for this variant");
}

template <class T>
static const void* block_fn(const Variant& v) {
#define MORAP_F(C, L) \
    if (v.cpl == C && v.lps == L) return reinterpret_cast<const void*>(&bellman_block<T, C, L, 2, 256, PAT_GRID>);
    MORAP_F(1, 1) MORAP_F(1, 2) MORAP_F(2, 1) MORAP_F(1, 4) MORAP_F(2, 2) MORAP_F(4, 1)
    MORAP_F(1, 8) MORAP_F(2, 4) MORAP_F(4, 2) MORAP_F(1, 16) MORAP_F(2, 8) MORAP_F(4, 4)
    MORAP_F(1, 32) MORAP_F(2, 16) MORAP_F(4, 8) MORAP_F(2, 32) MORAP_F(4, 16)
#undef MORAP_F
    if (v.cpl == 1 && v.lps == 64) {
        if (v.unroll == 2) return reinterpret_cast<const void*>(&bellman_block_wave<T, 2, 256, PAT_GRID>);
        if (v.unroll == 8) return reinterpret_cast<const void*>(&bellman_block_wave<T, 8, 256, PAT_GRID>);
        return reinterpret_cast<const void*>(&bellman_block_wave<T, 4, 256, PAT_GRID>);
    }
    fail(MORAP_E_UNSUPPORTED, "no block sweep kernel for this variant");
}

int sweep_block_resident(int prec, const Variant& v) {
    int n = 0;
    MORAP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &n, prec == MORAP_F32 ? block_fn<float>(v) : block_fn<double>(v), 256, 0));
    return n;
}

void sweep_block(hipStream_t s, int prec, const Variant& v, int grid, int ktiles, const SweepArgs& a) {
    MORAP_CHECK(a.rec && a.ablk, MORAP_E_STATE, "the neighbourhood-block form was not built");
    if (prec == MORAP_F32) block_t<float>(s, v, grid, ktiles, a);
    else block_t<double>(s, v, grid, ktiles, a);
    MORAP_HIP(hipGetLastError());
}

}  // namespace k
}  // namespace morap
