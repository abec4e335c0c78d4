// Batched Bellman sweep with the successor values staged in LDS (Alg. 3, one
// Jacobi sweep of scalarised max-backups of every active (model, column)
// pair), for FP32 values and k-tiles of 64 columns.
//
// The states of a product are cut into halo tiles on the host: an agent's
// states are grown into connected regions of at most HALO_TILE states over
// its transition graph, the states of one product location in one region
// form a group, and groups are packed into tiles of at most HALO_TILE states
// whose value rows -- the tile's own states and all their successors --
// number at most HALO_MAX (the halo).  A tile's halo list holds the global
// state of every row, its own states first in record order; its 8-byte
// records name each successor slot by its place in the halo list (HALO_MAX =
// the zero row: slot unused or successor done).
//
// A workgroup of four waves takes one tile at a time: every wave copies a
// quarter of the tile's halo rows straight from HBM into LDS (direct
// global-to-LDS loads, 1 KB per instruction), the workgroup meets at a
// barrier, and each wave then backs up a quarter of the tile's states from
// LDS, lane = column, with the agent block in scalar registers and one
// streaming 256-byte store per state.  Every value row is read from HBM once
// per tile that needs it (1.3 rows per state on the 50 x 100 grids with
// 64-state tiles, against about two for the gather sweep), and the tiles of
// one XCD are walked in order so that rows shared by neighbouring tiles meet
// in its L2.  The next tile's row list, records and own states are fetched
// while the current one is backed up.  Small tiles keep several workgroups
// resident per compute unit (24.8 KB of LDS each), which hides the copy of one
// tile behind the backups of the others.
#include "common.h"
#include "kern.h"

#include <cfloat>

namespace morap {
namespace k {

namespace {

constexpr int NSLOT = 5;
constexpr int BLK = 32;
constexpr int WAVES = 4;
constexpr int ROUNDS = (HALO_MAX + 4 * WAVES - 1) / (4 * WAVES);   // 16 rows per round
// a load writes four rows from a multiple of 4 below the tile's row count:
// with HALO_MAX a multiple of 4 it never reaches the zero row
static_assert(HALO_MAX % 4 == 0, "HALO_MAX must be a multiple of 4");

typedef __attribute__((address_space(3))) void* lds_ptr_t;
typedef __attribute__((address_space(1))) const void* gbl_ptr_t;

constexpr uint32_t PAT_DENSE_H = (1u << 25) - 1;
constexpr uint32_t PAT_GRID_H = (1u << 0) | (1u << 1) | (1u << 3) | (1u << 4) |
                                (1u << 5) | (1u << 7) | (1u << 8) | (1u << 9) |
                                (1u << 10) | (1u << 11) | (1u << 12) | (1u << 13) |
                                (1u << 15) | (1u << 16) | (1u << 17) | (1u << 19) |
                                (1u << 20);
template <uint32_t PAT>
__device__ __forceinline__ constexpr bool nzh(int a, int d) { return (PAT >> (a * NSLOT + d)) & 1u; }

}  // namespace

template <int U, uint32_t PAT>
__global__ void __launch_bounds__(64 * WAVES)
bellman_halo(const HTile* __restrict__ tiles, const int32_t* __restrict__ act_tiles,
             const int64_t* __restrict__ counters, const uint2* __restrict__ hrec,
             const int32_t* __restrict__ hlist, const float* __restrict__ ablk,
             const float* __restrict__ wc_all, const float* __restrict__ wp_all,
             const uint8_t* __restrict__ active_all, const float* __restrict__ x_in, float* __restrict__ x_out,
             unsigned long long* __restrict__ res_all, unsigned long long* __restrict__ ymax_all, int Kp) {
    // halo rows of the current tile, 64 columns each; row HALO_MAX is the zero row
    __shared__ float lv[(HALO_MAX + 1) * 64];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int kt = blockIdx.y;
    const unsigned kc = (unsigned)kt * 64u + (unsigned)lane;

    const int n_tiles = (int)counters[1];
    // XCD x (workgroups are dealt round-robin to the 8 XCDs) takes the x-th
    // eighth of the active tiles in order; its workgroups take every n-th
    const int xcd = blockIdx.x & 7;
    const int step = gridDim.x >> 3;
    const int xb = (int)((int64_t)n_tiles * xcd / 8);
    const int xe = (int)((int64_t)n_tiles * (xcd + 1) / 8);
    int t = xb + (int)(blockIdx.x >> 3);
    if (t >= xe) return;   // the whole workgroup leaves together

    if (wave == 0) lv[HALO_MAX * 64 + lane] = 0.f;

    int cur_m = -1;
    bool act = false;
    float wc = 0.f, wp = 0.f;
    // the change |y - x| in FP32: exact whenever y and x are within a factor
    // of two of each other (Sterbenz), as near the stop test
    float res = 0.f, ym = 0.f;
    auto flush = [&](int m) {
        const int64_t idx = (int64_t)m * Kp + kc;
        max_flush(&res_all[idx], (double)res);
        max_flush(&ymax_all[idx], (double)ym);
        res = 0.f;
        ym = 0.f;
    };

    // a tile's descriptor and, per wave, the global states of its rows
    // (16 per round, four per load instruction: lane / 16), its records and
    // its own states; the next tile's are fetched while this one is backed up
    auto fetch = [&](const HTile& dd, int (&g)[ROUNDS], uint2& rec, int& gsv) {
        const int nn = dd.n & 0xffff, HH = dd.n >> 16;
        const int32_t* hl = hlist + dd.halo_begin;
        // lanes past the last row repeat it (into LDS rows below HALO_MAX
        // that no record names)
#pragma unroll
        for (int r = 0; r < ROUNDS; ++r) g[r] = hl[min(16 * r + 4 * wave + (lane >> 4), HH - 1)];
        const int p = min(wave * nn / WAVES + (lane & 31), nn - 1);
        rec = hrec[dd.rec_begin + p];
        gsv = hl[p];
    };
    // tile descriptors are wave-uniform: keep them in scalar registers
    auto uniform = [](const HTile& h) {
        return HTile{__builtin_amdgcn_readfirstlane(h.model), __builtin_amdgcn_readfirstlane(h.rec_begin),
                     __builtin_amdgcn_readfirstlane(h.n), __builtin_amdgcn_readfirstlane(h.halo_begin)};
    };
    HTile d = uniform(tiles[act_tiles[t]]);
    int g[ROUNDS];
    uint2 rec;
    int gsv;
    fetch(d, g, rec, gsv);
    while (true) {
        const int tn = t + step;
        const HTile dn = uniform(tiles[act_tiles[tn < xe ? tn : t]]);
        const int n = d.n & 0xffff, H = d.n >> 16;
        // this wave's rows straight into LDS
#pragma unroll
        for (int r = 0; r < ROUNDS; ++r) {
            const int row0 = 16 * r + 4 * wave;
            if (row0 >= H) break;   // uniform
            const float* src = x_in + (int64_t)g[r] * Kp + kt * 64 + (lane & 15) * 4;
            __builtin_amdgcn_global_load_lds((gbl_ptr_t)src, (lds_ptr_t)(lv + row0 * 64), 16, 0, 0);
        }
        if (d.model != cur_m) {
            if (cur_m >= 0) flush(cur_m);
            cur_m = d.model;
            const int64_t kk = (int64_t)d.model * Kp + kc;
            wc = wc_all[kk];
            wp = wp_all[kk];
            act = active_all[kk] != 0;
        }
        __syncthreads();   // every wave's rows are in LDS
        const uint2 rec_c = rec;
        const int gsv_c = gsv;
        if (tn < xe) fetch(dn, g, rec, gsv);

        // this wave's states: a quarter of the tile (at most 32)
        const int i0 = wave * n / WAVES;
        const int n_w = (wave + 1) * n / WAVES - i0;
        for (int i = 0; i < n_w; i += U) {
            uint32_t w0[U], w1[U];
            int gs[U];
#pragma unroll
            for (int q = 0; q < U; ++q) {
                const int j = min(i + q, n_w - 1);   // past the end: repeat the last state, not stored
                w0[q] = __builtin_amdgcn_readlane(rec_c.x, j);
                w1[q] = __builtin_amdgcn_readlane(rec_c.y, j);
                gs[q] = __builtin_amdgcn_readlane(gsv_c, j);
            }
            float xv[U][NSLOT], xo[U];
#pragma unroll
            for (int q = 0; q < U; ++q) {
#pragma unroll
                for (int s = 0; s < 4; ++s) xv[q][s] = lv[((w0[q] >> (8 * s)) & 255u) * 64 + lane];
                xv[q][4] = lv[(w1[q] & 255u) * 64 + lane];
                const int own = i0 + min(i + q, n_w - 1);
                xo[q] = lv[own * 64 + lane];
            }
#pragma unroll
            for (int q = 0; q < U; ++q) {
                if (i + q >= n_w) break;
                // the agent block (P[a][slot] then -cost[a]) in scalar registers
                float B[BLK];
                {
                    const float4* src = reinterpret_cast<const float4*>(ablk + (int64_t)(w1[q] >> 13) * BLK);
#pragma unroll
                    for (int k4 = 0; k4 < BLK / 4; ++k4) {
                        const float4 v = src[k4];
                        B[4 * k4] = v.x;
                        B[4 * k4 + 1] = v.y;
                        B[4 * k4 + 2] = v.z;
                        B[4 * k4 + 3] = v.w;
                    }
                }
                const int accm = (int)((w1[q] >> 8) & 31u);
                float best = -INFINITY;
                if (accm) {
                    // probability reward: the action's mass on accepting slots
#pragma unroll
                    for (int a = 0; a < 5; ++a) {
                        float rp = 0.f;
#pragma unroll
                        for (int s = 0; s < NSLOT; ++s)
                            if (nzh<PAT>(a, s) && ((accm >> s) & 1)) rp += B[a * NSLOT + s];
                        float acc = fmaf(wp, rp, wc * B[25 + a]);
#pragma unroll
                        for (int s = 0; s < NSLOT; ++s)
                            if (nzh<PAT>(a, s)) acc = fmaf(B[a * NSLOT + s], xv[q][s], acc);
                        best = fmaxf(best, acc);
                    }
                } else {
#pragma unroll
                    for (int a = 0; a < 5; ++a) {
                        float acc = wc * B[25 + a];
#pragma unroll
                        for (int s = 0; s < NSLOT; ++s)
                            if (nzh<PAT>(a, s)) acc = fmaf(B[a * NSLOT + s], xv[q][s], acc);
                        best = fmaxf(best, acc);
                    }
                }
                if (act) {
                    __builtin_nontemporal_store(best, (x_out + (int64_t)gs[q] * Kp) + kc);
                    res = fmaxf(res, fabsf(best - xo[q]));
                    ym = fmaxf(ym, fabsf(best));
                }
            }
        }
        __syncthreads();   // the rows may be overwritten by the next tile
        if (tn >= xe) break;
        t = tn;
        d = dn;
    }
    if (cur_m >= 0) flush(cur_m);
}

static uint32_t halo_pattern(uint32_t union_pattern) {
    return (union_pattern & ~PAT_GRID_H) == 0 ? PAT_GRID_H : PAT_DENSE_H;
}

template <int U>
static const void* halo_fn(uint32_t pattern) {
    if (halo_pattern(pattern) == PAT_GRID_H) return reinterpret_cast<const void*>(&bellman_halo<U, PAT_GRID_H>);
    return reinterpret_cast<const void*>(&bellman_halo<U, PAT_DENSE_H>);
}

int sweep_halo_resident(const Variant& v, uint32_t pattern) {
    int n = 0;
    const void* f = v.unroll == 4 ? halo_fn<4>(pattern) : halo_fn<2>(pattern);
    MORAP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, 64 * WAVES, 0));
    return n;
}

template <int U, uint32_t PAT>
static void launch_halo_p(hipStream_t s, int grid, int ktiles, const SweepArgs& a) {
    hipLaunchKernelGGL((bellman_halo<U, PAT>), dim3(grid, ktiles), dim3(64 * WAVES), 0, s, a.htiles, a.act_tiles,
                       a.counters, a.hrec, a.hlist, (const float*)a.ablk, (const float*)a.wc, (const float*)a.wp,
                       a.active, (const float*)a.x_in, (float*)a.x_out, a.res, a.ymax, a.Kp);
}

void sweep_halo(hipStream_t s, int prec, const Variant& v, int grid, int ktiles, const SweepArgs& a) {
    MORAP_CHECK(prec == MORAP_F32, MORAP_E_UNSUPPORTED, "the LDS-staged sweep runs FP32 values only");
    MORAP_CHECK(a.htiles && a.hrec && a.hlist && a.ablk, MORAP_E_STATE, "the halo tiles were not built");
    MORAP_CHECK(a.Kp % 64 == 0, MORAP_E_UNSUPPORTED, "the LDS-staged sweep needs k-tiles of 64 columns");
    const bool grid_pat = halo_pattern(a.pattern) == PAT_GRID_H;
    if (v.unroll == 4) {
        if (grid_pat) launch_halo_p<4, PAT_GRID_H>(s, grid, ktiles, a);
        else launch_halo_p<4, PAT_DENSE_H>(s, grid, ktiles, a);
    } else {
        if (grid_pat) launch_halo_p<2, PAT_GRID_H>(s, grid, ktiles, a);
        else launch_halo_p<2, PAT_DENSE_H>(s, grid, ktiles, a);
    }
    MORAP_HIP(hipGetLastError());
}

}  // namespace k
}  // namespace morap
