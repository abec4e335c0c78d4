// Stage retirement inside the Jacobi iteration (the staged form of Alg. 3
// that keeps the plain sweep count).
//
// A product's location groups (strongly connected sets of DFA locations)
// form a DAG in which every transition leads to the same or a lower group;
// a state's stage is the height of its group there (0: no lower group).
// The states of each model are split into units, one per stage, lowest
// first, and the sweep kernels run over the units' tiles as over models.
// After every sweep, per (model, column), the units are taken lowest first:
// a unit retires when every lower unit has retired and its own largest
// change in this sweep is within the stop rule; its tiles then leave the
// active list.  A retired unit is no longer written, so its final values
// (in the buffer the sweep just wrote) are copied into the other Jacobi
// buffer before the next sweep writes that buffer's other states: the units
// above it keep reading the same values in every later sweep.
#include "common.h"
#include "kern.h"

namespace morap {
namespace k {

// One thread per (model, column) pair.  counters: as the convergence kernel
// ([0] active pairs, [4] backups, [7] state-columns updated), with the
// (unit, column) pairs retired in this sweep appended to a.retired and
// counted in counters[a.slot].
template <class T>
__global__ void __launch_bounds__(256) stage_converge_kernel(StageArgs a) {
    const int64_t n = (int64_t)a.M * a.Kp;
    const int32_t next_sweep = (int32_t)(a.counters[5] + 1);
    unsigned long long bk = 0, sc = 0, cnt = 0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const int m = (int)(t / a.Kp);
        const int k = (int)(t % a.Kp);
        if (k >= a.K) continue;
        bool lower_done = true;
        for (int u = a.unit_base[m]; u < a.unit_base[m + 1]; ++u) {
            const int64_t j = (int64_t)u * a.Kp + k;
            if (!a.active[j]) continue;   // retired earlier (or never live)
            const double r = __longlong_as_double((long long)a.res[j]);
            const double y = __longlong_as_double((long long)a.ymax[j]);
            a.res[j] = 0ull;
            a.ymax[j] = 0ull;
            bk += (unsigned long long)a.rows[u];
            sc += (unsigned long long)a.states[u];
            const double tol = fmax(a.eps, a.unit * y);
            // FP32: a unit whose change has set no new minimum for
            // stall_sweeps sweeps and is within the rounding floor has
            // settled as far as FP32 backups go (as a pair of the plain solve)
            bool floor_stop = false;
            if (a.stall_sweeps > 0 && r > tol) {
                if (r < a.best_res[j]) {
                    a.best_res[j] = r;
                    a.stall[j] = 0;
                } else if (++a.stall[j] >= a.stall_sweeps && r <= a.floor * y) {
                    floor_stop = true;
                }
            }
            if (lower_done && (r <= tol || floor_stop)) {
                if (floor_stop) atomicAdd((unsigned long long*)&a.counters[8], 1ull);
                a.active[j] = 0;
                const unsigned long long p = atomicAdd((unsigned long long*)&a.counters[a.slot], 1ull);
                a.retired[p] = j;
                if (u == a.init_unit[m]) {
                    // the initial state's value is final
                    const int64_t i = (int64_t)m * a.Kp + k;
                    a.c[(int64_t)k * a.M + m] = (double)((const T*)a.x_out)[(int64_t)a.init[m] * a.Kp + k];
                    a.final_par[i] = (uint8_t)a.out_par;
                    a.pair_sweeps[i] = next_sweep;
                }
            } else {
                lower_done = false;
                a.model_active[u] = 1;
                ++cnt;
            }
        }
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

// The final values of the (unit, column) pairs retired in this sweep, copied
// from the buffer the sweep wrote into the one it read: one workgroup per
// retired pair at a time, its threads over the unit's records (each names
// its state).  The list count of the next sweep starts at 0 here.
template <class T>
__global__ void __launch_bounds__(256) stage_copy_kernel(StageArgs a) {
    if (blockIdx.x == 0 && threadIdx.x == 0) a.counters[a.slot == 9 ? 10 : 9] = 0;
    const int64_t n = a.counters[a.slot];
    for (int64_t e = blockIdx.x; e < n; e += gridDim.x) {
        const int64_t j = a.retired[e];
        const int u = (int)(j / a.Kp);
        const int k = (int)(j % a.Kp);
        for (int tt = a.tile_base[u]; tt < a.tile_base[u + 1]; ++tt) {
            const Tile tl = a.tiles[tt];
            for (int p = tl.s_begin + (int)threadIdx.x; p < tl.s_end; p += blockDim.x) {
                const int64_t g = a.rec[(int64_t)p * 8 + 7];
                ((T*)a.x_in)[g * a.Kp + k] = ((const T*)a.x_out)[g * a.Kp + k];
            }
        }
    }
}

void stage_converge(hipStream_t s, const StageArgs& a) {
    const int64_t n = (int64_t)a.M * a.Kp;
    const unsigned blocks = (unsigned)std::min<int64_t>(256, std::max<int64_t>(1, (n + 255) / 256));
    if (a.prec == MORAP_F32) hipLaunchKernelGGL(stage_converge_kernel<float>, dim3(blocks), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(stage_converge_kernel<double>, dim3(blocks), dim3(256), 0, s, a);
    MORAP_HIP(hipGetLastError());
}

void stage_copy(hipStream_t s, const StageArgs& a) {
    if (a.prec == MORAP_F32) hipLaunchKernelGGL(stage_copy_kernel<float>, dim3(256), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(stage_copy_kernel<double>, dim3(256), dim3(256), 0, s, a);
    MORAP_HIP(hipGetLastError());
}

}  // namespace k
}  // namespace morap
