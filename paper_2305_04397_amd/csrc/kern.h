// Device helpers shared by the sweep kernels (vi.hip, block.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace morap {
namespace k {

// ---------------------------------------------------------------------------
// vector helpers: CPL consecutive columns per lane
// ---------------------------------------------------------------------------
template <class T, int CPL> struct Vec { T v[CPL]; };

template <class T, int CPL>
__device__ __forceinline__ Vec<T, CPL> vload(const T* p) {
    Vec<T, CPL> r;
    if constexpr (CPL == 4 && sizeof(T) == 4) {
        float4 q = *reinterpret_cast<const float4*>(p);
        r.v[0] = q.x; r.v[1] = q.y; r.v[2] = q.z; r.v[3] = q.w;
    } else if constexpr (CPL == 2 && sizeof(T) == 4) {
        float2 q = *reinterpret_cast<const float2*>(p);
        r.v[0] = q.x; r.v[1] = q.y;
    } else if constexpr (CPL >= 2 && sizeof(T) == 8) {
#pragma unroll
        for (int c = 0; c < CPL; c += 2) {
            double2 q = *reinterpret_cast<const double2*>(p + c);
            r.v[c] = q.x; r.v[c + 1] = q.y;
        }
    } else {
#pragma unroll
        for (int c = 0; c < CPL; ++c) r.v[c] = p[c];
    }
    return r;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// reduce across lanes that hold the same columns: lane bits >= log2(LPS)
template <int LPS>
__device__ __forceinline__ double group_max(double v) {
#pragma unroll
    for (int o = 32; o >= LPS; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Raise the FP64 maximum stored (as its bit pattern) at p to v >= 0.  The
// current value is read first and the atomic skipped when it is already at
// least v: many workers flush maxima of the same (model, column) pairs, and
// most of them do not raise it, so this keeps atomics on a hot address few.
__device__ __forceinline__ void max_flush(unsigned long long* p, double v) {
    if (!(v > 0.0)) return;
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    // non-negative doubles order like their bit patterns
    if (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= b) return;
    atomicMax(p, b);
}

// Share [b, e) of n ordered work items for worker idx of count workers on XCD
// xcd.  Workgroups are dealt to the 8 XCDs round-robin by blockIdx.x, so each
// XCD takes one contiguous eighth of the items (neighbouring items share its
// L2) and splits it evenly over its own workers.
__device__ __forceinline__ void xcd_share(int n, int xcd, int idx, int count, int& b, int& e) {
    const int xb = (int)((int64_t)n * xcd / 8), xe = (int)((int64_t)n * (xcd + 1) / 8);
    const int m = xe - xb;
    b = xb + (int)((int64_t)m * idx / count);
    e = xb + (int)((int64_t)m * (idx + 1) / count);
}

}  // namespace k
}  // namespace morap
