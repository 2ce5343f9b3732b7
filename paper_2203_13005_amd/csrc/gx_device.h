// Device helpers shared by the gx kernels (block scans and reductions, the
// saturating add of the min-plus relaxation, a bounded grid barrier for
// cooperative persistent kernels).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "gx_internal.h"

namespace gx {

__device__ __forceinline__ uint32_t sat_add(uint32_t a, uint32_t b) {
    uint32_t s = a + b;
    return s < a ? INF : s;
}

// Exclusive prefix sum of a 64-bit value over a 256-thread block.
__device__ __forceinline__ unsigned long long block_excl_scan_u64(unsigned long long v, unsigned long long *total,
                                                                  unsigned long long *lds) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    unsigned long long x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        unsigned long long y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) lds[wid] = x;
    __syncthreads();
    unsigned long long pre = 0, tot = 0;
    for (int i = 0; i < nw; i++) {
        unsigned long long t = lds[i];
        if (i < wid) pre += t;
        tot += t;
    }
    *total = tot;
    __syncthreads();
    return pre + x - v;
}

// Sum over a block in a fixed tree (deterministic for floating point).
template <class T>
__device__ __forceinline__ T block_sum(T v, T *lds) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    T r = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < nw; i++) r += lds[i];
    __syncthreads();
    return r;  // valid in thread 0
}

// In-place inclusive max-scan of s[0..n) (n <= blockDim * VT), VT contiguous
// elements per thread.
template <int VT>
__device__ __forceinline__ void block_max_scan(int32_t *s, int n, int32_t *lds) {
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nw = blockDim.x >> 6;
    int32_t loc[VT];
    int32_t run = 0;
#pragma unroll
    for (int i = 0; i < VT; i++) {
        int p = tid * VT + i;
        int32_t v = p < n ? s[p] : 0;
        run = max(run, v);
        loc[i] = run;
    }
    int32_t x = run;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x = max(x, y);
    }
    if (lane == 63) lds[wid] = x;
    __syncthreads();
    int32_t pre = 0;
    for (int i = 0; i < wid; i++) pre = max(pre, lds[i]);
    (void)nw;
    int32_t excl = __shfl_up(x, 1, 64);
    if (lane == 0) excl = 0;
    excl = max(excl, pre);
#pragma unroll
    for (int i = 0; i < VT; i++) {
        int p = tid * VT + i;
        if (p < n) s[p] = max(loc[i], excl);
    }
    __syncthreads();
}


// The XCD (accelerator complex die) the calling wave runs on: bits 3:0 of
// the XCC_ID hardware register.
__device__ __forceinline__ uint32_t xcc_id() { return __builtin_amdgcn_s_getreg((3 << 11) | 20) & 15u; }

// Grid-wide barrier for a cooperative launch (all workgroups co-resident).
// Sense is a generation counter.  The wait is bounded in time: a workgroup
// that has waited `limit_ticks` of the constant-rate wall clock
// (wall_clock64) sets *error and leaves, and so does every workgroup that
// finds *error set, so a grid can never spin forever; the host reports the
// error.  Returns true when every workgroup arrived.
struct GridBar {
    unsigned int count;
    unsigned int gen;
    unsigned int error;
    unsigned int pad;
};

__device__ __forceinline__ bool grid_sync(GridBar *b, unsigned int nblocks, unsigned int *s_flag,
                                          unsigned long long limit_ticks) {
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned int g = __hip_atomic_load(&b->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        unsigned int arrived = atomicAdd(&b->count, 1u);
        if (arrived == nblocks - 1) {
            __hip_atomic_store(&b->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&b->gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            const unsigned long long t0 = (unsigned long long)wall_clock64();
            while (__hip_atomic_load(&b->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
                __builtin_amdgcn_s_sleep(2);
                if (__hip_atomic_load(&b->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) break;
                if ((unsigned long long)wall_clock64() - t0 > limit_ticks) {
                    atomicOr(&b->error, 1u);
                    break;
                }
            }
        }
        __threadfence();
        *s_flag = __hip_atomic_load(&b->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    return *s_flag == 0u;
}

}  // namespace gx
