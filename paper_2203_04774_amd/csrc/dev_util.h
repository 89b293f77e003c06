// Device-side helpers for 64-lane CDNA wavefronts.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define WAVE 64

__device__ __forceinline__ int lane_id() { return threadIdx.x & (WAVE - 1); }

// For values that are equal in every active lane: moved to scalar registers,
// so that the loops and branches they steer compile as wave-uniform (scalar
// branches, scalar loads) instead of per-lane masks.
__device__ __forceinline__ uint32_t uni32(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }
__device__ __forceinline__ uint64_t uni64(uint64_t v) {
    return ((uint64_t)uni32((uint32_t)(v >> 32)) << 32) | uni32((uint32_t)v);
}
// this lane's wavefront within its workgroup
// lane 0's value, as a wave-uniform (scalar) value
__device__ __forceinline__ uint64_t lane0_u64(uint64_t v) {
    return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 0) << 32) |
           (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 0);
}
// lane src's value (src wave-uniform), as a wave-uniform value
__device__ __forceinline__ uint64_t lane_u64(uint64_t v, int src) {
    return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), src) << 32) |
           (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, src);
}
__device__ __forceinline__ uint32_t wave_id() { return uni32(threadIdx.x / WAVE); }

// Orders a wavefront's own LDS accesses in the compiler (the hardware
// already runs one wavefront's LDS operations in issue order).
__device__ __forceinline__ void wave_lds_fence() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    int l = lane_id();
    return l ? (~0ull >> (64 - l)) : 0ull;
}

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src) {
    uint32_t lo = __shfl((uint32_t)v, src, WAVE);
    uint32_t hi = __shfl((uint32_t)(v >> 32), src, WAVE);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t shfl_up_u64(uint64_t v, int d) {
    uint32_t lo = __shfl_up((uint32_t)v, d, WAVE);
    uint32_t hi = __shfl_up((uint32_t)(v >> 32), d, WAVE);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
    uint32_t lo = __shfl_xor((uint32_t)v, m, WAVE);
    uint32_t hi = __shfl_xor((uint32_t)(v >> 32), m, WAVE);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v += shfl_xor_u64(v, m);
    return v;
}

__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t v) {
    int l = lane_id();
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        uint64_t t = shfl_up_u64(v, d);
        if (l >= d) v += t;
    }
    return v;
}

// Block-wide exclusive scan of one u64 per thread.  `lds` must hold
// BLOCK/64 entries.  Returns the exclusive prefix; `total` gets the block sum.
template <int BLOCK>
__device__ __forceinline__ uint64_t block_excl_scan_u64(uint64_t v, uint64_t *lds, uint64_t &total) {
    const int l = lane_id(), w = threadIdx.x / WAVE;
    uint64_t inc = wave_incl_scan_u64(v);
    if (l == WAVE - 1) lds[w] = inc;
    __syncthreads();
    uint64_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < BLOCK / WAVE; i++) {
        uint64_t s = lds[i];
        off += (i < w) ? s : 0;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return off + inc - v;
}

template <int BLOCK>
__device__ __forceinline__ uint64_t block_sum_u64(uint64_t v, uint64_t *lds) {
    const int l = lane_id(), w = threadIdx.x / WAVE;
    v = wave_sum_u64(v);
    if (l == 0) lds[w] = v;
    __syncthreads();
    uint64_t tot = 0;
#pragma unroll
    for (int i = 0; i < BLOCK / WAVE; i++) tot += lds[i];
    __syncthreads();
    return tot;
}

// first index i in [lo, hi) with a[i] >= x (hi if none)
template <class T>
__device__ __forceinline__ uint64_t lower_bound_dev(const T *a, uint64_t lo, uint64_t hi, T x) {
    while (lo < hi) {
        uint64_t mid = lo + ((hi - lo) >> 1);
        if (a[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// first index i in [lo, hi) with a[i] > x (hi if none)
template <class T>
__device__ __forceinline__ uint64_t upper_bound_dev(const T *a, uint64_t lo, uint64_t hi, T x) {
    while (lo < hi) {
        uint64_t mid = lo + ((hi - lo) >> 1);
        if (a[mid] <= x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// The same searches, probing first the few entries next to one end of the
// range (they share its cache lines) before halving the rest.  A window
// bound that lies near that end then costs one or two lines instead of a
// line per halving step; elsewhere it costs the plain search plus those
// probes.  Results are those of lower_bound_dev / upper_bound_dev.
template <class T>
__device__ __forceinline__ uint64_t lower_bound_front(const T *a, uint64_t lo, uint64_t hi, T x) {
    uint64_t step = 1, prev = lo;
    while (step <= 8 && lo + step - 1 < hi) {  // a[lo], a[lo+1], a[lo+3], a[lo+7]
        if (!(a[lo + step - 1] < x)) return lower_bound_dev<T>(a, prev, lo + step - 1, x);
        prev = lo + step;
        step <<= 1;
    }
    return lower_bound_dev<T>(a, prev, hi, x);
}
template <class T>
__device__ __forceinline__ uint64_t upper_bound_back(const T *a, uint64_t lo, uint64_t hi, T x) {
    uint64_t step = 1, prev = hi;
    while (step <= 8 && hi >= lo + step) {  // a[hi-1], a[hi-2], a[hi-4], a[hi-8]
        if (a[hi - step] <= x) return upper_bound_dev<T>(a, hi - step + 1, prev, x);
        prev = hi - step;
        step <<= 1;
    }
    return upper_bound_dev<T>(a, lo, prev, x);
}

// splitmix64 output function (Steele, Lea, Flood, OOPSLA 2014)
__device__ __forceinline__ uint64_t sm64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// digest of a triangle given as three original ids in any order
__device__ __forceinline__ void canon3(uint32_t &a, uint32_t &b, uint32_t &c) {
    uint32_t t;
    if (a > b) { t = a; a = b; b = t; }
    if (b > c) { t = b; b = c; c = t; }
    if (a > b) { t = a; a = b; b = t; }
}

__device__ __forceinline__ uint64_t tri_digest(uint32_t a, uint32_t b, uint32_t c) {
    return sm64_mix(sm64_mix(((uint64_t)a << 32) | b) + c);
}

// XCD-aware split of [0, n) for a grid whose size is a multiple of 8:
// workgroups are dispatched to the 8 XCDs in turn (workgroup b on XCD
// b % 8), so each XCD takes one contiguous eighth of the range and its
// workgroups stride through that eighth together; what they touch at a
// time then stays in that XCD's own L2.  first/stride/end describe this
// thread's walk; `base` is where its wavefront starts (for wave-uniform
// trip counts).
struct XcdRange {
    uint64_t first, stride, end, base;
    __device__ __forceinline__ explicit XcdRange(uint64_t n) {
        const uint32_t nx = 8u, xcd = blockIdx.x % nx, per_xcd = gridDim.x / nx, lb = blockIdx.x / nx;
        const uint64_t chunk = (n + nx - 1) / nx;
        const uint64_t lo = (uint64_t)xcd * chunk;
        end = lo + chunk < n ? lo + chunk : n;
        if (lo > end) end = lo;
        stride = (uint64_t)per_xcd * blockDim.x;
        base = lo + (uint64_t)lb * blockDim.x + (threadIdx.x & ~(uint64_t)(WAVE - 1));
        first = base + (threadIdx.x & (WAVE - 1));
    }
    // iterations of this wavefront (the same for all its lanes)
    __device__ __forceinline__ uint64_t wave_iters() const {
        return end > base ? (end - base + stride - 1) / stride : 0;
    }
};

#define GRID_STRIDE(i, n)                                                                \
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (uint64_t)(n); \
         i += (uint64_t)gridDim.x * blockDim.x)
