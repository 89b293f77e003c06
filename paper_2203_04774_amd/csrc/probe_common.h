// Device-side pieces shared by the listing and batched-listing kernels:
// the oriented graph view, the geometry of a seed edge for the three
// forms, and the walk over a flattened, prefix-summed work space.
#pragma once

#include "tl_internal.h"
#include "dev_util.h"

namespace {

struct GView {
    const u64 *off_f, *off_b;
    const u32 *adj_f, *adj_b, *row_f, *row_b, *inv;
    u64 m;
    const u32 *twin_b;  // twin_b[e]: where backward entry e's edge sits in adj_f
};

// Seed-edge geometry for the three forms.
template <int ALGO>
struct Seed {
    u32 p, x;          // pivot and the seed edge's other endpoint
    const u32 *S;      // scanned list base (S[s_lo .. s_hi))
    u64 s_lo, s_hi;
    const u32 *T;      // target array, candidates T[t_lo .. t_hi)
    u64 t_lo, t_hi;
    u32 twin;          // A++: index of p in S (S[twin] = p)
    __device__ __forceinline__ Seed(const GView &g, u64 e) {
        twin = 0;
        if (ALGO == 0) {
            p = g.row_b[e]; x = g.adj_b[e];
            S = g.adj_f; s_lo = g.off_f[x]; s_hi = g.off_f[x + 1];
            T = g.adj_b; t_lo = e + 1; t_hi = g.off_b[p + 1];
            twin = g.twin_b[e];
        } else if (ALGO == 1) {
            p = g.row_f[e]; x = g.adj_f[e];
            S = g.adj_f; s_lo = g.off_f[x]; s_hi = g.off_f[x + 1];
            T = g.adj_f; t_lo = e + 1; t_hi = g.off_f[p + 1];
        } else {
            p = g.row_f[e]; x = g.adj_f[e];
            S = g.adj_b; s_lo = g.off_b[x]; s_hi = g.off_b[x + 1];
            T = g.adj_b; t_lo = g.off_b[p]; t_hi = g.off_b[p + 1];
        }
    }
};

// Arrays that index seeds, scanned lists and pivot lists for a form.
template <int ALGO>
struct Form {
    // seed edges are the entries of this CSR (pivot-major)
    static __device__ __forceinline__ const u64 *seed_off(const GView &g) { return ALGO == 0 ? g.off_b : g.off_f; }
    static __device__ __forceinline__ const u32 *seed_adj(const GView &g) { return ALGO == 0 ? g.adj_b : g.adj_f; }
    // scanned lists
    static __device__ __forceinline__ const u32 *scan_adj(const GView &g) { return ALGO == 2 ? g.adj_b : g.adj_f; }
    // pivot (marked) list
    static __device__ __forceinline__ const u64 *piv_off(const GView &g) { return ALGO == 1 ? g.off_f : g.off_b; }
    static __device__ __forceinline__ const u32 *piv_adj(const GView &g) { return ALGO == 1 ? g.adj_f : g.adj_b; }
};


// Walks a run of the flattened work space 64 items at a time and gives each
// lane the compacted seed c with cpre[c] <= k < cpre[c+1] of its item k, and
// the item's offset inside that seed's window.  When the whole chunk lies in
// one seed (long windows) no search is needed; otherwise the chunk spans at
// most 64 seeds starting at the current one, found by a binary search over
// a 64-entry window of cpre held one entry per lane.
struct SeedCursor {
    const u64 *cpre;
    u64 ncap;         // cpre[0..ncap] is readable
    u64 c_lo;         // seed of the chunk's first item
    u64 base, end;    // cpre[c_lo], cpre[c_lo + 1]

    __device__ __forceinline__ SeedCursor() : cpre(nullptr), ncap(0), c_lo(0), base(0), end(0) {}
    // (all arguments wave-uniform; the cursor's fields stay wave-uniform)
    __device__ __forceinline__ SeedCursor(const u64 *cp, u64 lo, u64 nc, u64 first_item) : cpre(cp), ncap(nc) {
        c_lo = uni64(upper_bound_dev<u64>(cpre, lo, ncap + 1, first_item) - 1);
        base = uni64(cpre[c_lo]);
        end = uni64(cpre[c_lo + 1]);
    }
    // when the seed of the first item is already known
    __device__ __forceinline__ SeedCursor(const u64 *cp, u64 nc, u64 c) : cpre(cp), ncap(nc), c_lo(uni64(c)) {
        base = uni64(cpre[c_lo]);
        end = uni64(cpre[c_lo + 1]);
    }

    __device__ __forceinline__ u64 locate(u64 kb, u64 k, u64 &rel) const {
        if (end >= kb + WAVE) {  // wave-uniform
            rel = k - base;
            return c_lo;
        }
        const int lane = lane_id();
        const u64 P = (c_lo + lane <= ncap) ? cpre[c_lo + lane] : ~0ull;
        int lo = 0;
#pragma unroll
        for (int st = 32; st > 0; st >>= 1) {
            u64 pv = shfl_u64(P, lo + st);
            if (pv <= k) lo += st;
        }
        rel = k - shfl_u64(P, lo);
        return c_lo + lo;
    }

    // continue from seed c (known to hold the next item)
    __device__ __forceinline__ void reset(u64 c) {
        c_lo = uni64(c);
        base = uni64(cpre[c_lo]);
        end = uni64(cpre[c_lo + 1]);
    }

    // move to the seed of item nk, given c = seed of the last lane's item
    // (the last lane's item may lie past the final seed when the walk ends:
    // then c = ncap and the cursor parks there without reading past cpre[ncap])
    __device__ __forceinline__ void advance(u64 nk, u64 c) {
        if (nk < end) return;
        c_lo = uni64(shfl_u64(c, WAVE - 1));
        if (c_lo < ncap && uni64(cpre[c_lo + 1]) <= nk) c_lo++;
        base = uni64(cpre[c_lo]);
        end = c_lo < ncap ? uni64(cpre[c_lo + 1]) : base;
    }
};

constexpr int UN = 4;  // chunks per iteration when they share one seed window

// Seeds of the UN chunks of 64 items from kb on, when they all lie in the 64
// consecutive seeds whose work prefixes P the lanes hold (lane 0's seed
// holds item kb).  Every seed marks the item it starts at, relative to kb,
// in the wavefront's 256 bytes of LDS flags; for chunk j, a ballot of the
// flags and a count of the set ones up to a lane give lo[j], the lane
// (seed) that holds item kb + 64 j + lane.  Returns the seed of the last
// item.  Compacted seeds have non-empty windows, so starts are distinct.
__device__ __forceinline__ int locate_short(u64 P, u64 kb, unsigned char *flag, int (&lo)[UN]) {
    const int lane = lane_id();
    const u32 Q = P <= kb ? 0u : (P - kb > 0xffffffffull ? 0xffffffffu : (u32)(P - kb));
    reinterpret_cast<u32 *>(flag)[lane] = 0u;
    wave_lds_fence();
    if (Q < (u32)(UN * WAVE)) flag[Q] = 1;  // the first seed marks item 0
    wave_lds_fence();
    u32 started = 0;  // seeds started in the chunks before j
#pragma unroll
    for (int j = 0; j < UN; j++) {
        const u32 f = flag[j * WAVE + lane];
        const u64 S = __ballot(f != 0u);
        lo[j] = (int)(started + f + (u32)__popcll(S & lanemask_lt())) - 1;
        started += (u32)__popcll(S);
    }
    wave_lds_fence();
    return (int)started - 1;
}

// As locate_short, for a window whose lane s0 (wave-uniform) holds the seed
// of item kb and whose lanes below s0 hold earlier seeds (ignored): lo[j]
// and the result are lanes of the window.  Lanes above s0 start after kb,
// since compacted seeds are non-empty.
__device__ __forceinline__ int locate_short_at(u64 P, u64 kb, int s0, unsigned char *flag, int (&lo)[UN]) {
    const int lane = lane_id();
    const u32 Q = lane <= s0 ? 0u : (P - kb > 0xffffffffull ? 0xffffffffu : (u32)(P - kb));
    reinterpret_cast<u32 *>(flag)[lane] = 0u;
    wave_lds_fence();
    if (lane >= s0 && Q < (u32)(UN * WAVE)) flag[Q] = 1;  // the seed of kb marks item 0
    wave_lds_fence();
    u32 started = 0;
#pragma unroll
    for (int j = 0; j < UN; j++) {
        const u32 f = flag[j * WAVE + lane];
        const u64 S = __ballot(f != 0u);
        lo[j] = s0 + (int)(started + f + (u32)__popcll(S & lanemask_lt())) - 1;
        started += (u32)__popcll(S);
    }
    wave_lds_fence();
    return s0 + (int)started - 1;
}

// UN independent branchless membership tests of y[j] in the sorted list
// T[lo, hi) (the same list for all j), so their loads overlap.  Indices are
// 32-bit: adjacency arrays hold fewer than 2^32 entries.
__device__ __forceinline__ void member_multi(const u32 *T, u64 lo64, u64 hi64, const u32 (&y)[UN], bool (&hit)[UN]) {
    const u32 lo = (u32)lo64;
    u32 n = (u32)(hi64 - lo64);
    if (n == 0) {
#pragma unroll
        for (int j = 0; j < UN; j++) hit[j] = false;
        return;
    }
    u32 b[UN];
#pragma unroll
    for (int j = 0; j < UN; j++) b[j] = lo;
    while (n > 1) {
        const u32 half = n >> 1;
#pragma unroll
        for (int j = 0; j < UN; j++) b[j] = (T[b[j] + half] <= y[j]) ? b[j] + half : b[j];
        n -= half;
    }
#pragma unroll
    for (int j = 0; j < UN; j++) hit[j] = T[b[j]] == y[j];
}

// For each element, the last index b[j] in T[lo[j], hi[j]) with T[b] <= y[j]
// (lo[j] when the range is empty or T[lo[j]] > y[j]); interleaved as
// member_multi_var32.
__device__ __forceinline__ void bound_multi_var32(const u32 *T, const u32 (&lo)[UN], const u32 (&hi)[UN],
                                                  const u32 (&y)[UN], u32 (&b)[UN]) {
    u32 n[UN];
    u32 nmax = 0;
#pragma unroll
    for (int j = 0; j < UN; j++) {
        b[j] = lo[j];
        n[j] = hi[j] > lo[j] ? hi[j] - lo[j] : 0u;
        nmax = n[j] > nmax ? n[j] : nmax;
    }
    while (nmax > 1) {
        nmax = 0;
#pragma unroll
        for (int j = 0; j < UN; j++) {
            if (n[j] > 1) {
                const u32 half = n[j] >> 1;
                b[j] = (T[b[j] + half] <= y[j]) ? b[j] + half : b[j];
                n[j] -= half;
            }
            nmax = n[j] > nmax ? n[j] : nmax;
        }
    }
}

// As member_multi_var, with 32-bit bounds.
__device__ __forceinline__ void member_multi_var32(const u32 *T, const u32 (&lo)[UN], const u32 (&hi)[UN],
                                                   const u32 (&y)[UN], bool (&hit)[UN]) {
    u32 b[UN], n[UN];
    u32 nmax = 0;
#pragma unroll
    for (int j = 0; j < UN; j++) {
        b[j] = lo[j];
        n[j] = hi[j] > lo[j] ? hi[j] - lo[j] : 0u;
        nmax = n[j] > nmax ? n[j] : nmax;
    }
    while (nmax > 1) {
        nmax = 0;
#pragma unroll
        for (int j = 0; j < UN; j++) {
            if (n[j] > 1) {
                const u32 half = n[j] >> 1;
                b[j] = (T[b[j] + half] <= y[j]) ? b[j] + half : b[j];
                n[j] -= half;
            }
            nmax = n[j] > nmax ? n[j] : nmax;
        }
    }
#pragma unroll
    for (int j = 0; j < UN; j++) hit[j] = n[j] == 1 && T[b[j]] == y[j];
}

// As member_multi, with a different list T[lo[j], hi[j]) per element.
__device__ __forceinline__ void member_multi_var(const u32 *T, const u64 (&lo)[UN], const u64 (&hi)[UN],
                                                 const u32 (&y)[UN], bool (&hit)[UN]) {
    u32 b[UN], n[UN];
    u32 nmax = 0;
#pragma unroll
    for (int j = 0; j < UN; j++) {
        b[j] = (u32)lo[j];
        n[j] = hi[j] > lo[j] ? (u32)(hi[j] - lo[j]) : 0u;
        nmax = n[j] > nmax ? n[j] : nmax;
    }
    while (nmax > 1) {
        nmax = 0;
#pragma unroll
        for (int j = 0; j < UN; j++) {
            if (n[j] > 1) {
                const u32 half = n[j] >> 1;
                b[j] = (T[b[j] + half] <= y[j]) ? b[j] + half : b[j];
                n[j] -= half;
            }
            nmax = n[j] > nmax ? n[j] : nmax;
        }
    }
#pragma unroll
    for (int j = 0; j < UN; j++) hit[j] = n[j] == 1 && T[b[j]] == y[j];
}

}  // namespace
