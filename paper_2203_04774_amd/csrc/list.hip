// Triangle listing over the oriented CSR: Algorithm 1 (A++), Algorithm 2
// (A+-) and the S2-seeded variant (A--).
//
// Every form has the same shape: a pivot p whose list T is marked (the
// paper's boolean array B), seed edges (p, x) with x in T, and for each seed
// edge a scanned list S_x whose elements are tested against T.
//   A++  pivot w, T = N-_w, seed (u,w): S = N+_u      work d+_u  (C++)
//   A+-  pivot u, T = N+_u, seed (u,v): S = N+_v      work d+_v  (C+-)
//   A--  pivot v, T = N-_v, seed (v,w): S = N-_w      work d-_w  (sum d-d-)
// Lists are sorted ranks, so only the part of S inside [min, max] of the
// candidate part of T can match; for A++ and A+- the candidates are the
// entries of T after x itself (a triangle needs the third vertex on the far
// side of x, and every element of S_x already lies there).
//
// Plan (per listing): a window per seed edge; per-pivot work W_p; pivots with
// enough work become "heavy"; non-empty seed edges are compacted with the
// light pivots' ones first, then the heavy ones (pivot-major), and their
// window lengths prefix-summed into one flattened work space.
// Probe: light items are spread evenly over wavefronts, one scanned element
// per lane, tested by binary search in T (global memory).  Heavy pivots are
// cut into tasks of item slices; a 1024-thread workgroup per task stages T in
// LDS -- as the paper's boolean array B (a bitmap over T's rank window) when
// that window fits, else as a sorted array -- and then tests each scanned
// element with one (or log |T|) LDS reads.
#include <algorithm>
#include <cstdio>
#include <vector>
#include <cstdlib>
#include <mutex>

#include <type_traits>

#include "tl_internal.h"
#include "dev_util.h"
#include "timing.h"
#include "holes.h"
#include "probe_common.h"

namespace {

#ifndef TL_KEEP_WINDOW
#define TL_KEEP_WINDOW 1
#endif

// Heavy-kernel shape, fixed at build time (measured on RMAT scale 26):
//   TL_HB      threads per heavy workgroup (1024: 16 wavefronts hide latency;
//              512 measured 45% slower even with deeper load batches)
//   TL_HG      long-window groups of UN chunks loaded together (2; 3 and 4
//              measured no faster, nor did loading the next batch before
//              testing this one)
//   TL_SG      short-window groups located and loaded before the first is
//              tested (3; 1 and 2 measured slower, 4 exceeds 128 registers)
//   TL_SUB_S/D units of a task per wavefront walked as its own share / taken
//              from the shared tail
constexpr int PB = 256;        // threads per block, light kernels
#ifndef TL_HB
#define TL_HB 1024
#endif
#ifndef TL_HG
#define TL_HG 2
#endif
#ifndef TL_SG
#define TL_SG 3
#endif
#ifndef TL_SUB_S
#define TL_SUB_S 1
#endif
#ifndef TL_SUB_D
#define TL_SUB_D 3
#endif
constexpr int HB = TL_HB;      // threads per block, heavy-pivot kernel
constexpr u32 LDS_BYTES = 128 * 1024;
constexpr u32 LDS_WORDS = LDS_BYTES / 4;
constexpr u64 LDS_BITS = (u64)LDS_BYTES * 8;
constexpr u32 LOW_WORDS = 5088;  // SPLIT: list entries below the bitmap's window kept in LDS
constexpr u32 STAGE_WORDS = 2 * WAVE;  // per wavefront: 64 staged (endpoint, third vertex) pairs
constexpr u32 FLAG_WORDS = UN * WAVE / 4;  // per wavefront: seed-start flags of the short-window walk
#ifndef TL_LIGHT_LDS
#define TL_LIGHT_LDS 1
#endif
// light kernel: pivot-list entries in each wavefront's LDS window (256, 1024
// and 2048 measured no faster on Chung-Lu 2^20)
constexpr u32 LIGHT_LB = 512;
// bitmap + low entries + staging and flags for every wavefront: 160 KB in all
constexpr u32 HEAVY_LDS_BYTES = LDS_BYTES + LOW_WORDS * 4 + (HB / WAVE) * (STAGE_WORDS + FLAG_WORDS) * 4;
// (+128: the heavy kernel's own __shared__ variables)
static_assert(HEAVY_LDS_BYTES + 128 <= 160 * 1024, "heavy kernel LDS");
// Smallest task the balance cap (task_div) makes.
constexpr u64 BAL_TASK_MIN = 65536;
// Tunable launch parameters (defaults; tl_set_tuning or TL_TUNE_* env vars).
struct Tuning {
    // defaults from sweeps on the Chung-Lu 2^20 workload (random and degree
    // orders, A++ and A+-) on MI355X
    u64 heavy_min = 8192;        // items of a pivot before it gets a workgroup
    u64 slice_min = 262144;      // items per heavy task, at least
    u64 slice_mult = 2;          // ... and at least this many times its staging cost
    u64 task_div = 32;           // ... but at most the listing's work / (this * heavy workgroups), at
                                 // least BAL_TASK_MIN (0: no such cap)
    u64 heavy_blocks_per_cu = 1; // heavy grid = this many workgroups per CU
    u64 queue = 1;               // 1: heavy tasks handed out by an atomic queue
    u64 splits = 1;              // 1: wavefront start seeds precomputed at plan time
    u64 keep_staged = 1;         // 1: a workgroup keeps its pivot's list staged for a next task of that pivot
    u64 lean = 1;                // 1: the BITMAP/SPLIT-only heavy kernel when no task has another form
    u64 light_blocks_per_cu = 16; // light grid cap
    u64 light_wave_items = 8192;  // light grid: at least this many items per wavefront
    u64 reverse = 0;             // 1: REVERSE instead of GLOBAL for lists that fit no LDS form
    u64 hash = 0;                // 1: HASH before ARRAY when B's window does not fit LDS
    u64 bucket = 0;              // 1: BUCKET before ARRAY when B's window does not fit LDS
    u64 split = 2;               // 1: SPLIT for lists too long for LDS; 2: also before ARRAY/BUCKET
    u64 orient_sort = 1;         // 1: orientation by radix sort; 0: by per-vertex counters and scatter
    u64 force_mode = 255;        // testing: use this MODE_* for every heavy pivot where it fits
    u64 plan_full = 16;          // scanned lists this short are taken whole (no window searches);
                                 // below UN * WAVE, so that whole lists never fill a long window
    // callback mode, chunks of K triangles (sweeps on RMAT scale 26, A++):
    u64 chunk_task_div = 64;     // heavy tasks hold at most room K / (this * heavy workgroups) items,
                                 // so that each slice's launch ends with a short tail (64: 856 ->
                                 // 849 ms heavy per RMAT-26 listing against 32)
    u64 chunk_growth = 1;        // a slice's items grow at most this factor per slice (1: room x K
                                 // items each, which can never overflow the chunk)
    u64 chunk_margin = 125;      // percent margin over the last slice's triangles per item
    u64 chunk_room = 4;          // the device chunk holds this many times K triangles, handed out K
                                 // at a time: slices of room x K items (sweeps on RMAT scale 26)
};
Tuning &tuning();

// How a heavy task tests "y is marked" (y in the pivot's list T):
//   BITMAP   T's rank window fits LDS: one LDS read (the paper's B)
//   ARRAY    T itself fits LDS: binary search in LDS
//   GLOBAL   binary search of T in global memory
//   REVERSE  test the same edge from y's side: for A++ and A--, y in N-_p
//            iff p in N+_y; for A+-, y in N+_p iff p in N-_y -- a search of
//            y's own sorted list
//   HASH     T in an LDS open-addressing table (linear probing, load <= 1/2)
//   BUCKET   T in LDS with a table of where each of 8192 equal slices of its
//            rank window starts: one table read, then a binary search of the
//            few entries of y's slice
//   SPLIT    the top LDS_BITS ranks of T's window as an LDS bitmap (B for the
//            entries that lie there), the entries below binary-searched in
//            an LDS array when at most LOW_WORDS of them, else in global
//            memory; under orders that put hubs last most scanned elements
//            fall in the top part
enum { MODE_BITMAP = 0, MODE_ARRAY = 1, MODE_GLOBAL = 2, MODE_REVERSE = 3, MODE_HASH = 4, MODE_BUCKET = 5,
       MODE_SPLIT = 6 };
constexpr int NMODES = 7;
constexpr int ACC_PATHS = 10 + NMODES;  // heavy-walk counters in the listing's accumulator array
constexpr int NACC = ACC_PATHS + 8;
constexpr u32 BUCKETS = 8192;                              // slices of the rank window
constexpr u32 BUCKET_MAX = LDS_WORDS - (BUCKETS + 2) / 2;  // list entries beside a u16 start table

// log2 of the slice width: the smallest s with (range - 1) >> s < BUCKETS
__host__ __device__ __forceinline__ u32 bucket_shift(u64 range) {
    u32 sh = 0;
    while (((range - 1) >> sh) >= BUCKETS) sh++;
    return sh;
}

constexpr u32 HASH_MAX = LDS_WORDS / 2;  // list entries a task's hash table holds

__device__ __forceinline__ u32 hash_bits_for(u32 tlen) {
    u32 k = 1;
    while ((1u << k) < 2 * tlen) k++;
    return k;  // table of 2^k slots, 2^k >= 2 |T|
}

__device__ __forceinline__ u32 hash_slot(u32 y, u32 k) { return (y * 2654435761u) >> (32 - k); }

// the list searched by MODE_REVERSE for an element y of the scanned list
template <int ALGO>
struct Reverse {
    static __device__ __forceinline__ const u64 *off(const GView &g) { return ALGO == 1 ? g.off_b : g.off_f; }
    static __device__ __forceinline__ const u32 *adj(const GView &g) { return ALGO == 1 ? g.adj_b : g.adj_f; }
};

constexpr int HW = HB / 64;    // wavefronts per heavy workgroup
constexpr int HG = TL_HG;      // groups of UN chunks loaded together in the bitmap forms' long windows

struct Task {
    u64 a, b;      // item range
    u64 cb, ce;    // compacted seed range of the pivot
    u64 t0, t1;    // the pivot's list T: piv_adj[t0, t1)
    u64 ts;        // SPLIT: T's first entry inside the bitmap's window (else t0)
    u32 p;         // pivot
    u32 mode;
    u32 tmin, tmax;  // T's first and last entries
    u32 pinv;      // original id of the pivot
    u32 ss[(1 + TL_SUB_D) * HW];  // seed (relative to cb) of each sub-range's first item
};

// SPLIT: the bitmap covers ranks [split_wlo, tmax], the top LDS_BITS ranks
// up to the list's last entry (or the whole range when it fits)
__host__ __device__ __forceinline__ u32 split_wlo(u32 tmin, u32 tmax) {
    return (u64)tmax - tmin + 1 > LDS_BITS ? (u32)((u64)tmax + 1 - LDS_BITS) : tmin;
}

// A task's items [a, b) in (S + D) HW units (64-aligned), in (1 + D) HW
// sub-ranges: sub-range w < HW, S units, is wavefront w's own share; each
// of the last D HW units is a sub-range that the first wavefronts to finish
// take in turn, so that a task ends with its wavefronts at most about one
// unit apart instead of waiting at the next task's barrier for the slowest
// share.  (S, D) = (1, 3) measured best on RMAT scale 26 among (3, 1),
// (2, 2), (1, 1), (3, 2), (1, 5), (1, 7), (0, 4) and (2, 4).
constexpr u32 SUB_S = TL_SUB_S, SUB_D = TL_SUB_D;
constexpr u32 NSUB = (1 + SUB_D) * HW;
__host__ __device__ __forceinline__ void sub_range(u64 a, u64 b, u32 i, u64 &sa, u64 &sb) {
    constexpr u64 units = (u64)(SUB_S + SUB_D) * HW;
    const u64 per = ((((b - a) + units - 1) / units) + 63) & ~(u64)63;
    const u64 u0 = i < (u32)HW ? (u64)SUB_S * i : (u64)SUB_S * HW + (i - HW);
    const u64 u1 = i < (u32)HW ? u0 + SUB_S : u0 + 1;
    sa = a + u0 * per < b ? a + u0 * per : b;
    sb = a + u1 * per < b ? a + u1 * per : b;
}

// ---------------------------------------------------------------- plan

// Window of every seed edge; per-pivot items W_p and per-pivot paper's work
// (segmented by pivot, since seeds are pivot-major); the paper's work for the
// listed pivots.
// A++ windows: whether to leave the entries of N+_x between the last
// candidate t_max and the pivot p in the window (they are scanned and fail
// the membership test) instead of searching for t_max: when that rank span
// is under 1/64 of the candidates' span [t_min, p), the search's cache lines
// cost more than the few entries (RMAT-26, degree order: plan 98 -> 81 ms for
// 0.07% more items; under random orders the span is about 2/degree of it
// and the search is kept).
__host__ __device__ __forceinline__ bool tail_is_short(u32 p, u32 tmin, u32 tmax) {
    return (u64)(p - tmax) * 64 <= (u64)(p - tmin);
}

template <int ALGO>
__global__ __launch_bounds__(PB) void k_plan(GView g, u32 plo, u32 phi, u32 full_max, u32 *len, u64 *sabs, u64 *wp,
                                             u64 *wpw, u64 *acc) {
    __shared__ u64 lds[PB / WAVE];
    u64 work = 0;
    const int lane = lane_id();
    const u64 stride = (u64)gridDim.x * blockDim.x;
    const u64 first = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    const u64 iters = g.m > first - lane ? (g.m - (first - lane) + stride - 1) / stride : 0;  // wave-uniform
    for (u64 it = 0; it < iters; it++) {
        const u64 e = first + it * stride;
        const bool valid = e < g.m;
        u32 l = 0, p = 0xffffffffu;
        u64 abs = 0, pw = 0;
        if (valid) {
            Seed<ALGO> sd(g, e);
            p = sd.p;
            if (sd.p >= plo && sd.p < phi) {
                pw = sd.s_hi - sd.s_lo;
                work += pw;
                if (sd.t_lo < sd.t_hi && sd.s_lo < sd.s_hi) {
                    if (sd.s_hi - sd.s_lo <= full_max) {
                        // short list: scanned whole; the elements outside the
                        // window fail the membership test like any non-member
                        l = (u32)(sd.s_hi - sd.s_lo);
                        abs = sd.s_lo;
                    } else {
                        const u32 tmin = sd.T[sd.t_lo], tmax = sd.T[sd.t_hi - 1];
                        // A++: the pivot p itself sits in S = N+_x at twin_b[e], above
                        // every candidate, so the window ends there or earlier
                        const u64 hi = ALGO == 0 ? (u64)sd.twin : sd.s_hi;
                        const u64 a = lower_bound_front<u32>(sd.S, sd.s_lo, hi, tmin);
                        const u64 b = ALGO == 0 && tail_is_short(sd.p, tmin, tmax)
                                          ? hi : upper_bound_back<u32>(sd.S, a, hi, tmax);
                        l = (u32)(b - a);
                        abs = a;
                    }
                }
            }
            len[e] = l;
            sabs[e] = abs;
        }
        // segmented sums of l and of the paper's work over runs of equal pivot
        // within the wavefront
        u64 v = l, vw = pw;
#pragma unroll
        for (int d = 1; d < WAVE; d <<= 1) {
            const u64 t = shfl_up_u64(v, d), tw = shfl_up_u64(vw, d);
            const u32 q = __shfl_up(p, d, WAVE);
            if (lane >= d && q == p) {
                v += t;
                vw += tw;
            }
        }
        const u32 pn = __shfl_down(p, 1, WAVE);
        const bool last = valid && (lane == WAVE - 1 || pn != p || !(e + 1 < g.m));
        if (last && v) atomicAdd((unsigned long long *)&wp[p], (unsigned long long)v);
        if (last && vw) atomicAdd((unsigned long long *)&wpw[p], (unsigned long long)vw);
    }
    u64 tot = block_sum_u64<PB>(work, lds);
    if (threadIdx.x == 0 && tot) atomicAdd((unsigned long long *)&acc[2], (unsigned long long)tot);
}

// Heavy/light decision and task count per pivot.
template <int ALGO>
__global__ __launch_bounds__(PB) void k_pivot_class(GView g, u32 n, const u64 *wp, const u64 *wpw, u32 *mode,
                                                    u32 *ntask,
                                                    u64 *slice, u64 heavy_min, u64 slice_min, u64 slice_mult,
                                                    u64 max_task, u64 bal_div, u64 reverse, u64 use_hash,
                                                    u64 use_bucket, u64 use_split, u64 force_mode, u64 *acc) {
    __shared__ u64 lds[PB / WAVE];
    __shared__ u64 mode_items[NMODES];  // heavy items per form, summed in LDS (one global atomic per form)
    if (threadIdx.x < NMODES) mode_items[threadIdx.x] = 0;
    __syncthreads();
    // balance: no task above 1/bal_div of the listing's work (acc[2], summed
    // by the plan kernel), so that a few hub pivots do not end the launch alone
    u64 bal = 0;
    if (bal_div) {
        bal = acc[2] / bal_div;
        if (bal < BAL_TASK_MIN) bal = BAL_TASK_MIN;
    }
    u64 hp = 0, staged = 0, hwork = 0;
    GRID_STRIDE(p, n) {
        const u64 w = wp[p];
        u32 md = 0xffffffffu, nt = 0;
        u64 sl = 0;
        if (w >= heavy_min) {
            const u64 *po = Form<ALGO>::piv_off(g);
            const u32 *pa = Form<ALGO>::piv_adj(g);
            const u64 t0 = po[p], t1 = po[p + 1];
            const u64 tlen = t1 - t0;
            const u64 range = (u64)pa[t1 - 1] - pa[t0] + 1;
            const bool bm_ok = range <= LDS_BITS;
            const bool arr_ok = tlen <= LDS_WORDS;
            // the bitmap is kept clear between tasks, so marking and
            // unmarking cost 2 |T| (the paper's set/reset of B)
            u64 stage;
            if (force_mode == MODE_BITMAP && bm_ok) { md = MODE_BITMAP; stage = 2 * tlen; }
            else if (force_mode == MODE_ARRAY && arr_ok) { md = MODE_ARRAY; stage = 2 * tlen; }
            else if (force_mode == MODE_GLOBAL) { md = MODE_GLOBAL; stage = 0; }
            else if (force_mode == MODE_REVERSE) { md = MODE_REVERSE; stage = 0; }
            else if (force_mode == MODE_HASH && tlen <= HASH_MAX) { md = MODE_HASH; stage = 2 * tlen + 2 * tlen; }
            else if (force_mode == MODE_BUCKET && tlen <= BUCKET_MAX) {
                md = MODE_BUCKET;
                stage = 2 * tlen + 16 * BUCKETS;
            }
            else if (force_mode == MODE_SPLIT) { md = MODE_SPLIT; stage = 2 * tlen; }
            else if (bm_ok) { md = MODE_BITMAP; stage = 2 * tlen; }
            else if (use_split >= 2) { md = MODE_SPLIT; stage = 2 * tlen; }
            else if (use_hash && tlen <= HASH_MAX) { md = MODE_HASH; stage = 4 * tlen; }
            else if (use_bucket && tlen <= BUCKET_MAX) { md = MODE_BUCKET; stage = 2 * tlen + 16 * BUCKETS; }
            else if (arr_ok) { md = MODE_ARRAY; stage = 2 * tlen; }
            else if (use_split) { md = MODE_SPLIT; stage = 2 * tlen; }
            else if (reverse) { md = MODE_REVERSE; stage = 0; }
            else { md = MODE_GLOBAL; stage = 0; }
            sl = slice_mult * stage;
            if (sl < slice_min) sl = slice_min;
            if (bal && sl > bal) sl = bal;
            if (max_task && sl > max_task) sl = max_task;
            nt = (u32)((w + sl - 1) / sl);
            hp += 1;
            staged += tlen;
            hwork += wpw[p];

            atomicAdd((unsigned long long *)&mode_items[md], (unsigned long long)w);
        }
        mode[p] = md;
        ntask[p] = nt;
        slice[p] = sl;
    }
    hp = block_sum_u64<PB>(hp, lds);  // synchronises: mode_items is complete
    staged = block_sum_u64<PB>(staged, lds);
    hwork = block_sum_u64<PB>(hwork, lds);
    if (threadIdx.x == 0 && hp) {
        atomicAdd((unsigned long long *)&acc[7], (unsigned long long)hp);
        atomicAdd((unsigned long long *)&acc[9], (unsigned long long)staged);
        atomicAdd((unsigned long long *)&acc[6], (unsigned long long)hwork);  // the heavy pivots' paper's work
    }
    if (threadIdx.x < NMODES && mode_items[threadIdx.x])
        atomicAdd((unsigned long long *)&acc[10 + threadIdx.x], (unsigned long long)mode_items[threadIdx.x]);
}

// Class flag per seed, packed for one scan: low half light, high half heavy.
template <int ALGO>
__global__ __launch_bounds__(PB) void k_seed_class(GView g, const u32 *len, const u32 *mode, u64 *flags) {
    GRID_STRIDE(e, g.m) {
        u64 f = 0;
        if (len[e]) {
            const u32 p = ALGO == 0 ? g.row_b[e] : g.row_f[e];
            f = mode[p] == 0xffffffffu ? 1ull : 1ull << 32;
        }
        flags[e] = f;
    }
}

// Light seeds first, then heavy seeds, both in seed (pivot-major) order.
// Also records, per compacted seed, the original id of the seed edge's other
// endpoint, so that a hit needs no dependent lookups to name it.
// Light seeds also get their candidate range of T and the pivot's id.
template <int ALGO>
__global__ void k_compact(GView g, const u32 *len, const u64 *sabs, const u64 *pos, u64 *cabs,
                          u32 *cxinv, u32 *clen, u32 *ctlo, u32 *cthi, u32 *cpinv) {
    const u64 m = g.m;
    const u64 nl = pos[m] & 0xffffffffull;
    GRID_STRIDE(e, m) {
        const u32 l = len[e];
        if (l) {
            const u64 ps = pos[e];
            const bool heavy = ((ps >> 32) != (pos[e + 1] >> 32));
            const u64 d = heavy ? nl + (ps >> 32) : (ps & 0xffffffffull);
            cabs[d] = sabs[e];
            cxinv[d] = g.inv[Form<ALGO>::seed_adj(g)[e]];
            clen[d] = l;
            if (!heavy) {
                Seed<ALGO> sd(g, e);
                ctlo[d] = (u32)sd.t_lo;
                cthi[d] = (u32)sd.t_hi;
                cpinv[d] = g.inv[sd.p];
            }
        }
    }
}

// The plan's totals, gathered for one read by the host: packed compacted
// seed counts (light | heavy << 32), heavy tasks, light items, all items and
// the paper's work (acc[2]).
__global__ void k_plan_totals(const u64 *pos, u64 m, const u64 *tpos, u32 n, const u64 *cpre, const u64 *acc,
                              u64 *out) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const u64 hp = pos[m];
        out[0] = hp;
        out[1] = tpos[n];
        out[2] = cpre[hp & 0xffffffffull];
        out[3] = cpre[m];
        out[4] = acc[2];
        // items of heavy pivots in forms other than BITMAP and SPLIT
        u64 other = 0;
        for (int md = 0; md < NMODES; md++)
            if (md != MODE_BITMAP && md != MODE_SPLIT) other += acc[10 + md];
        out[5] = other;
    }
}

template <int ALGO>
__global__ void k_make_tasks(GView g, u32 n, const u32 *mode, const u32 *ntask, const u64 *slice, const u64 *tpos,
                             const u64 *pos, const u64 *cpre, u64 m, Task *tasks) {
    const u64 nl = pos[m] & 0xffffffffull;
    GRID_STRIDE(p, n) {
        const u32 nt = ntask[p];
        if (!nt) continue;
        const u64 *so = Form<ALGO>::seed_off(g);
        const u64 cb = nl + (pos[so[p]] >> 32), ce = nl + (pos[so[p + 1]] >> 32);
        const u64 a = cpre[cb], b = cpre[ce];
        const u64 sl = slice[p];
        // the pivot list's geometry, found once here rather than by dependent
        // loads (and SPLIT's search) each time a workgroup stages the list
        const u64 *po = Form<ALGO>::piv_off(g);
        const u32 *pa = Form<ALGO>::piv_adj(g);
        const u64 t0 = po[p], t1 = po[p + 1];
        const u32 tmin = pa[t0], tmax = pa[t1 - 1], md = mode[p];
        const u64 ts = md == MODE_SPLIT ? lower_bound_dev<u32>(pa, t0, t1, split_wlo(tmin, tmax)) : t0;
        const u32 pinv = g.inv[p];
        for (u32 i = 0; i < nt; i++) {
            Task t;
            t.a = a + (u64)i * sl;
            t.b = (t.a + sl < b) ? t.a + sl : b;
            t.cb = cb;
            t.ce = ce;
            t.t0 = t0;
            t.t1 = t1;
            t.ts = ts;
            t.p = (u32)p;
            t.mode = md;
            t.tmin = tmin;
            t.tmax = tmax;
            t.pinv = pinv;
            for (u32 w = 0; w < NSUB; w++) t.ss[w] = 0;
            tasks[tpos[p] + i] = t;
        }
    }
}

// Seed of every task sub-range's first item, found once at plan time (in
// parallel over tasks) instead of by a dependent search when a wavefront
// starts the sub-range.
__global__ void k_task_splits(Task *tasks, u64 ntasks, const u64 *cpre) {
    GRID_STRIDE(i, ntasks * NSUB) {
        const u64 ti = i / NSUB;
        const u32 w = (u32)(i % NSUB);
        const Task &t = tasks[ti];
        u64 sa, sb;
        sub_range(t.a, t.b, w, sa, sb);
        u32 rel = 0;
        if (sa < sb) rel = (u32)(upper_bound_dev<u64>(cpre, t.cb, t.ce + 1, sa) - 1 - t.cb);
        tasks[ti].ss[w] = rel;
    }
}

// ---------------------------------------------------------------- probe

// Where listed triangles go.  Positions come from a global cursor in blocks
// of RESERVE triangles per wavefront (one atomic per block, not per hit).
// Positions below cap land in the caller's buffer; the next spill_cap
// positions in a library spill area; the unused tail of each wavefront's
// last block is recorded as a hole, and a fix-up step moves spilled
// triangles into the holes so that the output is exactly [0, count).
constexpr u64 RESERVE = 1024;

struct Out {
    u32 *tri;
    u64 cap;
    u32 *spill;
    u64 spill_cap;
    u64 *acc;      // [0] count, [1] digest, [2] work, [3] cursor, [4] holes, [5] task queue,
                   // [6] heavy work, [7] heavy pivots, [8] heavy triangles, [9] heavy staged elements,
                   // [10, 10 + NMODES) heavy items per LDS form, [ACC_PATHS, + 5) heavy walk counters
    Hole *holes;
    u64 hole_cap;

    __device__ __forceinline__ void put(u64 pos, u32 a, u32 b, u32 c) const {
        u32 *d;
        if (pos < cap) d = tri + 3 * pos;
        else if (pos - cap < spill_cap) d = spill + 3 * (pos - cap);
        else return;
        *reinterpret_cast<uint3 *>(d) = make_uint3(a, b, c);  // one 12-byte store
    }
};

template <bool EMIT>
struct WaveEmitter {
    u64 rb = 0, re = 0;  // wave-uniform reservation [rb, re)

    __device__ __forceinline__ void push(bool hit, u32 a, u32 b, u32 c, const Out &o) {
        if (!EMIT) return;
        const u64 bal = __ballot(hit);
        if (!bal) return;
        const u64 k = __popcll(bal);
        const u64 idx = __popcll(bal & lanemask_lt());
        const u64 avail = re - rb;
        u64 pos;
        if (avail >= k) {
            pos = rb + idx;
            rb += k;
        } else {
            u64 nb = 0;
            if (lane_id() == 0) nb = atomicAdd((unsigned long long *)&o.acc[3], (unsigned long long)RESERVE);
            // scalar from here on: the reservation's later uses carry no wait on memory
            nb = lane0_u64(nb);
            pos = idx < avail ? rb + idx : nb + (idx - avail);
            rb = nb + (k - avail);
            re = nb + RESERVE;
        }
        if (hit) o.put(pos, a, b, c);
    }

    __device__ __forceinline__ void finish(const Out &o) {
        if (!EMIT || re == rb) return;
        if (lane_id() == 0) {
            const u64 h = atomicAdd((unsigned long long *)&o.acc[4], 1ull);
            if (h < o.hole_cap) o.holes[h] = Hole{rb, re - rb};
        }
    }
};

__device__ __forceinline__ void flush_counts(u64 cnt, u64 hsh, u64 *acc) {
    cnt = wave_sum_u64(cnt);
    hsh = wave_sum_u64(hsh);
    if (lane_id() == 0 && cnt) {
        atomicAdd((unsigned long long *)&acc[0], (unsigned long long)cnt);
        atomicAdd((unsigned long long *)&acc[1], (unsigned long long)hsh);
    }
}

// Per-seed arrays of the light items.
struct LightSeeds {
    const u64 *cpre, *cabs;
    const u32 *cxinv, *ctlo, *cthi, *cpinv;
};

// Light items [k0, k1): each wavefront takes a contiguous run of items and
// tests each scanned element by binary search in the pivot's list, UN
// chunks of 64 items at a time whenever they fall in one seed window or in
// the 64 seeds starting at the current one.
template <int ALGO, bool EMIT>
__global__ __launch_bounds__(PB) void k_probe_light(GView g, const u64 *__restrict__ cpre, const u64 *__restrict__ cabs,
                                                    const u32 *__restrict__ cxinv, const u32 *__restrict__ ctlo,
                                                    const u32 *__restrict__ cthi, const u32 *__restrict__ cpinv,
                                                    u64 ncap, u64 k0, u64 k1, Out o) {
    // restrict-qualified arguments: reads at wave-uniform indices become scalar loads
    const LightSeeds L{cpre, cabs, cxinv, ctlo, cthi, cpinv};
    const int lane = lane_id();
    const u64 gw = (u64)blockIdx.x * (blockDim.x / WAVE) + wave_id();
    const u64 nw = ((u64)gridDim.x * blockDim.x) / WAVE;
    const u64 span = k1 - k0;
    const u64 per = (((span + nw - 1) / nw) + WAVE - 1) & ~(u64)(WAVE - 1);
    const u64 wb = k0 + gw * per;
    const u64 we = (wb + per < k1) ? wb + per : k1;
    const u32 *SA = Form<ALGO>::scan_adj(g);
    const u32 *T = Form<ALGO>::piv_adj(g);
    WaveEmitter<EMIT> em;
    u64 cnt = 0, hsh = 0;
    // per wavefront: 64 staged hits (pivot, endpoint, third vertex) and the
    // seed-start flags of the short-window walk
    __shared__ uint4 stage_all[(PB / WAVE) * WAVE];
    __shared__ unsigned char flag_all[(PB / WAVE) * UN * WAVE];
    uint4 *stage = stage_all + wave_id() * WAVE;
    unsigned char *flag = flag_all + wave_id() * (UN * WAVE);
#if TL_LIGHT_LDS
    // A sliding window over the pivot-list array T in LDS, per wavefront.
    // Seeds are pivot-major, so the candidate ranges [t_lo, t_hi) of the
    // wavefront's successive seeds only move forward through T (and the
    // lists of successive pivots lie next to each other in it): each entry
    // of T that the wavefront searches is staged about once, and a group
    // whose seeds' ranges all fit the window searches LDS instead of global
    // memory.
    __shared__ u32 twin_all[(PB / WAVE) * LIGHT_LB];
    u32 *tw = twin_all + wave_id() * LIGHT_LB;
    u64 tw_lo = 0, tw_hi = 0;  // T[tw_lo, tw_hi) is staged (wave-uniform)
    // whether T[lo, hi) (wave-uniform) is in the window, staging it if it fits
    auto cover = [&](u64 lo, u64 hi) -> bool {
        if (hi - lo > LIGHT_LB) return false;
        if (lo >= tw_lo && hi <= tw_hi) return true;
        const u64 e = lo + LIGHT_LB < g.m ? lo + LIGHT_LB : g.m;
        const u32 n = (u32)(e - lo);
        u32 v[LIGHT_LB / WAVE];
#pragma unroll
        for (int k = 0; k < (int)(LIGHT_LB / WAVE); k++) {
            const u32 i = (u32)(k * WAVE + lane);
            v[k] = i < n ? T[lo + i] : 0u;
        }
        wave_lds_fence();  // (earlier searches of the window are done)
#pragma unroll
        for (int k = 0; k < (int)(LIGHT_LB / WAVE); k++) tw[k * WAVE + lane] = v[k];
        wave_lds_fence();
        tw_lo = lo;
        tw_hi = e;
        return true;
    };
#endif
    // hits are packed into the staging area across groups and finished 64
    // at a time: id lookup, canonical order, digest and store on full
    // wavefronts whatever the hit rate
    u32 staged = 0;  // wave-uniform
    // Each batch of 64 is finished one flush late, so that its third
    // vertices' id gathers overlap the walk (measured faster here, though not
    // in the heavy kernel).
    u32 pend_k = 0, pend_a = 0, pend_b = 0, pend_c = 0;
    auto finish = [&]() {
        if (pend_k) {
            const bool v = (u32)lane < pend_k;
            u32 ta = 0, tb = 0, tc = 0;
            if (v) {
                ta = pend_a; tb = pend_b; tc = pend_c;
                canon3(ta, tb, tc);
                cnt += 1;
                hsh += tri_digest(ta, tb, tc);
            }
            em.push(v, ta, tb, tc, o);
            pend_k = 0;
        }
    };
    auto flush = [&](u32 k) {
        wave_lds_fence();
        const bool v = (u32)lane < k;
        uint4 e = make_uint4(0u, 0u, 0u, 0u);
        if (v) e = stage[lane];
        wave_lds_fence();
        finish();
        pend_k = k;
        pend_a = e.x;
        pend_b = e.y;
        pend_c = v ? g.inv[e.z] : 0u;
    };
    auto report = [&](const u32 (&y)[UN], const bool (&h)[UN], const u32 (&pv)[UN], const u32 (&xv)[UN]) {
        u64 bal[UN];
        u32 q[UN], tot = 0;
        const u64 lt = lanemask_lt();
#pragma unroll
        for (int j = 0; j < UN; j++) {
            bal[j] = __ballot(h[j]);
            q[j] = tot + (u32)__popcll(bal[j] & lt);
            tot += (u32)__popcll(bal[j]);
        }
        for (u32 r0 = 0; r0 < tot;) {
            const u32 room = (u32)WAVE - staged;
#pragma unroll
            for (int j = 0; j < UN; j++) {
                if (h[j] && q[j] - r0 < room) stage[staged + (q[j] - r0)] = make_uint4(pv[j], xv[j], y[j], 0u);
            }
            const u32 take = tot - r0 < room ? tot - r0 : room;
            staged += take;
            r0 += take;
            if (staged == (u32)WAVE) {
                flush(WAVE);
                staged = 0;
            }
        }
    };
    if (wb < we) {
        SeedCursor cur(L.cpre, 0, ncap, wb);
        u64 kb = wb;
        while (kb < we) {
            if (cur.end >= kb + UN * WAVE && kb + UN * WAVE <= we) {
                // UN full chunks inside one seed window
                const u64 c = cur.c_lo;
                const u64 sab = L.cabs[c] + (kb - cur.base) + lane;
                const u64 t_lo = L.ctlo[c], t_hi = L.cthi[c];
                u32 y[UN], pv[UN], xv[UN];
                bool h[UN];
#pragma unroll
                for (int j = 0; j < UN; j++) y[j] = SA[sab + (u64)j * WAVE];
#if TL_LIGHT_LDS
                if (cover(t_lo, t_hi)) member_multi(tw, t_lo - tw_lo, t_hi - tw_lo, y, h);
                else
#endif
                member_multi(T, t_lo, t_hi, y, h);
                const u32 pi = L.cpinv[c], xi = L.cxinv[c];
#pragma unroll
                for (int j = 0; j < UN; j++) { pv[j] = pi; xv[j] = xi; }
                report(y, h, pv, xv);
                kb += UN * WAVE;
                cur.advance(kb, c);
                continue;
            }
            if (kb + UN * WAVE <= we) {
                const u64 ci = cur.c_lo + lane;
                const bool inw = ci < ncap;
                const u64 P = inw ? L.cpre[ci] : ~0ull;
                const u64 pend = (cur.c_lo + WAVE <= ncap) ? L.cpre[cur.c_lo + WAVE] : ~0ull;
                if (pend >= kb + UN * WAVE) {
                    // the next UN chunks lie in the 64 seeds from the current one
                    const u64 A = inw ? L.cabs[ci] : 0ull;
                    const u32 X = inw ? L.cxinv[ci] : 0u, PI = inw ? L.cpinv[ci] : 0u;
                    const u32 TL = inw ? L.ctlo[ci] : 0u, TH = inw ? L.cthi[ci] : 0u;
                    // item kb + i of seed c: scan index E[c] + i (mod 2^32; m < 2^32)
                    const u32 E = (u32)(A - P + kb);
                    int lo[UN];
                    const int lo_last = locate_short(P, kb, flag, lo);
                    u32 y[UN], pv[UN], xv[UN];
                    u64 tl[UN], th[UN];
                    bool h[UN];
#pragma unroll
                    for (int j = 0; j < UN; j++) {
                        y[j] = SA[(u32)(__shfl(E, lo[j], WAVE) + (u32)(j * WAVE + lane))];
                        xv[j] = __shfl(X, lo[j], WAVE);
                        pv[j] = __shfl(PI, lo[j], WAVE);
                        tl[j] = __shfl(TL, lo[j], WAVE);
                        th[j] = __shfl(TH, lo[j], WAVE);
                    }
#if TL_LIGHT_LDS
                    // the group's seeds are window lanes 0 .. lo_last, whose ranges
                    // start no earlier than lane 0's and end no later than lo_last's
                    const u64 g_lo = (u32)__builtin_amdgcn_readlane((int)TL, 0);
                    const u64 g_hi = (u32)__builtin_amdgcn_readlane((int)TH, lo_last);
                    if (cover(g_lo, g_hi)) {
                        u32 l32[UN], h32[UN];
#pragma unroll
                        for (int j = 0; j < UN; j++) {
                            l32[j] = (u32)(tl[j] - tw_lo);
                            h32[j] = (u32)(th[j] - tw_lo);
                        }
                        member_multi_var32(tw, l32, h32, y, h);
                    } else
#endif
                    member_multi_var(T, tl, th, y, h);
                    report(y, h, pv, xv);
                    kb += UN * WAVE;
                    if (kb < we) {
                        u64 c = cur.c_lo + (u64)lo_last;
                        const u64 pn = (lo_last + 1 < WAVE) ? shfl_u64(P, lo_last + 1) : pend;
                        if (pn <= kb) c++;
                        cur.reset(c);
                    }
                    continue;
                }
            }
            const u64 k = kb + lane;
            const bool act = k < we;
            u64 rel;
            const u64 c = cur.locate(kb, k, rel);
            bool hit = false;
            u32 a = 0, b = 0, cc = 0;
            if (act) {
                const u32 y = SA[L.cabs[c] + rel];
                const u64 t_lo = L.ctlo[c], t_hi = L.cthi[c];
                const u64 j = lower_bound_dev<u32>(T, t_lo, t_hi, y);
                if (j < t_hi && T[j] == y) {
                    hit = true;
                    a = L.cpinv[c]; b = L.cxinv[c]; cc = g.inv[y];
                    canon3(a, b, cc);
                    cnt += 1;
                    hsh += tri_digest(a, b, cc);
                }
            }
            em.push(hit, a, b, cc, o);
            kb += WAVE;
            cur.advance(kb, c);
        }
    }
    if (staged) flush(staged);
    finish();
    em.finish(o);
    flush_counts(cnt, hsh, o.acc);
}

// Heavy tasks: one workgroup stages the pivot's list in LDS, then its
// wavefronts share the task's items.  Items are clipped to [k0, k1).
// LEAN: compiled with the BITMAP and SPLIT walks only (the forms the
// default tuning ever chooses), for fewer registers; used when no task of
// the listing has another form.
template <int ALGO, bool EMIT, bool LEAN>
__global__ __launch_bounds__(HB) void k_probe_heavy(GView g, const Task *__restrict__ tasks, u64 ntasks,
                                                    const u64 *__restrict__ cabs,
                                                    const u32 *__restrict__ cxinv, const u64 *__restrict__ cpre,
                                                    u64 k0, u64 k1, Out o, int use_queue, int use_splits,
                                                    int keep_staged) {
    extern __shared__ u32 lds[];  // the pivot list: B as a bitmap, or a sorted array
    const int lane = lane_id(), wid = (int)wave_id();
    const u32 *SA = Form<ALGO>::scan_adj(g);
    const u64 *po = Form<ALGO>::piv_off(g);
    const u32 *pa = Form<ALGO>::piv_adj(g);
    WaveEmitter<EMIT> em;
    u64 cnt = 0, hsh = 0;
    // Measurement counters of the workgroup, in LDS (kept out of registers):
    // items by walk path, SPLIT elements below the bitmap's window (searched)
    // and of those searched in global memory, list entries staged, SPLIT
    // groups and those that ran the below-window search.
    enum { ST_LONG, ST_SHORT, ST_SINGLE, ST_BELOW, ST_BELOW_GLOB, ST_STAGED, ST_GROUPS, ST_BELOW_GROUPS, ST_N };
    // Per-group counts gather in one register of the wavefront (lane k holds
    // counter k: no branch, no atomic in the walk) and reach LDS once per task.
    __shared__ u64 wstat[ST_N];
    u32 stv = 0;
    auto stat_add = [&](int k, u64 v) {  // wave-uniform call
        stv += lane == k ? (u32)v : 0u;
    };
    auto stat_flush = [&]() {  // per task: a wavefront's counts stay far below 2^32
        if (lane < ST_N && stv) atomicAdd((unsigned long long *)&wstat[lane], (unsigned long long)stv);
        stv = 0;
    };
    if (threadIdx.x < ST_N) wstat[threadIdx.x] = 0;
    __shared__ u64 next_task;
    __shared__ u32 next_sub;  // the task's next shared sub-range
    // The pivot whose list LDS holds.  A task that continues the same pivot
    // (hub pivots span many consecutive tasks, and a workgroup often takes
    // several of them) skips staging; LDS is reset only when the workgroup
    // moves to another pivot.  Block-uniform.
    u32 res_p = 0xffffffffu, res_mode = 0;
    u32 res_words = 0;  // LDS words [0, res_words) the resident list may have set
    for (u32 i = threadIdx.x; i < LDS_WORDS; i += blockDim.x) lds[i] = 0u;  // B starts all false
    __syncthreads();
    for (u64 it = 0;; it++) {
        u64 ti;
        if (use_queue) {
            // tasks handed out dynamically: one atomic per task per workgroup
            // (taking the next index one task ahead measured slower)
            if (threadIdx.x == 0) next_task = atomicAdd((unsigned long long *)&o.acc[5], 1ull);
            __syncthreads();  // (every wavefront is done with the previous task)
            ti = uni64(next_task);
            if (threadIdx.x == 0) next_sub = HW;
            __syncthreads();
        } else {
            __syncthreads();
            if (threadIdx.x == 0) next_sub = HW;
            __syncthreads();
            ti = blockIdx.x + it * gridDim.x;
        }
        if (ti >= ntasks) break;
        if (use_queue && tasks[ti].a >= k1) break;  // sorted: no later task overlaps [k0, k1)
        // fields are read one by one: copying the struct and indexing its
        // per-wavefront array would put it in scratch memory
        const Task &tg = tasks[ti];
        struct {
            u64 a, b, cb, ce, t0, t1, ts;
            u32 p, mode, tmin, tmax, pinv;
        } tk{uni64(tg.a),  uni64(tg.b),  uni64(tg.cb),   uni64(tg.ce),   uni64(tg.t0),  uni64(tg.t1),
             uni64(tg.ts), uni32(tg.p),  uni32(tg.mode), uni32(tg.tmin), uni32(tg.tmax), uni32(tg.pinv)};
        const u64 a = tk.a > k0 ? tk.a : k0;
        const u64 b = tk.b < k1 ? tk.b : k1;
        if (a >= b) continue;  // uniform across the block
        const u32 p = tk.p;
        const bool restage = !keep_staged || p != res_p || tk.mode != res_mode;  // block-uniform
        if (restage && res_p != 0xffffffffu) {
            // LDS back to all zero (the paper resets B by unmarking the list's
            // entries; here the words the list can have set are cleared, 128-bit
            // writes from LDS alone, which costs no reads of the list), once
            // every wavefront is done with it
            if (!use_queue) __syncthreads();  // (the queue's barriers order it otherwise)
            const u32 q4 = (res_words + 3) / 4 < LDS_WORDS / 4 ? (res_words + 3) / 4 : LDS_WORDS / 4;
            uint4 *l4 = reinterpret_cast<uint4 *>(lds);
            for (u32 i = threadIdx.x; i < q4; i += blockDim.x) l4[i] = make_uint4(0u, 0u, 0u, 0u);
            __syncthreads();
            res_p = 0xffffffffu;
        }
        const u64 t0 = tk.t0, t1 = tk.t1;
        const u32 tmin = tk.tmin, tmax = tk.tmax;
        const u32 tlen = (u32)(t1 - t0);
        // SPLIT: the bitmap covers ranks [wlo, tmax]; entries [t0, ts) lie below
        const u32 wlo = split_wlo(tmin, tmax);
        const u64 ts = tk.ts;
        u32 *low = lds + LDS_WORDS;  // SPLIT: T[t0, ts) when it fits
        uint2 *stage = reinterpret_cast<uint2 *>(lds + LDS_WORDS + LOW_WORDS + (u32)wid * STAGE_WORDS);
        unsigned char *flag =
            reinterpret_cast<unsigned char *>(lds + LDS_WORDS + LOW_WORDS + HW * STAGE_WORDS + (u32)wid * FLAG_WORDS);
        const bool low_lds = tk.mode == MODE_SPLIT && ts - t0 <= LOW_WORDS;
        // SPLIT lists with more entries below the window than LOW holds: LOW
        // keeps every lstride-th of them, so that a search there leaves one
        // stride of the list to search in global memory
        const u32 lstride = (tk.mode == MODE_SPLIT && !low_lds) ? (u32)((ts - t0 + LOW_WORDS - 1) / LOW_WORDS) : 1u;
        const u32 lsamp = (tk.mode == MODE_SPLIT && !low_lds) ? (u32)((ts - t0 + lstride - 1) / lstride) : 0u;
        if (!restage) {
            // the list is already staged
        } else {
        res_p = p;
        res_mode = tk.mode;
        res_words = (tk.mode == MODE_BITMAP || tk.mode == MODE_SPLIT) ? ((tmax - wlo) >> 5) + 1
                    : tk.mode == MODE_ARRAY                          ? tlen
                    : tk.mode == MODE_BUCKET                         ? tlen + (BUCKETS + 2) / 2
                    : tk.mode == MODE_HASH                           ? 1u << hash_bits_for(tlen)
                                                                     : 0u;
        if (threadIdx.x == 0)
            atomicAdd((unsigned long long *)&wstat[ST_STAGED],
                      (unsigned long long)((tk.mode == MODE_BITMAP || tk.mode == MODE_SPLIT)
                                               ? (t1 - ts) + (low_lds ? ts - t0 : 0)
                                           : (tk.mode == MODE_GLOBAL || tk.mode == MODE_REVERSE) ? 0 : tlen));
        // staging loops keep SU loads of the list in flight per thread: a
        // list of L entries costs about L / (SU x 1024) memory round trips
        constexpr int SU = 8;
        if (tk.mode == MODE_SPLIT) {
            // all entries below the window, or every lstride-th of them
            const u32 *src = pa + t0;
            const u32 nl = low_lds ? (u32)(ts - t0) : lsamp, bd = blockDim.x;  // (lists hold < 2^32 entries)
            for (u32 i = threadIdx.x; i < nl; i += SU * bd) {
                u32 v[SU];
#pragma unroll
                for (int k = 0; k < SU; k++) v[k] = i + k * bd < nl ? src[(i + k * bd) * lstride] : 0u;
#pragma unroll
                for (int k = 0; k < SU; k++)
                    if (i + k * bd < nl) low[i + k * bd] = v[k];
            }
        }
        if (tk.mode == MODE_BITMAP || tk.mode == MODE_SPLIT) {
            const u32 *src = pa + ts;
            const u32 nb = (u32)(t1 - ts), bd = blockDim.x;
            for (u32 i = threadIdx.x; i < nb; i += SU * bd) {
                u32 v[SU];
#pragma unroll
                for (int k = 0; k < SU; k++) v[k] = i + k * bd < nb ? src[i + k * bd] : wlo;
#pragma unroll
                for (int k = 0; k < SU; k++) {
                    const u32 d = v[k] - wlo;
                    if (i + k * bd < nb) atomicOr(&lds[d >> 5], 1u << (d & 31));
                }
            }
            __syncthreads();
        } else if (tk.mode == MODE_ARRAY) {
            for (u32 i = threadIdx.x; i < tlen; i += blockDim.x) lds[i] = pa[t0 + i];
            __syncthreads();
        } else if (tk.mode == MODE_BUCKET) {
            for (u32 i = threadIdx.x; i < tlen; i += blockDim.x) lds[i] = pa[t0 + i];
            __syncthreads();
            // start of slice b: the first entry >= tmin + (b << sh)
            const u32 sh = bucket_shift((u64)tmax - tmin + 1);
            unsigned short *bs = reinterpret_cast<unsigned short *>(lds + tlen);
            for (u32 b = threadIdx.x; b <= BUCKETS; b += blockDim.x) {
                const u64 key = (u64)tmin + ((u64)b << sh);
                bs[b] = (unsigned short)(key > tmax ? tlen : lower_bound_dev<u32>(lds, 0, tlen, (u32)key));
            }
            __syncthreads();
        } else if (tk.mode == MODE_HASH) {
            // keys stored as value + 1 so that the all-zero LDS reads as empty
            const u32 hk = hash_bits_for(tlen), hmask = (1u << hk) - 1;
            for (u64 i = t0 + threadIdx.x; i < t1; i += blockDim.x) {
                const u32 key = pa[i] + 1;
                u32 h = hash_slot(key - 1, hk);
                while (atomicCAS(&lds[h], 0u, key) != 0u) h = (h + 1) & hmask;
            }
            __syncthreads();
        }
        }
        // the walk, compiled once per LDS form so that each has its own tight loop
        auto walk = [&](auto mode_tag) {
            constexpr int MD = decltype(mode_tag)::value;
            {
                SeedCursor cur;
                const u32 pinv = tk.pinv;
                u32 xinv = 0;
                u64 xinv_c = ~0ull;
                const u32 bsh = MD == MODE_BUCKET ? bucket_shift((u64)tmax - tmin + 1) : 0u;
                const unsigned short *bst = reinterpret_cast<const unsigned short *>(lds + tlen);
                auto member = [&](u32 y) -> bool {
                    if (MD == MODE_BITMAP) {
                        const u32 v = y - tmin;
                        return y >= tmin && y <= tmax && ((lds[v >> 5] >> (v & 31)) & 1u);
                    } else if (MD == MODE_SPLIT) {
                        if (y > tmax) return false;
                        if (y >= wlo) {
                            const u32 v = y - wlo;
                            return (lds[v >> 5] >> (v & 31)) & 1u;
                        }
                        if (low_lds) {
                            const u32 nl = (u32)(ts - t0);
                            const u64 j = lower_bound_dev<u32>(low, 0, nl, y);
                            return j < nl && low[j] == y;
                        }
                        const u64 j = lower_bound_dev<u32>(pa, t0, ts, y);
                        return j < ts && pa[j] == y;
                    } else if (MD == MODE_BUCKET) {
                        if (y < tmin || y > tmax) return false;
                        const u32 b = (y - tmin) >> bsh;
                        const u32 lo = bst[b], hi = bst[b + 1];
                        const u64 j = lower_bound_dev<u32>(lds, lo, hi, y);
                        return j < hi && lds[j] == y;
                    } else if (MD == MODE_ARRAY) {
                        const u64 j = lower_bound_dev<u32>(lds, 0, tlen, y);
                        return j < tlen && lds[j] == y;
                    } else if (MD == MODE_HASH) {
                        const u32 hk = hash_bits_for(tlen), hmask = (1u << hk) - 1;
                        u32 h = hash_slot(y, hk);
                        for (;;) {  // ends: the table is at most half full
                            const u32 v = lds[h];
                            if (v == y + 1) return true;
                            if (v == 0u) return false;
                            h = (h + 1) & hmask;
                        }
                    } else if (MD == MODE_REVERSE) {
                        const u64 *ro = Reverse<ALGO>::off(g);
                        const u32 *ra = Reverse<ALGO>::adj(g);
                        const u64 r0 = ro[y], r1 = ro[y + 1];
                        const u64 j = lower_bound_dev<u32>(ra, r0, r1, p);
                        return j < r1 && ra[j] == p;
                    }
                    const u64 j = lower_bound_dev<u32>(pa, t0, t1, y);
                    return j < t1 && pa[j] == y;
                };
                // membership of UN elements at once (interleaved where it is a search)
                auto member_all = [&](const u32 (&y)[UN], bool (&h)[UN]) {
                    if (MD == MODE_SPLIT) {
                        // the entries below the bitmap's window: interleaved searches,
                        // skipped when no lane has such an element (the usual case)
                        // (unsigned differences: one compare tests each range)
                        const u32 lspan = wlo - tmin, span = tmax - wlo;
                        bool below = false;
    #pragma unroll
                        for (int j = 0; j < UN; j++) below |= (y[j] - tmin) < lspan;
                        const bool any_below = __ballot(below) != 0;
                        stat_add(ST_GROUPS, 1);
                        if (any_below) {
                            stat_add(ST_BELOW_GROUPS, 1);
                            u32 nb = 0;
    #pragma unroll
                            for (int j = 0; j < UN; j++) nb += (u32)__popcll(__ballot((y[j] - tmin) < lspan));
                            stat_add(ST_BELOW, nb);
                            if (!low_lds) stat_add(ST_BELOW_GLOB, nb);
                            // (32-bit indices: adjacency arrays hold fewer than 2^32 entries)
                            u32 lo[UN], hi[UN];
                            const u32 top = low_lds ? (u32)(ts - t0) : lsamp;
    #pragma unroll
                            for (int j = 0; j < UN; j++) {
                                lo[j] = 0u;
                                hi[j] = (y[j] - tmin) < lspan ? top : 0u;
                            }
                            if (low_lds) {
                                member_multi_var32(low, lo, hi, y, h);
                            } else {
                                // the sample at or below y, then its stride of the list
                                u32 b[UN];
                                bound_multi_var32(low, lo, hi, y, b);
    #pragma unroll
                                for (int j = 0; j < UN; j++) {
                                    const bool in = hi[j] != 0u;
                                    lo[j] = in ? (u32)t0 + b[j] * lstride : 0u;
                                    const u32 e = lo[j] + lstride;
                                    hi[j] = in ? (e < (u32)ts ? e : (u32)ts) : 0u;
                                }
                                member_multi_var32(pa, lo, hi, y, h);
                            }
                        } else {
    #pragma unroll
                            for (int j = 0; j < UN; j++) h[j] = false;
                        }
                        // the bitmap part, branch-free: every word is read (index
                        // 0 outside the window) so that the UN reads overlap
                        u32 w[UN], v[UN];
                        bool in[UN];
    #pragma unroll
                        for (int j = 0; j < UN; j++) {
                            const u32 d = y[j] - wlo;
                            in[j] = d <= span;
                            v[j] = in[j] ? d : 0u;
                            w[j] = lds[v[j] >> 5];
                        }
    #pragma unroll
                        for (int j = 0; j < UN; j++) h[j] = in[j] ? (bool)((w[j] >> (v[j] & 31)) & 1u) : h[j];
                    } else if (MD == MODE_BITMAP) {
                        // branch-free: the index is clamped into the bitmap and the
                        // word always read, so that the UN reads overlap; an
                        // element outside [tmin, tmax] is rejected by the range test
                        const u32 span = tmax - tmin;
                        u32 w[UN], v[UN];
    #pragma unroll
                        for (int j = 0; j < UN; j++) {
                            const u32 d = y[j] - tmin;
                            v[j] = d < (u32)(LDS_BITS - 1) ? d : (u32)(LDS_BITS - 1);
                            w[j] = lds[v[j] >> 5];
                        }
    #pragma unroll
                        for (int j = 0; j < UN; j++) h[j] = ((y[j] - tmin) <= span) & ((w[j] >> (v[j] & 31)) & 1u);
                    } else if (MD == MODE_BUCKET) {
                        u64 lo[UN], hi[UN];
    #pragma unroll
                        for (int j = 0; j < UN; j++) {
                            const bool in = y[j] >= tmin && y[j] <= tmax;
                            const u32 b = in ? (y[j] - tmin) >> bsh : 0u;
                            lo[j] = in ? bst[b] : 0u;
                            hi[j] = in ? bst[b + 1] : 0u;
                        }
                        member_multi_var(lds, lo, hi, y, h);
                    } else if (MD == MODE_ARRAY) {
                        member_multi(lds, 0, tlen, y, h);
                    } else if (MD == MODE_GLOBAL) {
                        member_multi(pa, t0, t1, y, h);
                    } else {
    #pragma unroll
                        for (int j = 0; j < UN; j++) h[j] = member(y[j]);
                    }
                };
                // Long windows (at least UN chunks inside one seed) come from
                // the plan's window searches, never from a list taken whole
                // (plan_full < UN * WAVE), so every element lies in the seed's
                // candidate range and hence in [tmin, tmax]: the bitmap form
                // needs no range test.
                auto member_long = [&](const u32 (&y)[UN], bool (&h)[UN]) {
                    if (MD == MODE_BITMAP) {
                        u32 w[UN];
    #pragma unroll
                        for (int j = 0; j < UN; j++) w[j] = lds[(y[j] - tmin) >> 5];
    #pragma unroll
                        for (int j = 0; j < UN; j++) h[j] = (w[j] >> ((y[j] - tmin) & 31)) & 1u;
                    } else {
                        member_all(y, h);
                    }
                };
                // Listed triangles: the hits of every group are packed into
                // this wavefront's LDS staging area (consecutive slots, kept
                // across groups), and each time 64 are waiting they are
                // finished together: the id lookup, canonical order, digest
                // and store then run on full wavefronts whatever the hit rate.
                u32 staged = 0;  // hits waiting in the staging area (wave-uniform)
                auto flush = [&](u32 k) {
                    wave_lds_fence();
                    const bool v = (u32)lane < k;
                    u32 ta = 0, tb = 0, tc = 0;
                    if (v) {
                        const uint2 e = stage[lane];
                        ta = pinv; tb = e.x; tc = g.inv[e.y];
                        canon3(ta, tb, tc);
                        cnt += 1;
                        hsh += tri_digest(ta, tb, tc);
                    }
                    wave_lds_fence();
                    em.push(v, ta, tb, tc, o);
                };
                auto report = [&](const u32 (&y)[UN], const bool (&h)[UN], const u32 (&xv)[UN]) {
                    u64 bal[UN];
                    u32 q[UN], tot = 0;
                    const u64 lt = lanemask_lt();
    #pragma unroll
                    for (int j = 0; j < UN; j++) {
                        bal[j] = __ballot(h[j]);
                        q[j] = tot + (u32)__popcll(bal[j] & lt);  // position among the group's hits
                        tot += (u32)__popcll(bal[j]);
                    }
                    for (u32 r0 = 0; r0 < tot;) {
                        const u32 room = (u32)WAVE - staged;
    #pragma unroll
                        for (int j = 0; j < UN; j++) {
                            if (h[j] && q[j] - r0 < room) stage[staged + (q[j] - r0)] = make_uint2(xv[j], y[j]);
                        }
                        const u32 take = tot - r0 < room ? tot - r0 : room;
                        staged += take;
                        r0 += take;
                        if (staged == (u32)WAVE) {
                            flush(WAVE);
                            staged = 0;
                        }
                    }
                };
                // the 64-seed window starting at c0: prefixes, scan starts, endpoint ids
                auto fetch_window = [&](u64 c0, u64 &P, u64 &A, u32 &X, u64 &pend) {
                    const u64 ci = c0 + lane;
                    const bool inw = ci < tk.ce;
                    P = inw ? cpre[ci] : ~0ull;
                    A = inw ? cabs[ci] : 0ull;
                    X = inw ? cxinv[ci] : 0u;
                    pend = uni64((c0 + WAVE <= tk.ce) ? cpre[c0 + WAVE] : ~0ull);
                };
                u64 pf_c = ~0ull, pf_P = 0, pf_A = 0, pf_pend = 0;  // prefetched window (pf_c: its first seed)
                u32 pf_X = 0;
                // The window in use: seeds [wc, wc + 64) (wc wave-uniform, ~0: none),
                // kept while it still holds the next group's items, so that runs of
                // short windows cost one fetch of 64 seeds' geometry, not one per group.
                u64 wc = ~0ull, WP = 0, WA = 0, Wpend = 0;
                u32 WX = 0;
                // the wavefront's own sub-range, then shared ones while any is left
                for (u32 sub = (u32)wid;;) {
                u64 sa, sb;
                sub_range(tk.a, tk.b, sub, sa, sb);
                const u64 wb = sa > a ? sa : a, we = sb < b ? sb : b;  // (clipped to a chunk slice)
                if (wb < we) {
                if (use_splits && wb == sa) cur = SeedCursor(cpre, tk.ce, tk.cb + tg.ss[sub]);
                else cur = SeedCursor(cpre, tk.cb, tk.ce, wb);
                xinv_c = ~0ull;
                wc = ~0ull;
                pf_c = ~0ull;
                u64 kb = wb;
                while (kb < we) {
                    if ((MD == MODE_BITMAP || MD == MODE_SPLIT) && cur.end >= kb + HG * UN * WAVE &&
                        kb + HG * UN * WAVE <= we) {
                        // HG groups of UN full chunks inside one seed window: all
                        // loads in flight before the first test (one LDS read each)
                        if (xinv_c != cur.c_lo) {  // once per seed, before the element loads
                            xinv = cxinv[cur.c_lo];
                            xinv_c = cur.c_lo;
                        }
                        const u64 sab = cabs[cur.c_lo] + (kb - cur.base) + lane;
                        u32 y[HG][UN], xv[UN];
                        bool h[UN];
#pragma unroll
                        for (int q = 0; q < HG; q++)
#pragma unroll
                            for (int j = 0; j < UN; j++) y[q][j] = SA[sab + (u64)(q * UN + j) * WAVE];
#pragma unroll
                        for (int j = 0; j < UN; j++) xv[j] = xinv;
#pragma unroll
                        for (int q = 0; q < HG; q++) {
                            member_long(y[q], h);
                            report(y[q], h, xv);
                        }
                        kb += HG * UN * WAVE;
                        stat_add(ST_LONG, HG * UN * WAVE);
                        cur.advance(kb, cur.c_lo);
                        continue;
                    }
                    if (cur.end >= kb + UN * WAVE && kb + UN * WAVE <= we) {
                        // UN full chunks inside one seed window
                        if (xinv_c != cur.c_lo) {  // once per seed, before the element loads
                            xinv = cxinv[cur.c_lo];
                            xinv_c = cur.c_lo;
                        }
                        const u64 sab = cabs[cur.c_lo] + (kb - cur.base) + lane;
                        u32 y[UN], xv[UN];
                        bool h[UN];
    #pragma unroll
                        for (int j = 0; j < UN; j++) y[j] = SA[sab + (u64)j * WAVE];
    #pragma unroll
                        for (int j = 0; j < UN; j++) xv[j] = xinv;
                        member_long(y, h);
                        report(y, h, xv);
                        kb += UN * WAVE;
                        stat_add(ST_LONG, UN * WAVE);
                        cur.advance(kb, cur.c_lo);
                        continue;
                    }
                    if (kb + WAVE <= we) {
                        // short windows: the items of up to UN chunks from kb on, spread
                        // over the 64 seeds of the window, with the seeds' prefixes, scan
                        // starts and endpoint ids held one per lane
                        const bool have = TL_KEEP_WINDOW && wc != ~0ull && cur.c_lo >= wc && cur.c_lo < wc + WAVE &&
                                          (Wpend >= kb + UN * WAVE || Wpend >= we);
                        if (!have) {
                            if (pf_c == cur.c_lo) {
                                WP = pf_P; WA = pf_A; WX = pf_X; Wpend = pf_pend;
                            } else {
                                fetch_window(cur.c_lo, WP, WA, WX, Wpend);
                            }
                            wc = cur.c_lo;
                        }
                        const int s0 = (int)(cur.c_lo - wc);  // lane of the seed of item kb
                        // items the window holds within this wavefront's range; at
                        // least one full chunk, else the one-chunk path below (SPLIT
                        // takes only full groups: partial ones measured slower there)
                        const u64 lim = Wpend < we ? Wpend : we;
                        if (lim >= kb + (MD == MODE_SPLIT ? UN * WAVE : WAVE)) {
                            const bool full = lim >= kb + UN * WAVE;  // wave-uniform
                            // item kb + i of seed c: scan index E[c] + i (mod 2^32; m < 2^32)
                            const u32 E = (u32)(WA - WP + kb);
                            const u32 X = WX;
                            // the cursor to item kn (< we), whose seed is the window's lane
                            // lo_last or the next one; the next window is fetched here when
                            // the group after needs it, so that this group's element loads,
                            // issued next, cover its wait
                            auto step_cursor = [&](int lo_last, u64 kn) {
                                const u64 pn = (lo_last + 1 < WAVE) ? lane_u64(WP, lo_last + 1) : Wpend;
                                const int ln = lo_last + (pn <= kn ? 1 : 0);
                                const u64 c = wc + (u64)ln;
                                if (ln < WAVE) {  // the cursor from the window's registers
                                    cur.c_lo = c;
                                    cur.base = lane_u64(WP, ln);
                                    cur.end = ln + 1 < WAVE ? lane_u64(WP, ln + 1) : Wpend;
                                } else {
                                    cur.reset(c);
                                }
                                if ((!TL_KEEP_WINDOW || !(Wpend >= kn + UN * WAVE || Wpend >= we)) && pf_c != c) {
                                    fetch_window(c, pf_P, pf_A, pf_X, pf_pend);
                                    pf_c = c;
                                }
                            };
                            int lo[UN];
                            const int lo_last = locate_short_at(WP, kb, s0, flag, lo);
                            const u64 kn = full ? kb + UN * WAVE : lim;
                            if (kn < we) step_cursor(lo_last, kn);
                            u32 y[UN], xv[UN];
                            bool h[UN], act[UN];
#pragma unroll
                            for (int j = 0; j < UN; j++) {
                                // the shuffles run on every lane (a lane cannot read a
                                // value from a lane that skips the shuffle)
                                const u32 ej = (u32)__shfl(E, lo[j], WAVE);
                                xv[j] = __shfl(X, lo[j], WAVE);
                                // items at or past lim belong to no seed of the window:
                                // such lanes test tmax (a valid rank for every form's
                                // lookup, REVERSE's offsets included, and inside SPLIT's
                                // bitmap, so it starts no global search) and drop the result
                                act[j] = full || kb + (u64)(j * WAVE + lane) < lim;
                                y[j] = act[j] ? SA[ej + (u32)(j * WAVE + lane)] : tmax;
                            }
                            if ((MD == MODE_BITMAP || MD == MODE_SPLIT) && TL_SG > 1 && full) {
                                // up to SG - 1 more full groups from the same window: their
                                // loads are issued before the first group's tests, so all
                                // are in flight together (a group the long path would take,
                                // a seed with at least HG UN chunks left, ends the run)
                                u32 ys[TL_SG > 1 ? TL_SG - 1 : 1][UN], xs[TL_SG > 1 ? TL_SG - 1 : 1][UN];
                                int ng = 0;  // wave-uniform
                                u64 kend = kn;
#pragma unroll
                                for (int g2 = 0; g2 < TL_SG - 1; g2++) {
                                    if (ng == g2 && kend + UN * WAVE <= we && Wpend >= kend + UN * WAVE &&
                                        cur.c_lo - wc < (u64)WAVE && cur.end < kend + HG * UN * WAVE) {
                                        const int s1 = (int)(cur.c_lo - wc);
                                        const u32 E1 = (u32)(WA - WP + kend);
                                        int lo1[UN];
                                        const int lo_last1 = locate_short_at(WP, kend, s1, flag, lo1);
                                        const u64 kn1 = kend + UN * WAVE;
                                        if (kn1 < we) step_cursor(lo_last1, kn1);
#pragma unroll
                                        for (int j = 0; j < UN; j++) {
                                            const u32 ej = (u32)__shfl(E1, lo1[j], WAVE);
                                            xs[g2][j] = __shfl(X, lo1[j], WAVE);
                                            ys[g2][j] = SA[ej + (u32)(j * WAVE + lane)];
                                        }
                                        kend = kn1;
                                        ng++;
                                    }
                                }
                                if (ng > 0) {
                                    member_all(y, h);
                                    report(y, h, xv);
#pragma unroll
                                    for (int g2 = 0; g2 < TL_SG - 1; g2++) {
                                        if (g2 < ng) {
                                            member_all(ys[g2], h);
                                            report(ys[g2], h, xs[g2]);
                                        }
                                    }
                                    stat_add(ST_SHORT, kend - kb);
                                    kb = kend;
                                    continue;
                                }
                            }
                            member_all(y, h);
#pragma unroll
                            for (int j = 0; j < UN; j++) h[j] = h[j] && act[j];
                            report(y, h, xv);
                            stat_add(ST_SHORT, kn - kb);
                            kb = kn;
                            continue;
                        }
                    }
                    const u64 k = kb + lane;
                    const bool act = k < we;
                    u64 rel;
                    const u64 c = cur.locate(kb, k, rel);
                    bool hit = false;
                    u32 xa = 0, xb = 0, xc = 0;
                    if (act) {
                        const u32 y = SA[cabs[c] + rel];
                        hit = member(y);
                        if (hit) {
                            xa = pinv; xb = cxinv[c]; xc = g.inv[y];
                            canon3(xa, xb, xc);
                            cnt += 1;
                            hsh += tri_digest(xa, xb, xc);
                        }
                    }
                    em.push(hit, xa, xb, xc, o);
                    stat_add(ST_SINGLE, (we - kb < (u64)WAVE) ? we - kb : (u64)WAVE);
                    kb += WAVE;
                    cur.advance(kb, c);
                }
                }
                u32 nx = 0;
                if (lane == 0) nx = atomicAdd(&next_sub, 1u);
                sub = (u32)__builtin_amdgcn_readfirstlane((int)nx);
                if (sub >= NSUB) break;
                }
                if (staged) flush(staged);
            }
        };
        if constexpr (LEAN) {
            if (tk.mode == MODE_BITMAP) walk(std::integral_constant<int, MODE_BITMAP>{});
            else walk(std::integral_constant<int, MODE_SPLIT>{});
        } else {
            switch (tk.mode) {
                case MODE_BITMAP: walk(std::integral_constant<int, MODE_BITMAP>{}); break;
                case MODE_ARRAY: walk(std::integral_constant<int, MODE_ARRAY>{}); break;
                case MODE_GLOBAL: walk(std::integral_constant<int, MODE_GLOBAL>{}); break;
                case MODE_REVERSE: walk(std::integral_constant<int, MODE_REVERSE>{}); break;
                case MODE_HASH: walk(std::integral_constant<int, MODE_HASH>{}); break;
                case MODE_BUCKET: walk(std::integral_constant<int, MODE_BUCKET>{}); break;
                default: walk(std::integral_constant<int, MODE_SPLIT>{}); break;
            }
        }
        stat_flush();
    }
    em.finish(o);
    {
        const u64 c8 = wave_sum_u64(cnt);
        if (lane_id() == 0 && c8) atomicAdd((unsigned long long *)&o.acc[8], (unsigned long long)c8);
    }
    flush_counts(cnt, hsh, o.acc);
    __syncthreads();
    if (threadIdx.x < ST_N && wstat[threadIdx.x])
        atomicAdd((unsigned long long *)&o.acc[ACC_PATHS + threadIdx.x], (unsigned long long)wstat[threadIdx.x]);
}

// Heavy tasks are ordered by item range: start the queue at the first task
// that reaches past k0 (chunked listings probe one item slice at a time).
__global__ void k_task_first(const Task *tasks, u64 ntasks, u64 k0, u64 *queue) {
    u64 lo = 0, hi = ntasks;
    while (lo < hi) {
        const u64 mid = lo + (hi - lo) / 2;
        if (tasks[mid].b <= k0) lo = mid + 1; else hi = mid;
    }
    *queue = lo;
}

// Copies spilled (or misplaced) triangles into holes: one move per block.

__global__ void k_apply_moves(const Move *mv, u64 nmv, u32 *tri, u64 cap, const u32 *spill) {
    for (u64 i = blockIdx.x; i < nmv; i += gridDim.x) {
        const Move m = mv[i];
        for (u64 w = threadIdx.x; w < 3 * m.len; w += blockDim.x) {
            const u64 sp = 3 * m.src + w;
            const u32 v = (sp < 3 * cap) ? tri[sp] : spill[sp - 3 * cap];
            tri[3 * m.dst + w] = v;
        }
    }
}

__global__ __launch_bounds__(PB) void k_cost(const u64 *off_f, const u64 *off_b, u32 n, int algo, u64 *out) {
    __shared__ u64 lds[PB / WAVE];
    u64 v = 0;
    GRID_STRIDE(r, n) {
        u64 dp = off_f[r + 1] - off_f[r], dm = off_b[r + 1] - off_b[r];
        v += algo == 0 ? dp * dp : (algo == 1 ? dp * dm : dm * dm);
    }
    u64 tot = block_sum_u64<PB>(v, lds);
    if (threadIdx.x == 0 && tot) atomicAdd((unsigned long long *)out, (unsigned long long)tot);
}

u64 g_chunk_triangles = 1ull << 24;

// Chunked emission: a slice's length in items stays within this many chunks.
constexpr u64 CHUNK_GROWTH_MAX = 64;

// Items for the next slice: enough for K triangles at margin_pct percent of
// the rate the last slice saw (got triangles over `items`), at most `cap`,
// at least K (a slice of K items cannot overflow a chunk of K triangles).
inline u64 chunk_slice_items(u64 K, u64 got, u64 items, u64 cap, u64 margin_pct) {
    u64 L = cap;
    if (got) {
        const double want = (double)K * (double)items * 100.0 / ((double)margin_pct * (double)got);
        if (want < (double)L) L = (u64)want;
    }
    return L < K ? K : L;
}

GView view_of(const tl_csr *g) {
    return GView{g->off_f, g->off_b, g->adj_f, g->adj_b, g->row_f, g->row_b, g->inv, g->m, g->twin_b};
}

// Everything a listing's probe phase needs, produced by the plan.
struct Plan {
    DevBuf cabs, cxinv, cpre, tasks;
    DevBuf ctlo, cthi, cpinv;  // light seeds only
    u64 ncomp = 0;    // compacted seeds
    u64 nlight = 0;   // ... of which light
    u64 w_light = 0;  // light items [0, w_light)
    u64 w_total = 0;  // all items
    u64 ntasks = 0;
    u64 work = 0;     // the paper's work over the listed pivots
    bool lean = true; // every heavy task has the BITMAP or SPLIT form
};

// Largest grids the probe kernels are launched with; they bound the number
// of wavefronts, hence of holes, per launch.
inline u64 light_max_blocks() { return (u64)tl_num_cus() * tuning().light_blocks_per_cu; }
inline u64 heavy_max_blocks() { return (u64)tl_num_cus() * tuning().heavy_blocks_per_cu; }

template <int ALGO>
// max_task: items per heavy task at most (0: no limit).  A listing probed in
// item slices keeps tasks well below a slice, so that every slice has work
// for all workgroups.
void make_plan(const GView &v, u32 n, u32 plo, u32 phi, u64 max_task, u64 *d_acc, hipStream_t s, Plan &P) {
    const u64 m = v.m;
    const unsigned gm = grid_for(m, PB, (unsigned)tl_num_cus() * 16);
    const unsigned gn = grid_for(n, PB, (unsigned)tl_num_cus() * 16);
    DevBuf len(m * sizeof(u32), s), sabs(m * sizeof(u64), s), wp((u64)n * sizeof(u64), s),
        wpw((u64)n * sizeof(u64), s);
    TL_HIP(hipMemsetAsync(wp.p, 0, (u64)n * sizeof(u64), s));
    TL_HIP(hipMemsetAsync(wpw.p, 0, (u64)n * sizeof(u64), s));
    const u32 full_max = (u32)std::min<u64>(tuning().plan_full, UN * WAVE - 1);  // see member_long
    hipLaunchKernelGGL((k_plan<ALGO>), dim3(gm), dim3(PB), 0, s, v, plo, phi, full_max, len.as<u32>(),
                       sabs.as<u64>(), wp.as<u64>(), wpw.as<u64>(), d_acc);
    TL_HIP(hipGetLastError());
    DevBuf mode((u64)n * sizeof(u32), s), ntask((u64)n * sizeof(u32), s), slice((u64)n * sizeof(u64), s);
    const Tuning &tu = tuning();
    hipLaunchKernelGGL((k_pivot_class<ALGO>), dim3(gn), dim3(PB), 0, s, v, n, wp.as<u64>(), wpw.as<u64>(),
                       mode.as<u32>(),
                       ntask.as<u32>(), slice.as<u64>(), tu.heavy_min, tu.slice_min, tu.slice_mult, max_task,
                       tu.task_div ? tu.task_div * heavy_max_blocks() : 0, tu.reverse, tu.hash, tu.bucket, tu.split,
                       tu.force_mode, d_acc);
    TL_HIP(hipGetLastError());
    DevBuf flags(m * sizeof(u64), s), pos((m + 1) * sizeof(u64), s);
    hipLaunchKernelGGL((k_seed_class<ALGO>), dim3(gm), dim3(PB), 0, s, v, len.as<u32>(), mode.as<u32>(),
                       flags.as<u64>());
    TL_HIP(hipGetLastError());
    scan_u64_to_u64(flags.as<u64>(), pos.as<u64>(), m, s);
    P.cabs = DevBuf(m * sizeof(u64), s);
    u32 *clen = (u32 *)flags.p;  // the flags are consumed by the scan: reuse them as lengths
    TL_HIP(hipMemsetAsync(clen, 0, m * sizeof(u32), s));
    P.cxinv = DevBuf(m * sizeof(u32), s);
    P.ctlo = DevBuf(m * sizeof(u32), s);
    P.cthi = DevBuf(m * sizeof(u32), s);
    P.cpinv = DevBuf(m * sizeof(u32), s);
    hipLaunchKernelGGL((k_compact<ALGO>), dim3(gm), dim3(PB), 0, s, v, len.as<u32>(), sabs.as<u64>(), pos.as<u64>(),
                       P.cabs.as<u64>(), P.cxinv.as<u32>(), clen, P.ctlo.as<u32>(),
                       P.cthi.as<u32>(), P.cpinv.as<u32>());
    TL_HIP(hipGetLastError());
    P.cpre = DevBuf((m + 1) * sizeof(u64), s);
    scan_u32_to_u64(clen, P.cpre.as<u64>(), m, s);
    DevBuf tpos(((u64)n + 1) * sizeof(u64), s);
    scan_u32_to_u64(ntask.as<u32>(), tpos.as<u64>(), n, s);
    // every total the host needs, in one round trip
    DevBuf tot(6 * sizeof(u64), s);
    hipLaunchKernelGGL(k_plan_totals, dim3(1), dim3(WAVE), 0, s, pos.as<u64>(), m, tpos.as<u64>(), n,
                       P.cpre.as<u64>(), d_acc, tot.as<u64>());
    TL_HIP(hipGetLastError());
    u64 h_t[6] = {0, 0, 0, 0, 0, 0};
    d2h_sync(s, {{h_t, tot.p, sizeof h_t}});
    const u64 h_pos = h_t[0], h_nt = h_t[1];
    const u64 nl = h_pos & 0xffffffffull, nh = h_pos >> 32;
    P.ncomp = nl + nh;
    P.nlight = nl;
    P.ntasks = h_nt;
    P.w_light = h_t[2];
    P.w_total = h_t[3];
    P.work = h_t[4];
    P.lean = h_t[5] == 0;
    if (h_nt) {
        P.tasks = DevBuf(h_nt * sizeof(Task), s);
        hipLaunchKernelGGL((k_make_tasks<ALGO>), dim3(gn), dim3(PB), 0, s, v, n, mode.as<u32>(), ntask.as<u32>(),
                           slice.as<u64>(), tpos.as<u64>(), pos.as<u64>(), P.cpre.as<u64>(), m,
                           P.tasks.as<Task>());
        TL_HIP(hipGetLastError());
        if (tuning().splits) {
            hipLaunchKernelGGL(k_task_splits, dim3(grid_for(h_nt * NSUB, PB, (unsigned)tl_num_cus() * 16)), dim3(PB), 0,
                               s, P.tasks.as<Task>(), h_nt, P.cpre.as<u64>());
            TL_HIP(hipGetLastError());
        }
    }
}

inline u64 max_holes_per_probe() { return light_max_blocks() * (PB / WAVE) + heavy_max_blocks() * (HB / WAVE); }

inline LightSeeds light_seeds(const Plan &P) {
    return LightSeeds{P.cpre.as<u64>(), P.cabs.as<u64>(), P.cxinv.as<u32>(), P.ctlo.as<u32>(), P.cthi.as<u32>(),
                      P.cpinv.as<u32>()};
}

template <int ALGO>
void launch_probe(const GView &v, const Plan &P, u64 k0, u64 k1, bool emit, const Out &o, hipStream_t s) {
    // light part
    const u64 l0 = k0, l1 = k1 < P.w_light ? k1 : P.w_light;
    if (l0 < l1) {
        PhaseTimer tlight(TL_PHASE_PROBE_LIGHT, s);
        const u64 wi = tuning().light_wave_items;
        const u64 waves_needed = (l1 - l0 + wi - 1) / wi;
        u64 blocks = (waves_needed + (PB / WAVE) - 1) / (PB / WAVE);
        if (blocks > light_max_blocks()) blocks = light_max_blocks();
        if (blocks < 1) blocks = 1;
        const LightSeeds L = light_seeds(P);
        if (emit)
            hipLaunchKernelGGL((k_probe_light<ALGO, true>), dim3((unsigned)blocks), dim3(PB), 0, s, v, L.cpre, L.cabs,
                               L.cxinv, L.ctlo, L.cthi, L.cpinv, P.nlight, l0, l1, o);
        else
            hipLaunchKernelGGL((k_probe_light<ALGO, false>), dim3((unsigned)blocks), dim3(PB), 0, s, v, L.cpre, L.cabs,
                               L.cxinv, L.ctlo, L.cthi, L.cpinv, P.nlight, l0, l1, o);
        TL_HIP(hipGetLastError());
    }
    // heavy part
    const u64 h0 = k0 > P.w_light ? k0 : P.w_light, h1 = k1;
    if (h0 < h1 && P.ntasks) {
        PhaseTimer theavy(TL_PHASE_PROBE_HEAVY, s);
        if (tuning().queue) {
            hipLaunchKernelGGL(k_task_first, dim3(1), dim3(1), 0, s, P.tasks.as<Task>(), P.ntasks, h0, o.acc + 5);
            TL_HIP(hipGetLastError());
        }
        u64 blocks = P.ntasks;
        if (blocks > heavy_max_blocks()) blocks = heavy_max_blocks();
        auto go = [&](auto emit_tag, auto lean_tag) {
            hipLaunchKernelGGL((k_probe_heavy<ALGO, decltype(emit_tag)::value, decltype(lean_tag)::value>),
                               dim3((unsigned)blocks), dim3(HB), HEAVY_LDS_BYTES, s, v, P.tasks.as<Task>(), P.ntasks,
                               P.cabs.as<u64>(), P.cxinv.as<u32>(), P.cpre.as<u64>(), h0, h1, o,
                               (int)tuning().queue, (int)tuning().splits, (int)tuning().keep_staged);
        };
        using T_ = std::true_type;
        using F_ = std::false_type;
        const bool lean = P.lean && tuning().lean;
        if (emit) {
            if (lean) go(T_{}, T_{});
            else go(T_{}, F_{});
        } else {
            if (lean) go(F_{}, T_{});
            else go(F_{}, F_{});
        }
        TL_HIP(hipGetLastError());
    }
}

// After a probe with emission: count = triangles listed, reserved = cursor.
// Triangles occupy [0, reserved) minus the holes; move the ones at or above
// count into the holes below count so that the output is exactly [0, count).
void fix_holes(const Out &o, u64 count, u64 reserved, u64 nholes, hipStream_t s) {
    if (nholes == 0 || reserved == count) return;
    TL_REQUIRE(nholes <= o.hole_cap, TL_EHIP, "internal: hole list overflow");
    std::vector<Hole> holes(nholes);
    d2h_sync(s, {{holes.data(), o.holes, nholes * sizeof(Hole)}});
    std::vector<Move> mv;
    try {
        mv = plan_hole_moves(std::move(holes), count, reserved);
    } catch (const std::runtime_error &e) {
        throw TlError{TL_EHIP, std::string("internal: ") + e.what()};
    }
    if (mv.empty()) return;
    DevBuf dmv(mv.size() * sizeof(Move), s);
    h2d_sync(dmv.p, mv.data(), mv.size() * sizeof(Move), s);
    const unsigned blocks = (unsigned)std::min<u64>(mv.size(), (u64)tl_num_cus() * 4);
    hipLaunchKernelGGL(k_apply_moves, dim3(blocks), dim3(256), 0, s, dmv.as<Move>(), (u64)mv.size(), o.tri, o.cap,
                       o.spill);
    TL_HIP(hipGetLastError());
    TL_HIP(hipStreamSynchronize(s));
}

Tuning &tuning() {
    static Tuning t = [] {
        Tuning d;
        auto env = [](const char *k, u64 &v) {
            const char *e = getenv(k);
            if (e && *e) v = strtoull(e, nullptr, 10);
        };
        env("TL_TUNE_HEAVY_MIN", d.heavy_min);
        env("TL_TUNE_SLICE_MIN", d.slice_min);
        env("TL_TUNE_SLICE_MULT", d.slice_mult);
        env("TL_TUNE_TASK_DIV", d.task_div);
        env("TL_TUNE_KEEP_STAGED", d.keep_staged);
        env("TL_TUNE_LEAN", d.lean);
        if (d.task_div > 1024) d.task_div = 1024;
        env("TL_TUNE_HEAVY_BLOCKS_PER_CU", d.heavy_blocks_per_cu);
        env("TL_TUNE_QUEUE", d.queue);
        env("TL_TUNE_SPLITS", d.splits);
        env("TL_TUNE_LIGHT_BLOCKS_PER_CU", d.light_blocks_per_cu);
        env("TL_TUNE_LIGHT_WAVE_ITEMS", d.light_wave_items);
        if (d.light_wave_items < (u64)WAVE) d.light_wave_items = WAVE;
        env("TL_TUNE_REVERSE", d.reverse);
        env("TL_TUNE_HASH", d.hash);
        env("TL_TUNE_BUCKET", d.bucket);
        env("TL_TUNE_SPLIT", d.split);
        env("TL_TUNE_ORIENT_SORT", d.orient_sort);
        env("TL_TUNE_FORCE_MODE", d.force_mode);
        env("TL_TUNE_PLAN_FULL", d.plan_full);
        if (d.plan_full >= (u64)(UN * WAVE)) d.plan_full = UN * WAVE - 1;
        env("TL_TUNE_CHUNK_GROWTH", d.chunk_growth);
        env("TL_TUNE_CHUNK_MARGIN", d.chunk_margin);
        env("TL_TUNE_CHUNK_TASK_DIV", d.chunk_task_div);
        env("TL_TUNE_CHUNK_ROOM", d.chunk_room);
        d.chunk_growth = std::min<u64>(std::max<u64>(d.chunk_growth, 1), 64);
        d.chunk_margin = std::min<u64>(std::max<u64>(d.chunk_margin, 100), 1000);
        d.chunk_task_div = std::min<u64>(std::max<u64>(d.chunk_task_div, 1), 64);
        return d;
    }();
    return t;
}

bool debug_enabled() {
    static const bool on = [] {
        const char *e = getenv("TL_DEBUG");
        return e && *e && *e != '0';
    }();
    return on;
}

// Allow the heavy-pivot kernels their full dynamic LDS (once per process).
void prepare_kernels() {
    static std::once_flag once;
    std::call_once(once, [] {
        const void *fns[] = {
            (const void *)k_probe_heavy<0, true, false>, (const void *)k_probe_heavy<0, false, false>,
            (const void *)k_probe_heavy<1, true, false>, (const void *)k_probe_heavy<1, false, false>,
            (const void *)k_probe_heavy<2, true, false>, (const void *)k_probe_heavy<2, false, false>,
            (const void *)k_probe_heavy<0, true, true>,  (const void *)k_probe_heavy<0, false, true>,
            (const void *)k_probe_heavy<1, true, true>,  (const void *)k_probe_heavy<1, false, true>,
            (const void *)k_probe_heavy<2, true, true>,  (const void *)k_probe_heavy<2, false, true>};
        for (const void *f : fns)
            (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, HEAVY_LDS_BYTES);
        (void)hipGetLastError();
    });
}

}  // namespace

u64 list_count_scratch_bytes(u64 n, u64 m) {
    // every block list_impl (count only) and make_plan take from the pool,
    // in 256-byte units, heavy tasks excepted
    auto blk = [](u64 b) { return ((b ? b : 1) + 255) / 256 * 256; };
    const u64 ws_m = blk(scan_workspace_words(m) * sizeof(u64)), ws_n = blk(scan_workspace_words(n) * sizeof(u64));
    u64 t = blk(NACC * sizeof(u64));
    t += blk(m * 4) + blk(m * 8) + 2 * blk(n * 8);            // len, sabs, wp, wpw
    t += blk(n * 4) + blk(n * 4) + blk(n * 8);                // mode, ntask, slice
    t += blk(m * 8) + blk((m + 1) * 8) + (ws_m ? ws_m : 0);   // flags, pos and its scan
    t += blk(m * 8) + blk(m * 4);                             // cabs, cxinv
    t += 3 * blk(m * 4);                                      // ctlo, cthi, cpinv
    t += blk((m + 1) * 8) + (ws_m ? ws_m : 0);                // cpre and its scan
    t += blk((n + 1) * 8) + (ws_n ? ws_n : 0);                // tpos and its scan
    t += blk(6 * sizeof(u64));                                // totals
    return t;
}

u64 chunk_triangles() { return g_chunk_triangles; }
bool orient_by_sort() { return tuning().orient_sort != 0; }

tl_list_stats &last_stats() {
    thread_local tl_list_stats st{};
    return st;
}

int set_tuning(const char *key, u64 value) {
    Tuning &t = tuning();
    const std::string k(key ? key : "");
    if (k.rfind("batch_", 0) == 0) return batch_set_tuning(k, value);
    if (k == "heavy_min" && value >= 1) t.heavy_min = value;
    else if (k == "slice_min" && value >= 64) t.slice_min = value;
    else if (k == "slice_mult" && value >= 1) t.slice_mult = value;
    else if (k == "task_div" && value <= 1024) t.task_div = value;
    else if (k == "heavy_blocks_per_cu" && value >= 1 && value <= 64) t.heavy_blocks_per_cu = value;
    else if (k == "queue" && value <= 1) t.queue = value;
    else if (k == "splits" && value <= 1) t.splits = value;
    else if (k == "keep_staged" && value <= 1) t.keep_staged = value;
    else if (k == "lean" && value <= 1) t.lean = value;
    else if (k == "chunk_room" && value >= 1 && value <= 16) t.chunk_room = value;
    else if (k == "light_blocks_per_cu" && value >= 1 && value <= 64) t.light_blocks_per_cu = value;
    else if (k == "light_wave_items" && value >= (u64)WAVE && value <= (1ull << 30)) t.light_wave_items = value;
    else if (k == "reverse" && value <= 1) t.reverse = value;
    else if (k == "hash" && value <= 1) t.hash = value;
    else if (k == "bucket" && value <= 1) t.bucket = value;
    else if (k == "split" && value <= 2) t.split = value;
    else if (k == "orient_sort" && value <= 1) t.orient_sort = value;
    else if (k == "force_mode" && (value < NMODES || value == 255)) t.force_mode = value;
    else if (k == "plan_full" && value < (u64)(UN * WAVE)) t.plan_full = value;
    else if (k == "chunk_growth" && value >= 1 && value <= 64) t.chunk_growth = value;
    else if (k == "chunk_margin" && value >= 100 && value <= 1000) t.chunk_margin = value;
    else if (k == "chunk_task_div" && value >= 1 && value <= 64) t.chunk_task_div = value;
    else return TL_EINVAL;
    return TL_OK;
}

int get_tuning(const char *key, u64 *value) {
    const Tuning &t = tuning();
    const std::string k(key ? key : "");
    if (k.rfind("batch_", 0) == 0) return batch_get_tuning(k, value);
    if (k == "heavy_min") *value = t.heavy_min;
    else if (k == "slice_min") *value = t.slice_min;
    else if (k == "slice_mult") *value = t.slice_mult;
    else if (k == "task_div") *value = t.task_div;
    else if (k == "heavy_blocks_per_cu") *value = t.heavy_blocks_per_cu;
    else if (k == "queue") *value = t.queue;
    else if (k == "splits") *value = t.splits;
    else if (k == "keep_staged") *value = t.keep_staged;
    else if (k == "lean") *value = t.lean;
    else if (k == "chunk_room") *value = t.chunk_room;
    else if (k == "light_blocks_per_cu") *value = t.light_blocks_per_cu;
    else if (k == "light_wave_items") *value = t.light_wave_items;
    else if (k == "reverse") *value = t.reverse;
    else if (k == "hash") *value = t.hash;
    else if (k == "bucket") *value = t.bucket;
    else if (k == "split") *value = t.split;
    else if (k == "orient_sort") *value = t.orient_sort;
    else if (k == "force_mode") *value = t.force_mode;
    else if (k == "plan_full") *value = t.plan_full;
    else if (k == "chunk_growth") *value = t.chunk_growth;
    else if (k == "chunk_margin") *value = t.chunk_margin;
    else if (k == "chunk_task_div") *value = t.chunk_task_div;
    else return TL_EINVAL;
    return TL_OK;
}
void set_chunk_triangles(u64 k) { g_chunk_triangles = k; }

u64 cost_impl(const tl_csr *g, int algo, hipStream_t s) {
    PhaseTimer timer(TL_PHASE_COST, s);
    DevBuf out(sizeof(u64), s);
    TL_HIP(hipMemsetAsync(out.p, 0, sizeof(u64), s));
    if (g->n) {
        hipLaunchKernelGGL(k_cost, dim3(grid_for(g->n, PB, (unsigned)tl_num_cus() * 8)), dim3(PB), 0, s, g->off_f,
                           g->off_b, g->n, algo, out.as<u64>());
        TL_HIP(hipGetLastError());
    }
    timer.stop();
    u64 h = 0;
    d2h_sync(s, {{&h, out.p, sizeof(u64)}});
    return h;
}

int list_impl(const tl_csr *g, int algo, u32 plo, u32 phi, u32 *tri, u64 cap, tl_chunk_fn cb, void *user,
              hipStream_t s, tl_summary *out) {
    *out = tl_summary{0, 0, 0, 0};
    const u64 m = g->m;
    if (phi > g->n) phi = g->n;
    if (m == 0 || plo >= phi) return TL_OK;
    const GView v = view_of(g);
    prepare_kernels();

    DevBuf acc(NACC * sizeof(u64), s);
    TL_HIP(hipMemsetAsync(acc.p, 0, NACC * sizeof(u64), s));
    u64 *d_acc = acc.as<u64>();

    // ---- plan: windows, heavy/light classes, compaction, work prefix, tasks
    Plan P;
    {
        PhaseTimer plan_timer(TL_PHASE_PLAN, s);
        u64 max_task = 0;
        if (cb && !tri) {
            max_task = g_chunk_triangles * tuning().chunk_room / (tuning().chunk_task_div * heavy_max_blocks());
            if (max_task < 65536) max_task = 65536;
        }
        if (algo == 0) make_plan<0>(v, g->n, plo, phi, max_task, d_acc, s, P);
        else if (algo == 1) make_plan<1>(v, g->n, plo, phi, max_task, d_acc, s, P);
        else make_plan<2>(v, g->n, plo, phi, max_task, d_acc, s, P);
    }
    out->work = P.work;
    out->scanned = P.w_total;
    const u64 h_total = P.w_total;
    if (debug_enabled())
        fprintf(stderr, "[tl] list algo=%d m=%llu compacted=%llu light_items=%llu heavy_items=%llu tasks=%llu\n", algo,
                (unsigned long long)m, (unsigned long long)P.ncomp, (unsigned long long)P.w_light,
                (unsigned long long)(P.w_total - P.w_light), (unsigned long long)P.ntasks);

    // output plumbing shared by the emitting modes
    const bool emitting = (tri || cb) && h_total;
    const u64 hole_cap = max_holes_per_probe();
    DevBuf holes, spill, chunk;
    Out o{nullptr, 0, nullptr, 0, d_acc, nullptr, hole_cap};  // acc[5] = heavy task queue
    if (emitting) {
        holes = DevBuf(hole_cap * sizeof(Hole), s);
        o.holes = holes.as<Hole>();
        o.spill_cap = hole_cap * RESERVE;
        spill = DevBuf(o.spill_cap * 3 * sizeof(u32), s);
        o.spill = spill.as<u32>();
    }

    auto probe = [&](u64 k0, u64 k1, bool emit) {
        PhaseTimer t(TL_PHASE_PROBE, s);
        if (algo == 0) launch_probe<0>(v, P, k0, k1, emit, o, s);
        else if (algo == 1) launch_probe<1>(v, P, k0, k1, emit, o, s);
        else launch_probe<2>(v, P, k0, k1, emit, o, s);
    };

    int rc = TL_OK;
    u64 h_acc[NACC] = {0};
    u64 slices = h_total ? 1 : 0, redone = 0;
    if (h_total == 0) {
        // nothing to scan
    } else if (tri) {
        o.tri = tri;
        o.cap = cap;
        probe(0, h_total, true);
        d2h_sync(s, {{h_acc, d_acc, sizeof h_acc}});
        if (h_acc[0] > cap) rc = TL_ECAPACITY;
        else fix_holes(o, h_acc[0], h_acc[3], h_acc[4], s);
    } else if (cb) {
        // Each scanned element yields at most one triangle, so a slice of K
        // work items always fits a chunk of K triangles.  With chunk_growth
        // above 1, slices grow from the previous slice's triangles per item
        // (hit rates are far below one) for fuller chunks; a slice that finds
        // more than K triangles (the excess is counted but dropped) is redone
        // shorter from the accumulators saved before it.  A slice of K items
        // cannot overflow, so this ends.
        const u64 K = g_chunk_triangles;
        const u64 room = K * tuning().chunk_room;  // triangles the device chunk holds
        chunk = DevBuf(room * 3 * sizeof(u32), s);
        o.tri = chunk.as<u32>();
        o.cap = room;
        DevBuf saved(NACC * sizeof(u64), s);
        const Tuning &tu = tuning();
        // a slice of `room` items cannot find more triangles than the chunk holds
        const u64 L_max = room * CHUNK_GROWTH_MAX;
        u64 L = room, prev_count = 0;
        for (u64 k0 = 0; k0 < h_total;) {
            const u64 k1 = (h_total - k0 > L) ? k0 + L : h_total;
            TL_HIP(hipMemcpyAsync(saved.p, d_acc, NACC * sizeof(u64), hipMemcpyDeviceToDevice, s));
            TL_HIP(hipMemsetAsync(d_acc + 3, 0, 2 * sizeof(u64), s));  // cursor and holes
            probe(k0, k1, true);
            d2h_sync(s, {{h_acc, d_acc, sizeof h_acc}});
            const u64 got = h_acc[0] - prev_count;
            if (got > room) {
                TL_HIP(hipMemcpyAsync(d_acc, saved.p, NACC * sizeof(u64), hipMemcpyDeviceToDevice, s));
                L = chunk_slice_items(room, got, k1 - k0, L / 2, tu.chunk_margin);
                redone++;
                continue;
            }
            prev_count = h_acc[0];
            fix_holes(o, got, h_acc[3], h_acc[4], s);
            // handed out K triangles at a time
            for (u64 off = 0; off < got && rc == TL_OK; off += K) {
                const u64 k = got - off < K ? got - off : K;
                if (cb(o.tri + 3 * off, k, user) != 0) rc = TL_EABORT;
            }
            if (rc != TL_OK) break;
            L = chunk_slice_items(room, got, k1 - k0, std::min(L * tu.chunk_growth, L_max), tu.chunk_margin);
            k0 = k1;
            if (k0 < h_total) slices++;
        }
        d2h_sync(s, {{h_acc, d_acc, sizeof h_acc}});
    } else {
        probe(0, h_total, false);
        d2h_sync(s, {{h_acc, d_acc, sizeof h_acc}});
    }
    out->count = h_acc[0];
    out->hash = h_acc[1];
    tl_list_stats &st = last_stats();
    st.light_items = P.w_light;
    st.heavy_items = P.w_total - P.w_light;
    st.light_seeds = P.nlight;
    st.heavy_seeds = P.ncomp - P.nlight;
    st.heavy_work = h_acc[6];
    st.heavy_pivots = h_acc[7];
    st.heavy_triangles = h_acc[8];
    st.heavy_staged = h_acc[9];
    for (int md = 0; md < NMODES; md++) st.mode_items[md] = h_acc[10 + md];
    st.items_long = h_acc[ACC_PATHS + 0];
    st.items_short = h_acc[ACC_PATHS + 1];
    st.items_single = h_acc[ACC_PATHS + 2];
    st.split_below = h_acc[ACC_PATHS + 3];
    st.split_below_global = h_acc[ACC_PATHS + 4];
    st.heavy_task_staged = h_acc[ACC_PATHS + 5];
    st.split_groups = h_acc[ACC_PATHS + 6];
    st.split_below_groups = h_acc[ACC_PATHS + 7];
    st.tasks = P.ntasks;
    st.slices = slices;
    st.slices_redone = redone;
    return rc;
}
