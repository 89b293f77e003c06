// Batched listing: many independent graphs listed as one.
//
// The batch is the disjoint union of its graphs: graph i's vertex v becomes
// vbase[i] + v and its rank vbase[i] + rank_i[v], so the union's ordering
// keeps every graph's vertices contiguous in rank space and its triangles
// are exactly the graphs' triangles.  One orientation builds the union's
// CSR; one listing pass attributes every triangle (and every seed edge's
// work) to the graph owning its pivot and accumulates per-graph count,
// digest (over local ids) and paper work.
//
// The listing pipeline allocates nothing and never waits for the host: all
// of its buffers belong to the batch and all sizes are fixed by the union's
// n and m, so it is captured once per algorithm as a HIP graph and replayed.
// Its pivots fall in two bins: pivots whose pruned work reaches a threshold
// (and whose list's rank span fits an LDS bitmap) get a workgroup each, with
// the list marked in LDS (the paper's B array); all other seed edges form
// one flattened item space walked by fixed runs of 64-lane wavefronts.
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "tl_internal.h"
#include "dev_util.h"
#include "probe_common.h"
#include "timing.h"

namespace {

constexpr int BB = 256;

__global__ void k_fill_u64(u64 *p, u64 n, u64 v) {
    GRID_STRIDE(i, n) { p[i] = v; }
}
__global__ void k_fill_u32(u32 *p, u64 n, u32 v) {
    GRID_STRIDE(i, n) { p[i] = v; }
}

// Each wavefront takes one contiguous run of the items [0, total) and finds
// the graph of its first item once; later chunks step it forward (graph g
// holds items [base[g], base[g + 1]), in order; empty graphs are skipped).
template <class T>
struct GraphRun {
    u64 wb, we, g0;  // wave-uniform
    __device__ __forceinline__ GraphRun(const T *base, u32 k, u64 total) {
        const u64 nw = ((u64)gridDim.x * blockDim.x) / WAVE;
        const u64 gw = ((u64)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
        const u64 per = ((total + nw - 1) / nw + WAVE - 1) & ~(u64)(WAVE - 1);
        wb = gw * per < total ? gw * per : total;
        we = wb + per < total ? wb + per : total;
        g0 = wb < we ? uni64(upper_bound_dev<T>(base, 0, (u64)k + 1, (T)wb) - 1) : 0;
    }
    // the graph of item c (wave-uniform, c >= every earlier call's c)
    __device__ __forceinline__ void seek(const T *base, u64 c) {
        while ((u64)base[g0 + 1] <= c) g0++;
    }
    // the graph of item i >= the last seek's c (per lane: a few steps at most)
    __device__ __forceinline__ u32 of(const T *base, u64 i) const {
        u64 g = g0;
        while ((u64)base[g + 1] <= i) g++;
        return (u32)g;
    }
};

__global__ void k_union_vertices(const u32 *rank, const u32 *vbase, u32 k, u32 N, u32 *gid, u32 *urank, u32 *flag) {
    GraphRun<u32> run(vbase, k, N);
    for (u64 c = run.wb; c < run.we; c += WAVE) {
        run.seek(vbase, c);
        const u64 v = c + lane_id();
        if (v < run.we) {
            const u32 g = run.of(vbase, v);
            const u32 ng = vbase[g + 1] - vbase[g];
            const u32 r = rank[v];
            if (r >= ng) atomicOr(flag, 1u);
            gid[v] = g;
            urank[v] = vbase[g] + (r < ng ? r : 0u);
        }
    }
}

// Arrays of one oriented graph, for building a union from graphs already
// oriented (their ranks and edge indices shifted by the graph's bases).
struct CsrRef {
    const u64 *off_f, *off_b;
    const u32 *adj_f, *row_f, *adj_b, *row_b, *twin_b, *inv;
};

// The union's per-vertex arrays: offsets shifted by the graph's edge base,
// inverse permutation by its vertex base, and the graph id of each vertex.
__global__ void k_concat_vertices(const CsrRef *gs, const u32 *vbase, const u64 *ebase, u32 k, u32 N, u64 *off_f,
                                  u64 *off_b, u32 *inv, u32 *gid) {
    GraphRun<u32> run(vbase, k, N);
    for (u64 c0 = run.wb; c0 < run.we; c0 += WAVE) {
        run.seek(vbase, c0);
        const u64 v = c0 + lane_id();
        if (v < run.we) {
            const u32 g = run.of(vbase, v);
            const u32 r = (u32)(v - vbase[g]);
            const CsrRef c = gs[g];
            off_f[v] = c.off_f[r] + ebase[g];
            off_b[v] = c.off_b[r] + ebase[g];
            inv[v] = c.inv[r] + vbase[g];
            gid[v] = g;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        off_f[N] = ebase[k];
        off_b[N] = ebase[k];
    }
}

// The union's per-edge arrays: ranks shifted by the graph's vertex base,
// forward indices by its edge base.
__global__ void k_concat_edges(const CsrRef *gs, const u32 *vbase, const u64 *ebase, u32 k, u64 M, u32 *adj_f,
                               u32 *row_f, u32 *adj_b, u32 *row_b, u32 *twin_b) {
    GraphRun<u64> run(ebase, k, M);
    for (u64 c0 = run.wb; c0 < run.we; c0 += WAVE) {
        run.seek(ebase, c0);
        const u64 i = c0 + lane_id();
        if (i < run.we) {
            const u32 g = run.of(ebase, i);
            const u64 j = i - ebase[g];
            const u32 vb = vbase[g];
            const CsrRef c = gs[g];
            adj_f[i] = c.adj_f[j] + vb;
            row_f[i] = c.row_f[j] + vb;
            adj_b[i] = c.adj_b[j] + vb;
            row_b[i] = c.row_b[j] + vb;
            twin_b[i] = (u32)(c.twin_b[j] + ebase[g]);
        }
    }
}

__global__ void k_union_edges(const u32 *src, const u32 *dst, const u64 *ebase, const u32 *vbase, u32 k, u64 M,
                              u32 *usrc, u32 *udst, u32 *flag) {
    GraphRun<u64> run(ebase, k, M);
    for (u64 c = run.wb; c < run.we; c += WAVE) {
        run.seek(ebase, c);
        const u64 i = c + lane_id();
        if (i < run.we) {
            const u32 g = run.of(ebase, i);
            const u32 ng = vbase[g + 1] - vbase[g];
            u32 a = src[i], b = dst[i];
            if (a >= ng || b >= ng) {
                atomicOr(flag, 2u);
                a = 0;
                b = 0;  // a self-loop: dropped by the orientation
            }
            usrc[i] = vbase[g] + a;
            udst[i] = vbase[g] + b;
        }
    }
}

// Adds v to dest[key * stride] for runs of equal key across the lanes of a
// wavefront (keys non-decreasing along lanes); one atomic per run.
__device__ __forceinline__ void wave_segmented_add(bool valid, u32 key, u64 v, u64 *dest, int stride) {
    const int lane = lane_id();
    const u32 kk = valid ? key : 0xffffffffu;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        const u64 t = shfl_up_u64(v, d);
        const u32 q = __shfl_up(kk, d, WAVE);
        if (lane >= d && q == kk) v += t;
    }
    const u32 nk = __shfl_down(kk, 1, WAVE);
    const bool last = valid && (lane == WAVE - 1 || nk != kk);
    if (last && v) atomicAdd((unsigned long long *)&dest[(u64)kk * stride], (unsigned long long)v);
}

// ------------------------------------------------------------------ tuning

struct BatchTuning {
    u64 heavy_min = 4096;   // pruned items of a pivot before it gets a workgroup
    u64 heavy_block = 512;  // threads of a heavy workgroup: 256, 512 or 1024
    u64 heavy_per_cu = 2;   // heavy workgroups per CU
    u64 light_per_cu = 8;   // light workgroups (256 threads) per CU
    u64 plan_full = 8;      // scanned lists this short are taken whole (no window searches)
};

std::mutex g_btune_mu;

BatchTuning &btune() {
    static BatchTuning t = [] {
        BatchTuning d;
        auto env = [](const char *k, u64 &v) {
            const char *e = getenv(k);
            if (e && *e) v = strtoull(e, nullptr, 10);
        };
        env("TL_TUNE_BATCH_HEAVY_MIN", d.heavy_min);
        env("TL_TUNE_BATCH_HEAVY_BLOCK", d.heavy_block);
        env("TL_TUNE_BATCH_HEAVY_PER_CU", d.heavy_per_cu);
        env("TL_TUNE_BATCH_LIGHT_PER_CU", d.light_per_cu);
        env("TL_TUNE_BATCH_PLAN_FULL", d.plan_full);
        if (d.heavy_block != 256 && d.heavy_block != 1024) d.heavy_block = 512;
        if (d.heavy_per_cu < 1 || d.heavy_per_cu > 2) d.heavy_per_cu = 2;
        if (d.light_per_cu < 1 || d.light_per_cu > 64) d.light_per_cu = 8;
        return d;
    }();
    return t;
}

constexpr u32 BH_LDS_BYTES = 64u * 1024u;     // the heavy bin's bitmap
constexpr u32 BH_BITS = BH_LDS_BYTES * 8u;   // rank span it covers

// -------------------------------------------------------------- the pass

// The window of seed e in its scanned list: the part of S from the smallest
// candidate of T up to the largest (or, under A++, possibly up to the pivot
// itself); no other element can match.
template <int ALGO>
__device__ __forceinline__ u32 seed_window(const Seed<ALGO> &sd, u32 full_max, u64 &abs) {
    abs = 0;
    if (sd.t_lo < sd.t_hi && sd.s_lo < sd.s_hi && sd.s_hi - sd.s_lo <= full_max) {
        // short list: scanned whole; elements outside the window fail the
        // membership test like any non-member
        abs = sd.s_lo;
        return (u32)(sd.s_hi - sd.s_lo);
    }
    if (sd.t_lo < sd.t_hi && sd.s_lo < sd.s_hi) {
        const u32 tmin = sd.T[sd.t_lo], tmax = sd.T[sd.t_hi - 1];
        // A++: the pivot p itself sits in S = N+_x at twin_b[e], above every
        // candidate, so the window ends there or earlier; the entries between
        // the last candidate and p are left in it (and fail the membership
        // test) when their rank span is under 1/64 of the candidates'
        const u64 hi = ALGO == 0 ? (u64)sd.twin : sd.s_hi;
        const u64 a = lower_bound_front<u32>(sd.S, sd.s_lo, hi, tmin);
        const u64 b = ALGO == 0 && (u64)(sd.p - tmax) * 64 <= (u64)(sd.p - tmin)
                          ? hi : upper_bound_back<u32>(sd.S, a, hi, tmax);
        abs = a;
        return (u32)(b - a);
    }
    return 0;
}

// Per seed edge: its window, start sabs[e] and length lw[e]; per pivot: the
// sum of its seeds' lengths wp[p]; per graph: the paper's work (the scanned
// lists' lengths).
// pg holds (count, digest, work) per graph.
template <int ALGO>
__global__ __launch_bounds__(BB) void k_bplan(GView g, const u32 *gid, u32 full_max, u32 *lw, u64 *sabs, u64 *wp,
                                              u64 *pg) {
    const XcdRange rg(g.m);  // the grid is a multiple of 8 workgroups
    const u64 iters = uni64(rg.wave_iters());
    for (u64 it = 0; it < iters; it++) {
        const u64 e = rg.first + it * rg.stride;
        const bool valid = e < rg.end;
        u32 gr = 0, p = 0, l = 0;
        u64 w = 0;
        if (valid) {
            Seed<ALGO> sd(g, e);
            p = sd.p;
            gr = gid[p];
            w = sd.s_hi - sd.s_lo;
            u64 abs;
            l = seed_window<ALGO>(sd, full_max, abs);
            lw[e] = l;
            sabs[e] = abs;
        }
        wave_segmented_add(valid, gr, w, pg + 2, 3);
        wave_segmented_add(valid, p, l, wp, 1);
    }
}

// Pivot bins: 1 when the pivot's items reach heavy_min and its list's rank
// span fits the bitmap.
template <int ALGO>
__global__ void k_bclass(GView g, u32 N, const u64 *wp, u64 heavy_min, u32 *hflag) {
    const u64 *po = Form<ALGO>::piv_off(g);
    const u32 *pa = Form<ALGO>::piv_adj(g);
    GRID_STRIDE(p, N) {
        u32 h = 0;
        const u64 w = wp[p];
        if (w > 0 && w >= heavy_min) {
            const u64 t0 = po[p], t1 = po[p + 1];
            if (t1 > t0 && (u64)(pa[t1 - 1] - pa[t0]) < BH_BITS) h = 1u;
        }
        hflag[p] = h;
    }
}

// Seed flags for a two-part compaction: the low half counts seeds of light
// pivots, the high half seeds of heavy ones.
template <int ALGO>
__global__ void k_bflag(GView g, const u32 *lw, const u32 *hflag, u64 *f64) {
    GRID_STRIDE(e, g.m) {
        u64 f = 0;
        if (lw[e]) {
            const u32 p = ALGO == 0 ? g.row_b[e] : g.row_f[e];
            f = hflag[p] ? (1ull << 32) : 1ull;
        }
        f64[e] = f;
    }
}

// Seeds with a non-empty window, packed in seed order: light pivots' seeds
// at [0, nlight), heavy pivots' seeds after them.
template <int ALGO>
__global__ void k_bcompact(GView g, const u32 *gid, const u32 *lw, const u64 *sabs, const u64 *pos, u64 *cabs,
                           u32 *cxinv, u32 *ctlo, u32 *cthi, u32 *cpinv, u32 *cgid, u32 *clen) {
    const u64 nlight = pos[g.m] & 0xffffffffull;
    GRID_STRIDE(e, g.m) {
        const u64 pe = pos[e], pn = pos[e + 1];
        if (pn != pe) {
            const bool heavy = (pn >> 32) != (pe >> 32);
            const u64 d = heavy ? nlight + (pe >> 32) : (pe & 0xffffffffull);
            u32 p, x;
            u64 t_lo, t_hi;
            if (ALGO == 0) {
                p = g.row_b[e]; x = g.adj_b[e]; t_lo = e + 1; t_hi = g.off_b[p + 1];
            } else if (ALGO == 1) {
                p = g.row_f[e]; x = g.adj_f[e]; t_lo = e + 1; t_hi = g.off_f[p + 1];
            } else {
                p = g.row_f[e]; x = g.adj_f[e]; t_lo = g.off_b[p]; t_hi = g.off_b[p + 1];
            }
            cabs[d] = sabs[e];
            cxinv[d] = g.inv[x];
            ctlo[d] = (u32)t_lo;
            cthi[d] = (u32)t_hi;
            cpinv[d] = g.inv[p];
            cgid[d] = gid[p];
            clen[d] = lw[e];
        }
    }
}

__global__ void k_bhlist(u32 N, const u32 *hflag, const u64 *hpre, u32 *hpiv) {
    GRID_STRIDE(p, N) {
        if (hflag[p]) hpiv[hpre[p]] = (u32)p;
    }
}

struct BSeeds {
    const u64 *cpre, *cabs;
    const u32 *cxinv, *ctlo, *cthi, *cpinv, *cgid;
};

// Per-lane accumulator of (count, digest) for the graph of the lane's
// current items; a lane's items move through graphs in order, so each lane
// flushes once per graph it leaves.
struct GraphAcc {
    u32 gcur = 0xffffffffu;
    u64 cnt = 0, hsh = 0;
    __device__ __forceinline__ void add(u32 gr, u64 h, u64 *pg) {
        if (gr != gcur) {
            flush(pg);
            gcur = gr;
        }
        cnt += 1;
        hsh += h;
    }
    __device__ __forceinline__ void flush(u64 *pg) {
        if (cnt) {
            atomicAdd((unsigned long long *)&pg[3 * (u64)gcur + 0], (unsigned long long)cnt);
            atomicAdd((unsigned long long *)&pg[3 * (u64)gcur + 1], (unsigned long long)hsh);
        }
        cnt = 0;
        hsh = 0;
    }
};

// Light bin: the items [0, W) of the light seeds, W = cpre[nlight] read on
// the device; every wavefront of a fixed grid takes a contiguous run, 4
// chunks of 64 at a time when they lie in one window or in the 64 seeds
// from the current one.
template <int ALGO>
__global__ __launch_bounds__(BB) void k_bprobe(GView g, const u64 *__restrict__ cpre, const u64 *__restrict__ cabs,
                         const u32 *__restrict__ cxinv,
                         const u32 *__restrict__ ctlo, const u32 *__restrict__ cthi, const u32 *__restrict__ cpinv,
                         const u32 *__restrict__ cgid, const u64 *__restrict__ pos,
                                               const u32 *__restrict__ vbase, u64 *pg) {
    // restrict-qualified arguments: reads at wave-uniform indices become scalar loads
    const BSeeds L{cpre, cabs, cxinv, ctlo, cthi, cpinv, cgid};
    const int lane = lane_id();
    const u64 ncap = pos[g.m] & 0xffffffffull;
    const u64 W = L.cpre[ncap];
    const u64 gw = (u64)blockIdx.x * (blockDim.x / WAVE) + wave_id();
    const u64 nw = ((u64)gridDim.x * blockDim.x) / WAVE;
    const u64 per = (((W + nw - 1) / nw) + WAVE - 1) & ~(u64)(WAVE - 1);
    const u64 wb = gw * per;
    const u64 we = (wb + per < W) ? wb + per : W;
    const u32 *SA = Form<ALGO>::scan_adj(g);
    const u32 *T = Form<ALGO>::piv_adj(g);
    GraphAcc ga;
    // per wavefront: 64 staged hits (pivot, endpoint, third vertex, graph)
    // and the short-window walk's seed-start flags
    __shared__ uint4 stage_all[(BB / WAVE) * WAVE];
    __shared__ unsigned char flag_all[(BB / WAVE) * UN * WAVE];
    uint4 *stage = stage_all + wave_id() * WAVE;
    unsigned char *flag = flag_all + wave_id() * (UN * WAVE);
    // A sliding window over the pivot-list array T in LDS, per wavefront, as
    // in the plain light kernel: seeds are pivot-major (across the union's
    // graphs too), so the candidate ranges only move forward through T, and a
    // group whose ranges fit the window searches LDS instead of global memory.
    constexpr u32 TWL = 512;
    __shared__ u32 twin_all[(BB / WAVE) * TWL];
    u32 *tw = twin_all + wave_id() * TWL;
    u64 tw_lo = 0, tw_hi = 0;  // T[tw_lo, tw_hi) is staged (wave-uniform)
    auto cover = [&](u64 lo, u64 hi) -> bool {
        if (hi - lo > TWL) return false;
        if (lo >= tw_lo && hi <= tw_hi) return true;
        const u64 e = lo + TWL < g.m ? lo + TWL : g.m;
        const u32 n = (u32)(e - lo);
        u32 v[TWL / WAVE];
#pragma unroll
        for (int k = 0; k < (int)(TWL / WAVE); k++) {
            const u32 i = (u32)(k * WAVE + lane);
            v[k] = i < n ? T[lo + i] : 0u;
        }
        wave_lds_fence();  // (earlier searches of the window are done)
#pragma unroll
        for (int k = 0; k < (int)(TWL / WAVE); k++) tw[k * WAVE + lane] = v[k];
        wave_lds_fence();
        tw_lo = lo;
        tw_hi = e;
        return true;
    };
    // hits are packed into the staging area across groups and finished 64 at a time
    u32 staged = 0;  // wave-uniform
    auto flush = [&](u32 k) {
        wave_lds_fence();
        if ((u32)lane < k) {
            const uint4 e = stage[lane];
            const u32 vb = vbase[e.w];
            u32 a = e.x - vb, b = e.y - vb, c = g.inv[e.z] - vb;
            canon3(a, b, c);
            ga.add(e.w, tri_digest(a, b, c), pg);
        }
        wave_lds_fence();
    };
    auto report = [&](const u32 (&y)[UN], const bool (&h)[UN], const u32 (&pv)[UN], const u32 (&xv)[UN],
                      const u32 (&gv)[UN]) {
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
                if (h[j] && q[j] - r0 < room) stage[staged + (q[j] - r0)] = make_uint4(pv[j], xv[j], y[j], gv[j]);
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
                const u64 c = cur.c_lo;
                const u64 sab = L.cabs[c] + (kb - cur.base) + lane;
                const u64 t_lo = L.ctlo[c], t_hi = L.cthi[c];
                u32 y[UN], pv[UN], xv[UN], gv[UN];
                bool h[UN];
#pragma unroll
                for (int j = 0; j < UN; j++) y[j] = SA[sab + (u64)j * WAVE];
                if (cover(t_lo, t_hi)) member_multi(tw, t_lo - tw_lo, t_hi - tw_lo, y, h);
                else member_multi(T, t_lo, t_hi, y, h);
                const u32 pi = L.cpinv[c], xi = L.cxinv[c], gi = L.cgid[c];
#pragma unroll
                for (int j = 0; j < UN; j++) { pv[j] = pi; xv[j] = xi; gv[j] = gi; }
                report(y, h, pv, xv, gv);
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
                    const u64 A = inw ? L.cabs[ci] : 0ull;
                    const u32 X = inw ? L.cxinv[ci] : 0u, PI = inw ? L.cpinv[ci] : 0u, GI = inw ? L.cgid[ci] : 0u;
                    const u32 TL = inw ? L.ctlo[ci] : 0u, TH = inw ? L.cthi[ci] : 0u;
                    // item kb + i of seed c: scan index E[c] + i (mod 2^32; m < 2^32)
                    const u32 E = (u32)(A - P + kb);
                    int lo[UN];
                    const int lo_last = locate_short(P, kb, flag, lo);
                    u32 y[UN], pv[UN], xv[UN], gv[UN];
                    u64 tl[UN], th[UN];
                    bool h[UN];
#pragma unroll
                    for (int j = 0; j < UN; j++) {
                        y[j] = SA[(u32)(__shfl(E, lo[j], WAVE) + (u32)(j * WAVE + lane))];
                        xv[j] = __shfl(X, lo[j], WAVE);
                        pv[j] = __shfl(PI, lo[j], WAVE);
                        gv[j] = __shfl(GI, lo[j], WAVE);
                        tl[j] = __shfl(TL, lo[j], WAVE);
                        th[j] = __shfl(TH, lo[j], WAVE);
                    }
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
                    } else {
                        member_multi_var(T, tl, th, y, h);
                    }
                    report(y, h, pv, xv, gv);
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
            if (act) {
                const u32 y = SA[L.cabs[c] + rel];
                const u64 t_lo = L.ctlo[c], t_hi = L.cthi[c];
                const u64 j = lower_bound_dev<u32>(T, t_lo, t_hi, y);
                if (j < t_hi && T[j] == y) {
                    const u32 gi = L.cgid[c], vb = vbase[gi];
                    u32 a = L.cpinv[c] - vb, b = L.cxinv[c] - vb, cc = g.inv[y] - vb;
                    canon3(a, b, cc);
                    ga.add(gi, tri_digest(a, b, cc), pg);
                }
            }
            kb += WAVE;
            cur.advance(kb, c);
        }
    }
    if (staged) flush(staged);
    ga.flush(pg);
}

// Heavy bin: persistent workgroups take heavy pivots from a queue; each
// marks the pivot's list in an LDS bitmap (bit y - min of the list), then
// its wavefronts share the items of the pivot's compacted seeds, each item
// tested by one LDS read, and the marks are cleared for the next pivot.
// Every workgroup leaves once the queue passes the heavy pivot count.
template <int ALGO, int HBS>
__global__ __launch_bounds__(HBS) void k_bheavy(GView g, const u64 *__restrict__ cpre, const u64 *__restrict__ cabs,
                         const u32 *__restrict__ cxinv,
                         const u32 *__restrict__ ctlo, const u32 *__restrict__ cthi, const u32 *__restrict__ cpinv,
                         const u32 *__restrict__ cgid, const u64 *__restrict__ pos,
                                                const u32 *__restrict__ hpiv, const u64 *__restrict__ hpre, u32 N,
                                                const u32 *__restrict__ gid, const u32 *__restrict__ vbase,
                                                u64 *queue, u64 *pg) {
    const BSeeds L{cpre, cabs, cxinv, ctlo, cthi, cpinv, cgid};
    extern __shared__ u32 bits[];
    __shared__ u64 next;
    // per wavefront: 64 staged hits (endpoint, third vertex) and the
    // short-window walk's seed-start flags
    __shared__ uint2 stage_all[(HBS / WAVE) * WAVE];
    __shared__ unsigned char flag_all[(HBS / WAVE) * UN * WAVE];
    const int lane = lane_id(), wid = (int)wave_id(), nwv = HBS / WAVE;
    uint2 *stage = stage_all + wid * WAVE;
    unsigned char *flag = flag_all + wid * (UN * WAVE);
    const u64 nheavy = hpre[N];
    const u64 nlight = pos[g.m] & 0xffffffffull;
    const u64 *so = Form<ALGO>::seed_off(g);
    const u64 *po = Form<ALGO>::piv_off(g);
    const u32 *pa = Form<ALGO>::piv_adj(g);
    const u32 *SA = Form<ALGO>::scan_adj(g);
    for (u32 i = threadIdx.x; i < BH_BITS / 32; i += HBS) bits[i] = 0u;
    __syncthreads();
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd((unsigned long long *)queue, 1ull);
        __syncthreads();
        const u64 hi = uni64(next);
        __syncthreads();
        if (hi >= nheavy) break;  // uniform across the workgroup
        const u32 p = hpiv[hi];
        const u64 t0 = po[p], t1 = po[p + 1];
        const u32 tmin = pa[t0], tmax = pa[t1 - 1];
        for (u64 i = t0 + threadIdx.x; i < t1; i += HBS) {
            const u32 v = pa[i] - tmin;
            atomicOr(&bits[v >> 5], 1u << (v & 31));
        }
        __syncthreads();
        const u64 cb = nlight + (pos[so[p]] >> 32), ce = nlight + (pos[so[p + 1]] >> 32);
        const u64 a = L.cpre[cb], b = L.cpre[ce];
        u64 wb, we;
        {
            const u64 per = (((b - a + nwv - 1) / nwv) + 63) & ~(u64)63;
            wb = a + (u64)wid * per;
            we = (wb + per < b) ? wb + per : b;
        }
        const u32 gi = gid[p], vb = vbase[gi];
        const u32 pl = g.inv[p] - vb;
        u64 cnt = 0, hsh = 0;
        auto member = [&](u32 y) -> bool {
            const u32 v = y - tmin;
            return y >= tmin && y <= tmax && ((bits[v >> 5] >> (v & 31)) & 1u);
        };
        // hits packed into the staging area across groups, finished 64 at a
        // time (and at the end of the pivot)
        u32 staged = 0;  // wave-uniform
        auto flush = [&](u32 k) {
            wave_lds_fence();
            if ((u32)lane < k) {
                const uint2 e = stage[lane];
                u32 x0 = pl, x1 = e.x - vb, x2 = g.inv[e.y] - vb;
                canon3(x0, x1, x2);
                cnt += 1;
                hsh += tri_digest(x0, x1, x2);
            }
            wave_lds_fence();
        };
        auto report = [&](const u32 (&y)[UN], const bool (&h)[UN], const u32 (&xv)[UN]) {
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
        if (wb < we) {
            SeedCursor cur(L.cpre, cb, ce, wb);
            u64 kb = wb;
            while (kb < we) {
                if (cur.end >= kb + UN * WAVE && kb + UN * WAVE <= we) {
                    const u64 c = cur.c_lo;
                    const u64 sab = L.cabs[c] + (kb - cur.base) + lane;
                    u32 y[UN], xv[UN];
                    bool h[UN];
#pragma unroll
                    for (int j = 0; j < UN; j++) y[j] = SA[sab + (u64)j * WAVE];
                    const u32 xi = L.cxinv[c];
#pragma unroll
                    for (int j = 0; j < UN; j++) {
                        h[j] = member(y[j]);
                        xv[j] = xi;
                    }
                    report(y, h, xv);
                    kb += UN * WAVE;
                    cur.advance(kb, c);
                    continue;
                }
                if (kb + UN * WAVE <= we) {
                    const u64 ci = cur.c_lo + lane;
                    const bool inw = ci < ce;
                    const u64 P = inw ? L.cpre[ci] : ~0ull;
                    const u64 pend = (cur.c_lo + WAVE <= ce) ? L.cpre[cur.c_lo + WAVE] : ~0ull;
                    if (pend >= kb + UN * WAVE) {
                        const u64 A = inw ? L.cabs[ci] : 0ull;
                        const u32 X = inw ? L.cxinv[ci] : 0u;
                        // item kb + i of seed c: scan index E[c] + i (mod 2^32; m < 2^32)
                        const u32 E = (u32)(A - P + kb);
                        int lo[UN];
                        const int lo_last = locate_short(P, kb, flag, lo);
                        u32 y[UN], xv[UN];
                        bool h[UN];
#pragma unroll
                        for (int j = 0; j < UN; j++) {
                            y[j] = SA[(u32)(__shfl(E, lo[j], WAVE) + (u32)(j * WAVE + lane))];
                            xv[j] = __shfl(X, lo[j], WAVE);
                        }
#pragma unroll
                        for (int j = 0; j < UN; j++) h[j] = member(y[j]);
                        report(y, h, xv);
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
                if (act) {
                    const u32 y = SA[L.cabs[c] + rel];
                    if (member(y)) {
                        u32 x0 = pl, x1 = L.cxinv[c] - vb, x2 = g.inv[y] - vb;
                        canon3(x0, x1, x2);
                        cnt += 1;
                        hsh += tri_digest(x0, x1, x2);
                    }
                }
                kb += WAVE;
                cur.advance(kb, c);
            }
        }
        if (staged) flush(staged);
        cnt = wave_sum_u64(cnt);
        hsh = wave_sum_u64(hsh);
        if (lane == 0 && cnt) {
            atomicAdd((unsigned long long *)&pg[3 * (u64)gi + 0], (unsigned long long)cnt);
            atomicAdd((unsigned long long *)&pg[3 * (u64)gi + 1], (unsigned long long)hsh);
        }
        __syncthreads();  // every wavefront is done with the marks
        for (u64 i = t0 + threadIdx.x; i < t1; i += HBS) {
            const u32 v = pa[i] - tmin;
            bits[v >> 5] = 0u;
        }
        __syncthreads();
    }
}

unsigned grid_b(u64 items) { return grid_for(items, BB, (unsigned)tl_num_cus() * 16); }
// a grid of whole groups of 8 workgroups (for XcdRange walks)
unsigned grid_x8(u64 items) { return (grid_b(items) + 7u) & ~7u; }

// Lets the heavy-bin kernels use their whole dynamic LDS (once per process).
void prepare_batch_kernels() {
    static std::once_flag once;
    std::call_once(once, [] {
        const void *fns[] = {
            (const void *)k_bheavy<0, 256>, (const void *)k_bheavy<0, 512>, (const void *)k_bheavy<0, 1024>,
            (const void *)k_bheavy<1, 256>, (const void *)k_bheavy<1, 512>, (const void *)k_bheavy<1, 1024>,
            (const void *)k_bheavy<2, 256>, (const void *)k_bheavy<2, 512>, (const void *)k_bheavy<2, 1024>};
        for (const void *f : fns)
            (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)BH_LDS_BYTES);
        (void)hipGetLastError();
    });
}

}  // namespace

struct tl_batch {
    u32 k = 0, N = 0;
    u64 M = 0;
    tl_csr *g = nullptr;
    u32 *gid = nullptr, *vbase = nullptr;
    // listing scratch, owned for the batch's lifetime: per seed edge
    u32 *lw = nullptr, *cxinv = nullptr, *ctlo = nullptr, *cthi = nullptr, *cpinv = nullptr, *cgid = nullptr,
        *clen = nullptr;
    u64 *f64 = nullptr, *pos = nullptr, *cabs = nullptr, *cpre = nullptr;
    // per pivot
    u64 *wp = nullptr, *hpre = nullptr;
    u32 *hflag = nullptr, *hpiv = nullptr;
    u64 *ws = nullptr, *pg = nullptr, *ctl = nullptr;
    hipStream_t cap_stream[3] = {nullptr, nullptr, nullptr};
    hipGraphExec_t exec[3] = {nullptr, nullptr, nullptr};
    hipGraph_t graph[3] = {nullptr, nullptr, nullptr};
    BatchTuning cap_tune[3];  // the tuning each captured pass was built with
    int device = 0;
};

namespace {

bool same_tune(const BatchTuning &a, const BatchTuning &b) {
    return a.heavy_min == b.heavy_min && a.heavy_block == b.heavy_block && a.heavy_per_cu == b.heavy_per_cu &&
           a.light_per_cu == b.light_per_cu && a.plan_full == b.plan_full;
}

// Enqueue the whole listing pass on s (no host waits, no allocation).
template <int ALGO>
void enqueue_batch_list(tl_batch *b, const BatchTuning &tu, hipStream_t s) {
    const tl_csr *g = b->g;
    const GView v{g->off_f, g->off_b, g->adj_f, g->adj_b, g->row_f, g->row_b, g->inv, g->m, g->twin_b};
    const u64 m = g->m, N = b->N;
    const unsigned cus = (unsigned)tl_num_cus();
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_b(3ull * b->k)), dim3(BB), 0, s, b->pg, 3ull * b->k, 0ull);
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_b(N)), dim3(BB), 0, s, b->wp, N, 0ull);
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, s, b->ctl, 1ull, 0ull);
    // the seeds' window starts live in cpre's buffer until the compaction
    // has read them; the scan of the compacted lengths then overwrites them
    hipLaunchKernelGGL((k_bplan<ALGO>), dim3(grid_x8(m)), dim3(BB), 0, s, v, b->gid, (u32)tu.plan_full, b->lw, b->cpre,
                       b->wp, b->pg);
    hipLaunchKernelGGL((k_bclass<ALGO>), dim3(grid_b(N)), dim3(BB), 0, s, v, (u32)N, b->wp, tu.heavy_min, b->hflag);
    hipLaunchKernelGGL((k_bflag<ALGO>), dim3(grid_b(m)), dim3(BB), 0, s, v, b->lw, b->hflag, b->f64);
    scan_u64_to_u64(b->f64, b->pos, m, s, b->ws);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_b(m)), dim3(BB), 0, s, b->clen, m, 0u);
    hipLaunchKernelGGL((k_bcompact<ALGO>), dim3(grid_b(m)), dim3(BB), 0, s, v, b->gid, b->lw, b->cpre, b->pos,
                       b->cabs, b->cxinv, b->ctlo, b->cthi, b->cpinv, b->cgid, b->clen);
    scan_u32_to_u64(b->clen, b->cpre, m, s, b->ws);
    scan_u32_to_u64(b->hflag, b->hpre, N, s, b->ws);
    hipLaunchKernelGGL(k_bhlist, dim3(grid_b(N)), dim3(BB), 0, s, (u32)N, b->hflag, b->hpre, b->hpiv);
// the compacted seed arrays, as the walks' restrict-qualified arguments
#define TL_BSEEDS b->cpre, b->cabs, b->cxinv, b->ctlo, b->cthi, b->cpinv, b->cgid
    hipLaunchKernelGGL((k_bprobe<ALGO>), dim3(cus * (unsigned)tu.light_per_cu), dim3(BB), 0, s, v, TL_BSEEDS,
                       b->pos, b->vbase, b->pg);
    const dim3 hg(cus * (unsigned)tu.heavy_per_cu);
    if (tu.heavy_block == 256)
        hipLaunchKernelGGL((k_bheavy<ALGO, 256>), hg, dim3(256), BH_LDS_BYTES, s, v, TL_BSEEDS, b->pos, b->hpiv,
                           b->hpre, (u32)N, b->gid, b->vbase, b->ctl, b->pg);
    else if (tu.heavy_block == 1024)
        hipLaunchKernelGGL((k_bheavy<ALGO, 1024>), hg, dim3(1024), BH_LDS_BYTES, s, v, TL_BSEEDS, b->pos, b->hpiv,
                           b->hpre, (u32)N, b->gid, b->vbase, b->ctl, b->pg);
    else
        hipLaunchKernelGGL((k_bheavy<ALGO, 512>), hg, dim3(512), BH_LDS_BYTES, s, v, TL_BSEEDS, b->pos, b->hpiv,
                           b->hpre, (u32)N, b->gid, b->vbase, b->ctl, b->pg);
#undef TL_BSEEDS
    TL_HIP(hipGetLastError());
}

void enqueue_for(tl_batch *b, int algo, const BatchTuning &tu, hipStream_t s) {
    if (algo == 0) enqueue_batch_list<0>(b, tu, s);
    else if (algo == 1) enqueue_batch_list<1>(b, tu, s);
    else enqueue_batch_list<2>(b, tu, s);
}

}  // namespace

int batch_set_tuning(const std::string &key, u64 value) {
    std::lock_guard<std::mutex> lk(g_btune_mu);
    BatchTuning &t = btune();
    if (key == "batch_heavy_min") t.heavy_min = value;
    else if (key == "batch_heavy_block" && (value == 256 || value == 512 || value == 1024)) t.heavy_block = value;
    else if (key == "batch_heavy_per_cu" && value >= 1 && value <= 2) t.heavy_per_cu = value;
    else if (key == "batch_light_per_cu" && value >= 1 && value <= 64) t.light_per_cu = value;
    else if (key == "batch_plan_full" && value <= (1u << 20)) t.plan_full = value;
    else return TL_EINVAL;
    return TL_OK;
}

int batch_get_tuning(const std::string &key, u64 *value) {
    std::lock_guard<std::mutex> lk(g_btune_mu);
    const BatchTuning &t = btune();
    if (key == "batch_heavy_min") *value = t.heavy_min;
    else if (key == "batch_heavy_block") *value = t.heavy_block;
    else if (key == "batch_heavy_per_cu") *value = t.heavy_per_cu;
    else if (key == "batch_light_per_cu") *value = t.light_per_cu;
    else if (key == "batch_plan_full") *value = t.plan_full;
    else return TL_EINVAL;
    return TL_OK;
}

static void alloc_batch_scratch(tl_batch *b, hipStream_t s);

tl_batch *batch_orient_impl(u32 k, const u32 *n, const u64 *m, const u32 *src, const u32 *dst, const u32 *rank,
                            hipStream_t s) {
    TL_REQUIRE(k > 0, TL_EINVAL, "empty batch");
    TL_REQUIRE(n && m, TL_EINVAL, "NULL size arrays");
    std::vector<u32> vb(k + 1);
    std::vector<u64> eb(k + 1);
    u64 N = 0, M = 0;
    for (u32 i = 0; i < k; i++) {
        vb[i] = (u32)N;
        eb[i] = M;
        N += n[i];
        M += m[i];
        TL_REQUIRE(N < 0xffffffffull, TL_EINVAL, "batch has 2^32 - 1 vertices or more");
        TL_REQUIRE(M < (1ull << 32), TL_EINVAL, "batch has 2^32 edges or more");
    }
    vb[k] = (u32)N;
    eb[k] = M;
    TL_REQUIRE(M == 0 || (src && dst), TL_EINVAL, "src/dst is NULL");
    TL_REQUIRE(N == 0 || rank, TL_EINVAL, "rank is NULL");

    struct Owner {
        tl_batch *b;
        ~Owner() { if (b) batch_free_impl(b, true); }
    } own{new tl_batch()};
    tl_batch *b = own.b;
    b->k = k;
    b->N = (u32)N;
    b->M = M;
    TL_HIP(hipGetDevice(&b->device));
    b->vbase = (u32 *)tl_dev_alloc((k + 1) * sizeof(u32), s);
    b->gid = (u32 *)tl_dev_alloc((N ? N : 1) * sizeof(u32), s);
    DevBuf ebase((k + 1) * sizeof(u64), s), flag(sizeof(u32), s), urank((N ? N : 1) * sizeof(u32), s);
    DevBuf usrc((M ? M : 1) * sizeof(u32), s), udst((M ? M : 1) * sizeof(u32), s);
    h2d_sync(b->vbase, vb.data(), (k + 1) * sizeof(u32), s);
    h2d_sync(ebase.p, eb.data(), (k + 1) * sizeof(u64), s);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, flag.as<u32>(), 1ull, 0u);
    if (N)
        hipLaunchKernelGGL(k_union_vertices, dim3(grid_b(N)), dim3(BB), 0, s, rank, b->vbase, k, (u32)N, b->gid,
                           urank.as<u32>(), flag.as<u32>());
    if (M)
        hipLaunchKernelGGL(k_union_edges, dim3(grid_b(M)), dim3(BB), 0, s, src, dst, ebase.as<u64>(), b->vbase, k, M,
                           usrc.as<u32>(), udst.as<u32>(), flag.as<u32>());
    TL_HIP(hipGetLastError());
    u32 h_flag = 0;
    d2h_sync(s, {{&h_flag, flag.p, sizeof(u32)}});
    TL_REQUIRE(!(h_flag & 1u), TL_EINVAL, "a graph's rank is not within [0, n)");
    TL_REQUIRE(!(h_flag & 2u), TL_EINVAL, "an edge endpoint is >= its graph's n");
    b->g = orient_impl((u32)N, usrc.as<u32>(), udst.as<u32>(), M, urank.as<u32>(), s);
    alloc_batch_scratch(b, s);
    tl_batch *r = own.b;
    own.b = nullptr;
    return r;
}

// Listing scratch for the union's m and N (owned for the batch's lifetime).
static void alloc_batch_scratch(tl_batch *b, hipStream_t s) {
    const u32 k = b->k, N = b->N;
    const u64 mm = b->g->m ? b->g->m : 1, nn = N ? N : 1;
    b->lw = (u32 *)tl_dev_alloc(mm * 4, s);
    b->cxinv = (u32 *)tl_dev_alloc(mm * 4, s);
    b->ctlo = (u32 *)tl_dev_alloc(mm * 4, s);
    b->cthi = (u32 *)tl_dev_alloc(mm * 4, s);
    b->cpinv = (u32 *)tl_dev_alloc(mm * 4, s);
    b->cgid = (u32 *)tl_dev_alloc(mm * 4, s);
    b->clen = (u32 *)tl_dev_alloc(mm * 4, s);
    b->f64 = (u64 *)tl_dev_alloc(mm * 8, s);
    b->cabs = b->f64;  // the seed flags are consumed by their scan before compaction writes cabs
    b->pos = (u64 *)tl_dev_alloc((mm + 1) * 8, s);
    b->cpre = (u64 *)tl_dev_alloc((mm + 1) * 8, s);
    b->wp = (u64 *)tl_dev_alloc(nn * 8, s);
    b->hpre = (u64 *)tl_dev_alloc((nn + 1) * 8, s);
    b->hflag = (u32 *)tl_dev_alloc(nn * 4, s);
    b->hpiv = (u32 *)tl_dev_alloc(nn * 4, s);
    b->ws = (u64 *)tl_dev_alloc((scan_workspace_words(mm > nn ? mm : nn) + 1) * 8, s);
    b->pg = (u64 *)tl_dev_alloc(3ull * k * 8, s);
    b->ctl = (u64 *)tl_dev_alloc(8, s);
    prepare_batch_kernels();
    TL_HIP(hipStreamSynchronize(s));
}

tl_batch *batch_from_csrs_impl(u32 k, const tl_csr *const *gs, hipStream_t s) {
    TL_REQUIRE(k > 0, TL_EINVAL, "empty batch");
    TL_REQUIRE(gs, TL_EINVAL, "NULL graph array");
    std::vector<u32> vb(k + 1);
    std::vector<u64> eb(k + 1);
    std::vector<CsrRef> refs(k);
    u64 N = 0, M = 0;
    for (u32 i = 0; i < k; i++) {
        TL_REQUIRE(gs[i], TL_EINVAL, "NULL graph handle");
        vb[i] = (u32)N;
        eb[i] = M;
        N += gs[i]->n;
        M += gs[i]->m;
        TL_REQUIRE(N < 0xffffffffull, TL_EINVAL, "batch has 2^32 - 1 vertices or more");
        TL_REQUIRE(M < (1ull << 32), TL_EINVAL, "batch has 2^32 edges or more");
        const tl_csr *c = gs[i];
        refs[i] = CsrRef{c->off_f, c->off_b, c->adj_f, c->row_f, c->adj_b, c->row_b, c->twin_b, c->inv};
    }
    vb[k] = (u32)N;
    eb[k] = M;
    struct Owner {
        tl_batch *b;
        ~Owner() { if (b) batch_free_impl(b, true); }
    } own{new tl_batch()};
    tl_batch *b = own.b;
    b->k = k;
    b->N = (u32)N;
    b->M = M;
    TL_HIP(hipGetDevice(&b->device));
    b->vbase = (u32 *)tl_dev_alloc((k + 1) * sizeof(u32), s);
    b->gid = (u32 *)tl_dev_alloc((N ? N : 1) * sizeof(u32), s);
    DevBuf ebase((k + 1) * sizeof(u64), s), dref(k * sizeof(CsrRef), s);
    h2d_sync(b->vbase, vb.data(), (k + 1) * sizeof(u32), s);
    h2d_sync(ebase.p, eb.data(), (k + 1) * sizeof(u64), s);
    h2d_sync(dref.p, refs.data(), k * sizeof(CsrRef), s);
    tl_csr *g = new tl_csr();
    b->g = g;
    TL_HIP(hipGetDevice(&g->device));
    g->n = (u32)N;
    g->m = M;
    const u64 mm = M ? M : 1;
    g->off_f = (u64 *)tl_dev_alloc(((u64)N + 1) * 8, s);
    g->off_b = (u64 *)tl_dev_alloc(((u64)N + 1) * 8, s);
    g->inv = (u32 *)tl_dev_alloc((N ? N : 1) * 4ull, s);
    g->adj_f = (u32 *)tl_dev_alloc(mm * 4, s);
    g->row_f = (u32 *)tl_dev_alloc(mm * 4, s);
    g->adj_b = (u32 *)tl_dev_alloc(mm * 4, s);
    g->row_b = (u32 *)tl_dev_alloc(mm * 4, s);
    g->twin_b = (u32 *)tl_dev_alloc(mm * 4, s);
    hipLaunchKernelGGL(k_concat_vertices, dim3(grid_b((u64)N + 1)), dim3(BB), 0, s, dref.as<CsrRef>(), b->vbase,
                       ebase.as<u64>(), k, (u32)N, g->off_f, g->off_b, g->inv, b->gid);
    if (M)
        hipLaunchKernelGGL(k_concat_edges, dim3(grid_b(M)), dim3(BB), 0, s, dref.as<CsrRef>(), b->vbase,
                           ebase.as<u64>(), k, M, g->adj_f, g->row_f, g->adj_b, g->row_b, g->twin_b);
    TL_HIP(hipGetLastError());
    alloc_batch_scratch(b, s);  // (waits for the stream: the staged refs above are read by then)
    tl_batch *r = own.b;
    own.b = nullptr;
    return r;
}

void batch_list_impl(tl_batch *b, int algo, hipStream_t s, int use_graph, u64 *per_graph_host, u64 *per_graph_dev) {
    BatchTuning tu;
    {
        std::lock_guard<std::mutex> lk(g_btune_mu);
        tu = btune();
    }
    PhaseTimer timer(TL_PHASE_BATCH, s);
    if (b->g->m == 0) {
        hipLaunchKernelGGL(k_fill_u64, dim3(grid_b(3ull * b->k)), dim3(BB), 0, s, b->pg, 3ull * b->k, 0ull);
        TL_HIP(hipGetLastError());
    } else if (!use_graph) {
        enqueue_for(b, algo, tu, s);
    } else {
        if (b->exec[algo] && !same_tune(b->cap_tune[algo], tu)) {
            // the tuning changed since the capture: capture again
            TL_HIP(hipStreamSynchronize(s));
            (void)hipGraphExecDestroy(b->exec[algo]);
            (void)hipGraphDestroy(b->graph[algo]);
            b->exec[algo] = nullptr;
            b->graph[algo] = nullptr;
        }
        if (!b->exec[algo]) {
            // capture on a private stream, so that the caller's stream state
            // is untouched, then replay on the caller's stream
            if (!b->cap_stream[algo]) TL_HIP(hipStreamCreateWithFlags(&b->cap_stream[algo], hipStreamNonBlocking));
            TL_HIP(hipStreamBeginCapture(b->cap_stream[algo], hipStreamCaptureModeThreadLocal));
            try {
                enqueue_for(b, algo, tu, b->cap_stream[algo]);
            } catch (...) {
                hipGraph_t dead = nullptr;
                (void)hipStreamEndCapture(b->cap_stream[algo], &dead);
                if (dead) (void)hipGraphDestroy(dead);
                throw;
            }
            TL_HIP(hipStreamEndCapture(b->cap_stream[algo], &b->graph[algo]));
            TL_HIP(hipGraphInstantiate(&b->exec[algo], b->graph[algo], nullptr, nullptr, 0));
            b->cap_tune[algo] = tu;
        }
        TL_HIP(hipGraphLaunch(b->exec[algo], s));
    }
    if (per_graph_dev) {
        TL_HIP(hipMemcpyAsync(per_graph_dev, b->pg, 3ull * b->k * 8, hipMemcpyDeviceToDevice, s));
    }
    timer.stop();
    if (per_graph_host) d2h_sync(s, {{per_graph_host, b->pg, 3ull * b->k * 8}});
    else TL_HIP(hipStreamSynchronize(s));
}

void batch_free_impl(tl_batch *b, bool device_sync) {
    if (!b) return;
    if (device_sync) (void)hipDeviceSynchronize();  // replays on any stream may still read the buffers
    for (int a = 0; a < 3; a++) {
        if (b->exec[a]) (void)hipGraphExecDestroy(b->exec[a]);
        if (b->graph[a]) (void)hipGraphDestroy(b->graph[a]);
        if (b->cap_stream[a]) (void)hipStreamDestroy(b->cap_stream[a]);
    }
    if (b->g) tl_csr_free(b->g);
    void *bufs[] = {b->gid, b->vbase, b->lw, b->cxinv, b->ctlo, b->cthi, b->cpinv, b->cgid, b->clen, b->f64,
                    b->pos, b->cpre, b->wp, b->hpre, b->hflag, b->hpiv, b->ws, b->pg, b->ctl};
    for (void *p : bufs) tl_dev_free(p);
    delete b;
}

void batch_sizes(const tl_batch *b, u32 *k, u32 *n, u64 *m) {
    if (k) *k = b->k;
    if (n) *n = b->N;
    if (m) *m = b->g ? b->g->m : 0;
}

const tl_csr *batch_csr(const tl_batch *b) { return b->g; }
