// Orderings computed on the device from an oriented graph: the degree
// ordering (Section 2.2: non-decreasing degree, ties by id), Split
// (Section 3.3.3: the non-increasing degree ordering dealt alternately to
// the front and the back) and the core ordering (Section 1.3: non-decreasing
// coreness, ties by id; coreness by level-synchronous peeling).  Together with tl_orient and tl_list they make
// the full listing (ordering included) run on the GPU.
#include <hipcub/hipcub.hpp>

#include "tl_internal.h"
#include "dev_util.h"
#include "timing.h"

namespace {

// degree of every vertex in the simple graph: its successors plus its
// predecessors under any orientation
__global__ void k_vertex_degree(const u64 *off_f, const u64 *off_b, const u32 *inv, u32 n, u32 *deg, u32 *ids) {
    GRID_STRIDE(r, n) {
        const u32 u = inv[r];
        deg[u] = (u32)((off_f[r + 1] - off_f[r]) + (off_b[r + 1] - off_b[r]));
        ids[u] = u;
    }
}

__global__ void k_max_u32(const u32 *a, u64 n, u32 *out) {
    u32 m = 0;
    GRID_STRIDE(i, n) { m = a[i] > m ? a[i] : m; }
#pragma unroll
    for (int d = WAVE / 2; d > 0; d >>= 1) {
        const u32 o = __shfl_xor(m, d, WAVE);
        m = o > m ? o : m;
    }
    if (lane_id() == 0 && m) atomicMax(out, m);
}

// sorted[i] = vertex at position i of the degree ordering
__global__ void k_rank_of(const u32 *sorted, u32 n, int split, u32 *rank) {
    GRID_STRIDE(i, n) {
        const u32 u = sorted[i];
        if (!split) {
            rank[u] = (u32)i;
        } else {
            // position in the non-increasing ordering, 1-based
            const u32 pos = n - (u32)i;
            rank[u] = (pos & 1u) ? (pos - 1) / 2 : n - pos / 2;
        }
    }
}

unsigned grid_o(u64 items) { return grid_for(items, 256, (unsigned)tl_num_cus() * 16); }

constexpr u32 UNSET = 0xffffffffu;

// degree of every rank
__global__ void k_rank_degree(const u64 *off_f, const u64 *off_b, u32 n, u32 *deg, u32 *core) {
    GRID_STRIDE(r, n) {
        deg[r] = (u32)((off_f[r + 1] - off_f[r]) + (off_b[r + 1] - off_b[r]));
        core[r] = UNSET;
    }
}

// Peeling round at `level`: every vertex still present whose current degree
// is at most `level` leaves now with coreness `level` (one atomic per
// wavefront for the frontier's size).
__global__ void k_core_frontier(u32 n, const u32 *deg, u32 *core, u32 level, u32 *frontier, u32 *fcount) {
    const u64 stride = (u64)gridDim.x * blockDim.x;
    const u64 first = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    const u64 iters = (u64)n > first - lane_id() ? ((u64)n - (first - lane_id()) + stride - 1) / stride : 0;
    for (u64 it = 0; it < iters; it++) {
        const u64 r = first + it * stride;
        const bool take = r < n && core[r] == UNSET && deg[r] <= level;
        const u64 bal = __ballot(take);
        if (!bal) continue;
        u32 base = 0;
        if (lane_id() == 0) base = atomicAdd(fcount, (u32)__popcll(bal));
        base = __shfl(base, 0, WAVE);
        if (take) {
            core[r] = level;
            frontier[base + __popcll(bal & lanemask_lt())] = (u32)r;
        }
    }
}

// The frontier's vertices leave: one wavefront per vertex lowers the
// degree of each neighbour still present.
__global__ void k_core_peel(const u64 *off_f, const u32 *adj_f, const u64 *off_b, const u32 *adj_b,
                            const u32 *frontier, u32 nf, const u32 *core, u32 *deg) {
    const u64 w0 = ((u64)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const u64 nw = ((u64)gridDim.x * blockDim.x) / WAVE;
    for (u64 f = w0; f < nf; f += nw) {
        const u32 r = frontier[f];
        for (u64 j = off_f[r] + lane_id(); j < off_f[r + 1]; j += WAVE) {
            const u32 w = adj_f[j];
            if (core[w] == UNSET) atomicSub(&deg[w], 1u);
        }
        for (u64 j = off_b[r] + lane_id(); j < off_b[r + 1]; j += WAVE) {
            const u32 w = adj_b[j];
            if (core[w] == UNSET) atomicSub(&deg[w], 1u);
        }
    }
}

// smallest current degree among the vertices still present
__global__ void k_core_min(u32 n, const u32 *deg, const u32 *core, u32 *out) {
    u32 m = UNSET;
    GRID_STRIDE(r, n) {
        if (core[r] == UNSET && deg[r] < m) m = deg[r];
    }
#pragma unroll
    for (int d = WAVE / 2; d > 0; d >>= 1) {
        const u32 o = __shfl_xor(m, d, WAVE);
        m = o < m ? o : m;
    }
    if (lane_id() == 0 && m != UNSET) atomicMin(out, m);
}

// key of vertex inv[r]: its coreness
__global__ void k_core_keys(const u32 *core, const u32 *inv, u32 n, u32 *key, u32 *ids) {
    GRID_STRIDE(r, n) {
        const u32 u = inv[r];
        key[u] = core[r];
        ids[u] = u;
    }
}

}  // namespace

// Coreness of every rank by level-synchronous peeling, then keys (coreness
// per vertex id) and ids for the sort.
void coreness_keys(const tl_csr *g, u32 *key, u32 *ids, hipStream_t s) {
    const u32 n = g->n;
    DevBuf deg((u64)n * 4, s), core((u64)n * 4, s), frontier((u64)n * 4, s), cnt(8, s);
    u32 *fcount = cnt.as<u32>(), *mind = cnt.as<u32>() + 1;
    hipLaunchKernelGGL(k_rank_degree, dim3(grid_o(n)), dim3(256), 0, s, g->off_f, g->off_b, n, deg.as<u32>(),
                       core.as<u32>());
    TL_HIP(hipGetLastError());
    u32 level = 0;
    u64 remaining = n;
    while (remaining) {
        TL_HIP(hipMemsetAsync(fcount, 0, 4, s));
        hipLaunchKernelGGL(k_core_frontier, dim3(grid_o(n)), dim3(256), 0, s, n, deg.as<u32>(), core.as<u32>(), level,
                           frontier.as<u32>(), fcount);
        TL_HIP(hipGetLastError());
        u32 nf = 0;
        d2h_sync(s, {{&nf, fcount, 4}});
        if (nf == 0) {
            // nothing at this level any more: jump to the smallest degree left
            TL_HIP(hipMemsetAsync(mind, 0xff, 4, s));
            hipLaunchKernelGGL(k_core_min, dim3(grid_o(n)), dim3(256), 0, s, n, deg.as<u32>(), core.as<u32>(), mind);
            TL_HIP(hipGetLastError());
            u32 next = 0;
            d2h_sync(s, {{&next, mind, 4}});
            TL_REQUIRE(next != UNSET && next > level, TL_EHIP, "core peeling made no progress");
            level = next;
            continue;
        }
        remaining -= nf;
        hipLaunchKernelGGL(k_core_peel, dim3(grid_o((u64)nf * WAVE)), dim3(256), 0, s, g->off_f, g->adj_f, g->off_b,
                           g->adj_b, frontier.as<u32>(), nf, core.as<u32>(), deg.as<u32>());
        TL_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_core_keys, dim3(grid_o(n)), dim3(256), 0, s, core.as<u32>(), g->inv, n, key, ids);
    TL_HIP(hipGetLastError());
}

void order_impl(const tl_csr *g, int kind, u32 *rank, hipStream_t s) {
    TL_REQUIRE(kind >= 0 && kind <= 2, TL_EINVAL, "unknown ordering");
    const u32 n = g->n;
    if (n == 0) return;
    TL_REQUIRE(rank, TL_EINVAL, "rank is NULL");
    PhaseTimer timer(TL_PHASE_ORDER, s);
    DevBuf deg((u64)n * 4, s), ids((u64)n * 4, s), deg2((u64)n * 4, s), sorted((u64)n * 4, s), mx(4, s);
    if (kind == 2) coreness_keys(g, deg.as<u32>(), ids.as<u32>(), s);
    else
        hipLaunchKernelGGL(k_vertex_degree, dim3(grid_o(n)), dim3(256), 0, s, g->off_f, g->off_b, g->inv, n,
                           deg.as<u32>(), ids.as<u32>());
    TL_HIP(hipMemsetAsync(mx.p, 0, 4, s));
    hipLaunchKernelGGL(k_max_u32, dim3(grid_o(n)), dim3(256), 0, s, deg.as<u32>(), (u64)n, mx.as<u32>());
    TL_HIP(hipGetLastError());
    u32 maxdeg = 0;
    d2h_sync(s, {{&maxdeg, mx.p, 4}});
    int bits = 1;
    while (bits < 32 && (1ull << bits) <= maxdeg) bits++;
    // stable LSD radix sort of (degree, id) pairs by degree: ties keep the
    // increasing id order of the input
    size_t tmp_bytes = 0;
    TL_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, deg.as<u32>(), deg2.as<u32>(), ids.as<u32>(),
                                              sorted.as<u32>(), (int)n, 0, bits, s));
    DevBuf tmp(tmp_bytes ? tmp_bytes : 1, s);
    TL_HIP(hipcub::DeviceRadixSort::SortPairs(tmp.p, tmp_bytes, deg.as<u32>(), deg2.as<u32>(), ids.as<u32>(),
                                              sorted.as<u32>(), (int)n, 0, bits, s));
    hipLaunchKernelGGL(k_rank_of, dim3(grid_o(n)), dim3(256), 0, s, sorted.as<u32>(), n, kind == 1 ? 1 : 0, rank);
    TL_HIP(hipGetLastError());
    timer.stop();
    TL_HIP(hipStreamSynchronize(s));
}
