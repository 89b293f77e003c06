// Orderings computed on the device from an oriented graph: the degree
// ordering (Section 2.2: non-decreasing degree, ties by id) and Split
// (Section 3.3.3: the non-increasing degree ordering dealt alternately to
// the front and the back).  Together with tl_orient and tl_list they make
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

}  // namespace

void order_impl(const tl_csr *g, int kind, u32 *rank, hipStream_t s) {
    TL_REQUIRE(kind == 0 || kind == 1, TL_EINVAL, "unknown ordering");
    const u32 n = g->n;
    if (n == 0) return;
    TL_REQUIRE(rank, TL_EINVAL, "rank is NULL");
    PhaseTimer timer(TL_PHASE_ORDER, s);
    DevBuf deg((u64)n * 4, s), ids((u64)n * 4, s), deg2((u64)n * 4, s), sorted((u64)n * 4, s), mx(4, s);
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
    hipLaunchKernelGGL(k_rank_of, dim3(grid_o(n)), dim3(256), 0, s, sorted.as<u32>(), n, kind, rank);
    TL_HIP(hipGetLastError());
    timer.stop();
    TL_HIP(hipStreamSynchronize(s));
}
