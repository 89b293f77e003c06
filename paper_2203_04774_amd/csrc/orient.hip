// Orientation of an undirected edge list by a vertex ordering (Section 1.3:
// (u,v) is in E_pi iff pi_u < pi_v) into rank-space forward and backward
// CSR arrays.
//
// Pipeline, all on the caller's stream:
//   1. validate: rank is a permutation of [0,n) and every endpoint id < n
//   2. relabel + orient: edge {a,b} -> (lo,hi) = (min, max)(rank[a], rank[b]);
//      self-loops dropped
//   3-4. forward CSR with sorted rows and repeated pairs dropped, built one
//      of two ways:
//      sort:    keys lo * 2^b + hi (2^b > n) sorted by a device radix sort;
//               equal neighbours dropped; row sizes from runs of equal lo
//      scatter: per-row counts of lo (atomics), scan, scatter hi into row
//               lo, sort each row, compact if some pairs repeated
//   5. backward CSR: keys hi * 2^b + lo sorted (sort), or count by target,
//      scan, scatter, sort rows (scatter)
//   6. inverse permutation inv[rank[u]] = u
// The sort way does no atomics on per-vertex counters, so hubs whose rows
// or columns are long cost no serialisation; its work is independent of
// the ordering.
#include "tl_internal.h"
#include "dev_util.h"
#include "timing.h"

namespace {

__global__ void k_rank_count(const u32 *rank, u32 n, u32 *cnt, u32 *flag) {
    GRID_STRIDE(i, n) {
        u32 r = rank[i];
        if (r >= n) atomicOr(flag, 1u);
        else atomicAdd(&cnt[r], 1u);
    }
}

__global__ void k_rank_verify(const u32 *cnt, u32 n, u32 *flag) {
    GRID_STRIDE(i, n) {
        if (cnt[i] != 1u) atomicOr(flag, 1u);
    }
}

__global__ void k_edge_verify(const u32 *src, const u32 *dst, u64 m_in, u32 n, u32 *flag) {
    GRID_STRIDE(i, m_in) {
        if (src[i] >= n || dst[i] >= n) atomicOr(flag, 2u);
    }
}

// rank and ids are validated before this runs
__global__ void k_row_count(const u32 *src, const u32 *dst, u64 m_in, const u32 *rank, u32 *cnt) {
    GRID_STRIDE(i, m_in) {
        u32 ra = rank[src[i]], rb = rank[dst[i]];
        if (ra != rb) atomicAdd(&cnt[ra < rb ? ra : rb], 1u);
    }
}

__global__ void k_row_scatter(const u32 *src, const u32 *dst, u64 m_in, const u32 *rank, const u64 *off,
                              u32 *cursor, u32 *adj, u32 *row) {
    GRID_STRIDE(i, m_in) {
        u32 ra = rank[src[i]], rb = rank[dst[i]];
        if (ra == rb) continue;
        u32 lo = ra < rb ? ra : rb, hi = ra < rb ? rb : ra;
        u64 pos = off[lo] + atomicAdd(&cursor[lo], 1u);
        adj[pos] = hi;
        row[pos] = lo;
    }
}

// keep the first uniq[row] entries of each raw row, at their new offsets
__global__ void k_compact_rows(const u64 *raw_off, const u32 *raw_adj, const u32 *raw_row, u64 nnz_raw,
                               const u32 *uniq, const u64 *off, u32 *adj, u32 *row) {
    GRID_STRIDE(j, nnz_raw) {
        u32 r = raw_row[j];
        u64 k = j - raw_off[r];
        if (k < uniq[r]) {
            adj[off[r] + k] = raw_adj[j];
            row[off[r] + k] = r;
        }
    }
}

__global__ void k_count_targets(const u32 *adj, u64 m, u32 *cnt) {
    GRID_STRIDE(j, m) { atomicAdd(&cnt[adj[j]], 1u); }
}

__global__ void k_transpose_scatter(const u32 *adj_f, const u32 *row_f, u64 m, const u64 *off_b, u32 *cursor,
                                    u32 *adj_b, u32 *row_b) {
    GRID_STRIDE(j, m) {
        u32 v = adj_f[j];
        u64 pos = off_b[v] + atomicAdd(&cursor[v], 1u);
        adj_b[pos] = row_f[j];
        row_b[pos] = v;
    }
}

// ---- the sort way

__global__ void k_fwd_keys(const u32 *src, const u32 *dst, u64 m_in, const u32 *rank, int b, u64 sent, u64 *keys) {
    GRID_STRIDE(i, m_in) {
        const u32 ra = rank[src[i]], rb = rank[dst[i]];
        keys[i] = ra == rb ? sent : (ra < rb ? ((u64)ra << b) | rb : ((u64)rb << b) | ra);
    }
}

// 1 for the first of each run of equal keys, sentinel (loops) excluded
__global__ void k_unique_flags(const u64 *keys, u64 n, u64 sent, u32 *flag) {
    GRID_STRIDE(i, n) {
        const u64 k = keys[i];
        flag[i] = (k != sent && (i == 0 || keys[i - 1] != k)) ? 1u : 0u;
    }
}

__global__ void k_fwd_emit(const u64 *keys, const u32 *flag, const u64 *pos, u64 n, int b, u32 *adj, u32 *row) {
    const u64 mask = (1ull << b) - 1;
    GRID_STRIDE(i, n) {
        if (flag[i]) {
            const u64 k = keys[i], j = pos[i];
            adj[j] = (u32)(k & mask);
            row[j] = (u32)(k >> b);
        }
    }
}

// cnt[r] += length of each run of r in the sorted array row[0..m): one
// atomic per run per wavefront
__global__ void k_run_count(const u32 *row, u64 m, u32 *cnt) {
    const int lane = lane_id();
    const u64 stride = (u64)gridDim.x * blockDim.x;
    const u64 first = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    const u64 iters = m > first - lane ? (m - (first - lane) + stride - 1) / stride : 0;  // wave-uniform
    for (u64 it = 0; it < iters; it++) {
        const u64 j = first + it * stride;
        const bool valid = j < m;
        const u32 key = valid ? row[j] : 0xffffffffu;
        u32 v = valid ? 1u : 0u;
#pragma unroll
        for (int d = 1; d < WAVE; d <<= 1) {
            const u32 t = __shfl_up(v, d, WAVE);
            const u32 q = __shfl_up(key, d, WAVE);
            if (lane >= d && q == key) v += t;
        }
        const u32 nk = __shfl_down(key, 1, WAVE);
        if (valid && (lane == WAVE - 1 || nk != key)) atomicAdd(&cnt[key], v);
    }
}

// backward keys: column above, the forward entry's index below (m < 2^32);
// a stable sort on the column field keeps each column's entries in forward
// order, i.e. by row
__global__ void k_bwd_keys(const u32 *adj_f, u64 m, u64 *keys) {
    GRID_STRIDE(j, m) { keys[j] = ((u64)adj_f[j] << 32) | (u32)j; }
}

__global__ void k_bwd_emit(const u64 *keys, u64 m, const u32 *row_f, u32 *adj_b, u32 *row_b, u32 *twin_b) {
    GRID_STRIDE(j, m) {
        const u64 k = keys[j];
        const u32 i = (u32)k;
        adj_b[j] = row_f[i];
        row_b[j] = (u32)(k >> 32);
        twin_b[j] = i;
    }
}

// twin_b[j] for a backward CSR built without the index: the position of the
// entry's row in its column vertex's successor list
__global__ void k_twin_search(const u64 *off_f, const u32 *adj_f, const u32 *adj_b, const u32 *row_b, u64 m,
                              u32 *twin_b) {
    GRID_STRIDE(j, m) {
        const u32 u = adj_b[j], v = row_b[j];
        twin_b[j] = (u32)lower_bound_dev<u32>(adj_f, off_f[u], off_f[u + 1], v);
    }
}

__global__ void k_inverse(const u32 *rank, u32 n, u32 *inv) {
    GRID_STRIDE(i, n) { inv[rank[i]] = (u32)i; }
}

unsigned grid_n(u64 items) { return grid_for(items, 256, (unsigned)tl_num_cus() * 16); }

struct CsrOwner {
    tl_csr *g;
    explicit CsrOwner(tl_csr *p) : g(p) {}
    ~CsrOwner() { if (g) tl_csr_free(g); }
    tl_csr *release() { tl_csr *p = g; g = nullptr; return p; }
};

}  // namespace

namespace {

// Steps 2-5 by sorting (see the file comment); cnt: n + 1 scratch counters.
void orient_sorted(tl_csr *g, u32 n, const u32 *src, const u32 *dst, u64 m_in, const u32 *rank, u32 *cnt,
                   hipStream_t s) {
    int b = 1;
    while ((1ull << b) <= (u64)n) b++;  // ids < n <= 2^b - 1: the all-ones key is free
    const u64 sent = 2 * b >= 64 ? ~0ull : (1ull << (2 * b)) - 1;
    const u64 mi = m_in ? m_in : 1;
    DevBuf keys(mi * sizeof(u64), s), tmp(mi * sizeof(u64), s);
    u64 m = 0;
    DevBuf pos((mi + 1) * sizeof(u64), s);
    if (m_in) {
        hipLaunchKernelGGL(k_fwd_keys, dim3(grid_n(m_in)), dim3(256), 0, s, src, dst, m_in, rank, b, sent,
                           keys.as<u64>());
        TL_HIP(hipGetLastError());
        const u64 *sorted = radix_sort_u64(keys.as<u64>(), tmp.as<u64>(), m_in, 0, 2 * b, s);
        u64 *other = sorted == keys.as<u64>() ? tmp.as<u64>() : keys.as<u64>();
        u32 *flag = reinterpret_cast<u32 *>(other);  // the other buffer is free now
        hipLaunchKernelGGL(k_unique_flags, dim3(grid_n(m_in)), dim3(256), 0, s, sorted, m_in, sent, flag);
        TL_HIP(hipGetLastError());
        scan_u32_to_u64(flag, pos.as<u64>(), m_in, s);
        d2h_sync(s, {{&m, pos.as<u64>() + m_in, sizeof(u64)}});
        g->m = m;
        g->adj_f = (u32 *)tl_dev_alloc((m ? m : 1) * sizeof(u32), s);
        g->row_f = (u32 *)tl_dev_alloc((m ? m : 1) * sizeof(u32), s);
        hipLaunchKernelGGL(k_fwd_emit, dim3(grid_n(m_in)), dim3(256), 0, s, sorted, flag, pos.as<u64>(), m_in, b,
                           g->adj_f, g->row_f);
        TL_HIP(hipGetLastError());
    } else {
        g->m = 0;
        g->adj_f = (u32 *)tl_dev_alloc(sizeof(u32), s);
        g->row_f = (u32 *)tl_dev_alloc(sizeof(u32), s);
    }
    if (n) TL_HIP(hipMemsetAsync(cnt, 0, (u64)n * sizeof(u32), s));
    if (m) {
        hipLaunchKernelGGL(k_run_count, dim3(grid_n(m)), dim3(256), 0, s, g->row_f, m, cnt);
        TL_HIP(hipGetLastError());
    }
    scan_u32_to_u64(cnt, g->off_f, n, s);
    // backward CSR: the same entries sorted by (hi, lo).  They are sorted by
    // (lo, hi) already, so a stable sort on the hi field alone suffices.
    g->adj_b = (u32 *)tl_dev_alloc((m ? m : 1) * sizeof(u32), s);
    g->row_b = (u32 *)tl_dev_alloc((m ? m : 1) * sizeof(u32), s);
    g->twin_b = (u32 *)tl_dev_alloc((m ? m : 1) * sizeof(u32), s);
    if (n) TL_HIP(hipMemsetAsync(cnt, 0, (u64)n * sizeof(u32), s));
    if (m) {
        hipLaunchKernelGGL(k_bwd_keys, dim3(grid_n(m)), dim3(256), 0, s, g->adj_f, m, keys.as<u64>());
        TL_HIP(hipGetLastError());
        const u64 *sorted = radix_sort_u64(keys.as<u64>(), tmp.as<u64>(), m, 32, b, s);
        hipLaunchKernelGGL(k_bwd_emit, dim3(grid_n(m)), dim3(256), 0, s, sorted, m, g->row_f, g->adj_b, g->row_b,
                           g->twin_b);
        TL_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_run_count, dim3(grid_n(m)), dim3(256), 0, s, g->row_b, m, cnt);
        TL_HIP(hipGetLastError());
    }
    scan_u32_to_u64(cnt, g->off_b, n, s);
}

}  // namespace

tl_csr *orient_impl(u32 n, const u32 *src, const u32 *dst, u64 m_in, const u32 *rank, hipStream_t s) {
    TL_REQUIRE(n < 0xffffffffu, TL_EINVAL, "n must be below 2^32 - 1");
    TL_REQUIRE(m_in < (1ull << 32), TL_EINVAL, "m_in must be below 2^32");
    TL_REQUIRE(n == 0 || rank, TL_EINVAL, "rank is NULL");
    TL_REQUIRE(m_in == 0 || (src && dst), TL_EINVAL, "src/dst is NULL");
    TL_REQUIRE(n > 0 || m_in == 0, TL_EINVAL, "edges given for an empty vertex set");

    PhaseTimer timer(TL_PHASE_ORIENT, s);
    // ---- 1. validation
    DevBuf cnt((u64)(n + 1) * sizeof(u32), s);
    DevBuf flag(sizeof(u32), s);
    TL_HIP(hipMemsetAsync(flag.p, 0, sizeof(u32), s));
    if (n) {
        TL_HIP(hipMemsetAsync(cnt.p, 0, (u64)n * sizeof(u32), s));
        hipLaunchKernelGGL(k_rank_count, dim3(grid_n(n)), dim3(256), 0, s, rank, n, cnt.as<u32>(), flag.as<u32>());
        TL_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_rank_verify, dim3(grid_n(n)), dim3(256), 0, s, cnt.as<u32>(), n, flag.as<u32>());
        TL_HIP(hipGetLastError());
    }
    if (m_in) {
        hipLaunchKernelGGL(k_edge_verify, dim3(grid_n(m_in)), dim3(256), 0, s, src, dst, m_in, n, flag.as<u32>());
        TL_HIP(hipGetLastError());
    }
    u32 h_flag = 0;
    d2h_sync(s, {{&h_flag, flag.p, sizeof(u32)}});
    TL_REQUIRE(!(h_flag & 1u), TL_EINVAL, "rank is not a permutation of [0, n)");
    TL_REQUIRE(!(h_flag & 2u), TL_EINVAL, "an edge endpoint is >= n");

    CsrOwner own(new tl_csr());
    tl_csr *g = own.g;
    g->n = n;
    TL_HIP(hipGetDevice(&g->device));
    g->off_f = (u64 *)tl_dev_alloc((u64)(n + 1) * sizeof(u64), s);
    g->off_b = (u64 *)tl_dev_alloc((u64)(n + 1) * sizeof(u64), s);
    g->inv = (u32 *)tl_dev_alloc((u64)(n ? n : 1) * sizeof(u32), s);

    if (orient_by_sort()) {
        orient_sorted(g, n, src, dst, m_in, rank, cnt.as<u32>(), s);
        if (n) {
            hipLaunchKernelGGL(k_inverse, dim3(grid_n(n)), dim3(256), 0, s, rank, n, g->inv);
            TL_HIP(hipGetLastError());
        }
        timer.stop();
        TL_HIP(hipStreamSynchronize(s));
        return own.release();
    }

    // ---- 2-3. count rows, scan, scatter
    u32 *rowcnt = cnt.as<u32>();
    if (n) TL_HIP(hipMemsetAsync(rowcnt, 0, (u64)n * sizeof(u32), s));
    if (m_in) {
        hipLaunchKernelGGL(k_row_count, dim3(grid_n(m_in)), dim3(256), 0, s, src, dst, m_in, rank, rowcnt);
        TL_HIP(hipGetLastError());
    }
    DevBuf raw_off((u64)(n + 1) * sizeof(u64), s);
    scan_u32_to_u64(rowcnt, raw_off.as<u64>(), n, s);
    u64 nnz_raw = 0;
    d2h_sync(s, {{&nnz_raw, raw_off.as<u64>() + n, sizeof(u64)}});

    u32 *raw_adj = (u32 *)tl_dev_alloc((nnz_raw ? nnz_raw : 1) * sizeof(u32), s);
    u32 *raw_row = (u32 *)tl_dev_alloc((nnz_raw ? nnz_raw : 1) * sizeof(u32), s);
    g->adj_f = raw_adj;  // owned by g from here (freed on error)
    g->row_f = raw_row;
    if (nnz_raw) {
        TL_HIP(hipMemsetAsync(rowcnt, 0, (u64)n * sizeof(u32), s));
        hipLaunchKernelGGL(k_row_scatter, dim3(grid_n(m_in)), dim3(256), 0, s, src, dst, m_in, rank,
                           raw_off.as<u64>(), rowcnt, raw_adj, raw_row);
        TL_HIP(hipGetLastError());
    }

    // ---- 4. sort rows, drop repeated pairs
    DevBuf uniq((u64)(n + 1) * sizeof(u32), s);
    segmented_sort_unique(raw_off.as<u64>(), n, raw_adj, nnz_raw, n, uniq.as<u32>(), s);
    scan_u32_to_u64(uniq.as<u32>(), g->off_f, n, s);
    u64 m = 0;
    d2h_sync(s, {{&m, g->off_f + n, sizeof(u64)}});
    g->m = m;
    if (m != nnz_raw) {
        u32 *adj = (u32 *)tl_dev_alloc((m ? m : 1) * sizeof(u32), s);
        u32 *row = (u32 *)tl_dev_alloc((m ? m : 1) * sizeof(u32), s);
        hipLaunchKernelGGL(k_compact_rows, dim3(grid_n(nnz_raw)), dim3(256), 0, s, raw_off.as<u64>(), raw_adj,
                           raw_row, nnz_raw, uniq.as<u32>(), g->off_f, adj, row);
        TL_HIP(hipGetLastError());
        tl_dev_free(raw_adj);  // stream-ordered reuse only
        tl_dev_free(raw_row);
        g->adj_f = adj;
        g->row_f = row;
    }

    // ---- 5. backward CSR (predecessor lists)
    g->adj_b = (u32 *)tl_dev_alloc((m ? m : 1) * sizeof(u32), s);
    g->row_b = (u32 *)tl_dev_alloc((m ? m : 1) * sizeof(u32), s);
    g->twin_b = (u32 *)tl_dev_alloc((m ? m : 1) * sizeof(u32), s);
    if (n) TL_HIP(hipMemsetAsync(rowcnt, 0, (u64)n * sizeof(u32), s));
    if (m) {
        hipLaunchKernelGGL(k_count_targets, dim3(grid_n(m)), dim3(256), 0, s, g->adj_f, m, rowcnt);
        TL_HIP(hipGetLastError());
    }
    scan_u32_to_u64(rowcnt, g->off_b, n, s);
    if (m) {
        TL_HIP(hipMemsetAsync(rowcnt, 0, (u64)n * sizeof(u32), s));
        hipLaunchKernelGGL(k_transpose_scatter, dim3(grid_n(m)), dim3(256), 0, s, g->adj_f, g->row_f, m, g->off_b,
                           rowcnt, g->adj_b, g->row_b);
        TL_HIP(hipGetLastError());
        segmented_sort_unique(g->off_b, n, g->adj_b, m, n, uniq.as<u32>(), s);
        hipLaunchKernelGGL(k_twin_search, dim3(grid_n(m)), dim3(256), 0, s, g->off_f, g->adj_f, g->adj_b, g->row_b,
                           m, g->twin_b);
        TL_HIP(hipGetLastError());
    }

    // ---- 6. inverse permutation
    if (n) {
        hipLaunchKernelGGL(k_inverse, dim3(grid_n(n)), dim3(256), 0, s, rank, n, g->inv);
        TL_HIP(hipGetLastError());
    }
    timer.stop();
    TL_HIP(hipStreamSynchronize(s));
    return own.release();
}
