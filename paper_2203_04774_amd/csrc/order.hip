// Orderings computed on the device from an oriented graph: the degree
// ordering (Section 2.2: non-decreasing degree, ties by id), Split
// (Section 3.3.3: the non-increasing degree ordering dealt alternately to
// the front and the back), the core ordering (Section 1.3: non-decreasing
// coreness, ties by id; coreness by level-synchronous peeling) and Check
// (Section 3.3.2: by non-increasing degree, each vertex after the beginning
// block or before the end block, whichever gives it the smaller C+- share;
// decided level by level, see below).  Together with tl_orient and tl_list
// they make the full listing (ordering included) run on the GPU.

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

// (key, id) pairs packed as key << 32 | id for the library's radix sort
__global__ void k_pack_keys(const u32 *key, const u32 *ids, u32 n, u64 *out) {
    GRID_STRIDE(i, n) { out[i] = ((u64)key[i] << 32) | ids[i]; }
}

__global__ void k_low32(const u64 *in, u32 n, u32 *out) {
    GRID_STRIDE(i, n) { out[i] = (u32)in[i]; }
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

// Start of a level: the level is the smallest degree left (*plevel, from
// k_core_min); every vertex still present with that degree leaves now with
// coreness `level` (one atomic per wavefront for the frontier's size).
__global__ void k_core_frontier(u32 n, const u32 *deg, u32 *core, const u32 *plevel, u32 *frontier, u32 *fcount) {
    const u32 level = *plevel;
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

constexpr int VB = 256;  // threads per frontier vertex (one workgroup each)

// appends the lanes' ready vertices to out (one atomic per wavefront)
__device__ __forceinline__ void wave_push(bool ready, u32 w, u32 *out, u32 *count) {
    const u64 bal = __ballot(ready);
    if (!bal) return;
    u32 base = 0;
    if (lane_id() == 0) base = atomicAdd(count, (u32)__popcll(bal));
    base = __shfl(base, 0, WAVE);
    if (ready) out[base + __popcll(bal & lanemask_lt())] = w;
}

// The frontier's vertices leave, a workgroup per vertex (hubs' lists are
// shared by its 256 threads): every neighbour still present loses one
// degree, and the one whose degree drops to `level` leaves next, with
// coreness `level` (exactly one decrement sees the drop).
__global__ __launch_bounds__(VB) void k_core_peel(const u64 *off_f, const u32 *adj_f, const u64 *off_b,
                                                  const u32 *adj_b, const u32 *frontier, u32 nf, u32 level,
                                                  u32 *core, u32 *deg, u32 *next, u32 *ncount) {
    for (u32 f = blockIdx.x; f < nf; f += gridDim.x) {
        const u32 r = frontier[f];
        const u64 f0 = off_f[r], nfw = off_f[r + 1] - f0, b0 = off_b[r];
        const u64 d = nfw + (off_b[r + 1] - b0);
        const u64 trips = (d + VB - 1) / VB;  // the same for the whole workgroup
        for (u64 t = 0; t < trips; t++) {
            const u64 j = t * VB + threadIdx.x;
            bool ready = false;
            u32 w = 0;
            if (j < d) {
                w = j < nfw ? adj_f[f0 + j] : adj_b[b0 + (j - nfw)];
                if (core[w] == UNSET && atomicSub(&deg[w], 1u) == level + 1) {
                    core[w] = level;
                    ready = true;
                }
            }
            wave_push(ready, w, next, ncount);
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

// ------------------------------------------------------------------ Check
//
// A vertex's choice depends only on the sides of its neighbours taken
// before it, so the sequential greedy is replayed exactly by levels: a
// vertex is decided once every earlier neighbour is (pending = 0), and the
// vertices of one level share no edge.  Positions follow from the sides:
// beginning vertices in the order taken, end vertices in reverse.

constexpr unsigned char SIDE_BEGIN = 0, SIDE_END = 1;

// dpos[r]: when rank r is taken (0 = first, the largest degree)
__global__ void k_check_dpos(const u32 *sorted, const u32 *inv, u32 n, u32 *posid, u32 *dpos, int phase) {
    GRID_STRIDE(i, n) {
        if (phase == 0) posid[sorted[i]] = (u32)i;
        else dpos[i] = n - 1 - posid[inv[i]];
    }
}

// pending[r] = neighbours taken before r: each edge counts once for its
// later end (edge-parallel, so hubs cost no more than other vertices)
__global__ void k_check_pending(const u32 *row_f, const u32 *adj_f, u64 m, const u32 *dpos, u32 *pending) {
    GRID_STRIDE(i, m) {
        const u32 u = row_f[i], v = adj_f[i];
        atomicAdd(&pending[dpos[u] < dpos[v] ? v : u], 1u);
    }
}

// ranks with no earlier neighbour start the first level
__global__ void k_check_first(const u32 *pending, u32 n, u32 *frontier, u32 *fcount) {
    const u64 stride = (u64)gridDim.x * blockDim.x;
    const u64 first = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    const u64 iters = (u64)n > first - lane_id() ? ((u64)n - (first - lane_id()) + stride - 1) / stride : 0;
    for (u64 it = 0; it < iters; it++) {
        const u64 r = first + it * stride;
        wave_push(r < n && pending[r] == 0, (u32)r, frontier, fcount);
    }
}

// One level, a workgroup per vertex: count the vertex's earlier neighbours
// on each side, take the cheaper side, then release its later neighbours
// (those whose last earlier neighbour this was join the next level).
__global__ __launch_bounds__(VB) void k_check_level(const u64 *off_f, const u32 *adj_f, const u64 *off_b,
                                                    const u32 *adj_b, const u32 *dpos, const u32 *frontier, u32 nf,
                                                    unsigned char *side, u32 *pending, u32 *next, u32 *ncount) {
    __shared__ u64 part[2][VB / WAVE];
    __shared__ unsigned char sd;
    const int lane = lane_id(), wid = (int)wave_id();
    for (u32 f = blockIdx.x; f < nf; f += gridDim.x) {
        const u32 r = frontier[f];
        const u32 d = dpos[r];
        const u64 f0 = off_f[r], nfw = off_f[r + 1] - f0, b0 = off_b[r];
        const u64 deg = nfw + (off_b[r + 1] - b0);
        u64 nb = 0, ne = 0;
        for (u64 j = threadIdx.x; j < deg; j += VB) {
            const u32 w = j < nfw ? adj_f[f0 + j] : adj_b[b0 + (j - nfw)];
            if (dpos[w] < d) {
                if (side[w] == SIDE_BEGIN) nb++;
                else ne++;
            }
        }
        nb = wave_sum_u64(nb);
        ne = wave_sum_u64(ne);
        if (lane == 0) {
            part[0][wid] = nb;
            part[1][wid] = ne;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            u64 tb = 0, te = 0;
            for (int w = 0; w < VB / WAVE; w++) {
                tb += part[0][w];
                te += part[1][w];
            }
            const u64 nq = deg - tb - te;
            sd = tb * (te + nq) <= (tb + nq) * te ? SIDE_BEGIN : SIDE_END;
            side[r] = sd;
        }
        __syncthreads();
        const u64 trips = (deg + VB - 1) / VB;
        for (u64 t = 0; t < trips; t++) {
            const u64 j = t * VB + threadIdx.x;
            bool ready = false;
            u32 w = 0;
            if (j < deg) {
                w = j < nfw ? adj_f[f0 + j] : adj_b[b0 + (j - nfw)];
                if (dpos[w] > d) ready = atomicSub(&pending[w], 1u) == 1u;
            }
            wave_push(ready, w, next, ncount);
        }
        __syncthreads();  // part[] and sd are reused by the next vertex
    }
}

// begin[i] = 1 when the vertex taken i-th went to the beginning
__global__ void k_check_flags(const u32 *dpos, const unsigned char *side, u32 n, u32 *begin) {
    GRID_STRIDE(r, n) { begin[dpos[r]] = side[r] == SIDE_BEGIN ? 1u : 0u; }
}

// beginning: position = beginning vertices taken before; end: n - 1 minus
// the end vertices taken before
__global__ void k_check_rank(const u32 *dpos, const unsigned char *side, const u64 *bpre, const u32 *inv, u32 n,
                             u32 *rank) {
    GRID_STRIDE(r, n) {
        const u32 i = dpos[r];
        const u64 b = bpre[i];
        rank[inv[r]] = side[r] == SIDE_BEGIN ? (u32)b : (u32)(n - 1 - (i - b));
    }
}

}  // namespace

// Coreness of every rank by level-synchronous peeling, then keys (coreness
// per vertex id) and ids for the sort.
void coreness_keys(const tl_csr *g, u32 *key, u32 *ids, hipStream_t s) {
    const u32 n = g->n;
    DevBuf deg((u64)n * 4, s), core((u64)n * 4, s), fa((u64)n * 4, s), fb((u64)n * 4, s), cnt(8, s);
    u32 *fcount = cnt.as<u32>(), *mind = cnt.as<u32>() + 1;
    u32 *cur = fa.as<u32>(), *nxt = fb.as<u32>();
    hipLaunchKernelGGL(k_rank_degree, dim3(grid_o(n)), dim3(256), 0, s, g->off_f, g->off_b, n, deg.as<u32>(),
                       core.as<u32>());
    TL_HIP(hipGetLastError());
    u64 remaining = n;
    bool first = true;
    u32 level = 0;
    while (remaining) {
        // the next level is the smallest degree left (above the last level:
        // every vertex at or below it has left); its vertices are gathered
        // on the device, one host wait per level
        TL_HIP(hipMemsetAsync(cnt.p, 0, 4, s));
        TL_HIP(hipMemsetAsync(mind, 0xff, 4, s));
        hipLaunchKernelGGL(k_core_min, dim3(grid_o(n)), dim3(256), 0, s, n, deg.as<u32>(), core.as<u32>(), mind);
        TL_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_core_frontier, dim3(grid_o(n)), dim3(256), 0, s, n, deg.as<u32>(), core.as<u32>(), mind,
                           cur, fcount);
        TL_HIP(hipGetLastError());
        u32 st[2] = {0, 0};
        d2h_sync(s, {{st, cnt.p, 8}});
        u32 nf = st[0];
        TL_REQUIRE(nf > 0 && st[1] != UNSET && (first || st[1] > level), TL_EHIP, "core peeling made no progress");
        level = st[1];
        first = false;
        // peel: every round's leavers bring the next ones down to `level`
        while (nf) {
            remaining -= nf;
            TL_HIP(hipMemsetAsync(fcount, 0, 4, s));
            hipLaunchKernelGGL(k_core_peel, dim3(nf < 65536 ? nf : 65536), dim3(VB), 0, s, g->off_f, g->adj_f,
                               g->off_b, g->adj_b, cur, nf, level, core.as<u32>(), deg.as<u32>(), nxt, fcount);
            TL_HIP(hipGetLastError());
            d2h_sync(s, {{&nf, fcount, 4}});
            std::swap(cur, nxt);
        }
    }
    hipLaunchKernelGGL(k_core_keys, dim3(grid_o(n)), dim3(256), 0, s, core.as<u32>(), g->inv, n, key, ids);
    TL_HIP(hipGetLastError());
}

// Check's ranks from the degree ordering's `sorted` (ids by non-decreasing
// degree, ties by id), read backwards as the order in which vertices are taken.
void check_ranks(const tl_csr *g, const u32 *sorted, u32 *rank, hipStream_t s) {
    const u32 n = g->n;
    DevBuf posid((u64)n * 4, s), dpos((u64)n * 4, s), pending((u64)n * 4, s), fa((u64)n * 4, s),
        fb((u64)n * 4, s), side((u64)n, s), cnt(8, s), bpre(((u64)n + 1) * 8, s);
    for (int phase = 0; phase < 2; phase++) {
        hipLaunchKernelGGL(k_check_dpos, dim3(grid_o(n)), dim3(256), 0, s, sorted, g->inv, n, posid.as<u32>(),
                           dpos.as<u32>(), phase);
        TL_HIP(hipGetLastError());
    }
    TL_HIP(hipMemsetAsync(cnt.p, 0, 8, s));
    TL_HIP(hipMemsetAsync(pending.p, 0, (u64)n * 4, s));
    if (g->m) {
        hipLaunchKernelGGL(k_check_pending, dim3(grid_o(g->m)), dim3(256), 0, s, g->row_f, g->adj_f, g->m,
                           dpos.as<u32>(), pending.as<u32>());
        TL_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_check_first, dim3(grid_o(n)), dim3(256), 0, s, pending.as<u32>(), n, fa.as<u32>(),
                       cnt.as<u32>());
    TL_HIP(hipGetLastError());
    u32 nf = 0;
    d2h_sync(s, {{&nf, cnt.p, 4}});
    u32 *cur = fa.as<u32>(), *nxt = fb.as<u32>();
    u64 done = 0;
    while (nf) {
        done += nf;
        TL_HIP(hipMemsetAsync(cnt.p, 0, 4, s));
        hipLaunchKernelGGL(k_check_level, dim3(nf < 65536 ? nf : 65536), dim3(VB), 0, s, g->off_f, g->adj_f,
                           g->off_b, g->adj_b, dpos.as<u32>(), cur, nf, side.as<unsigned char>(), pending.as<u32>(),
                           nxt, cnt.as<u32>());
        TL_HIP(hipGetLastError());
        d2h_sync(s, {{&nf, cnt.p, 4}});
        std::swap(cur, nxt);
    }
    TL_REQUIRE(done == n, TL_EHIP, "Check levels did not reach every vertex");
    hipLaunchKernelGGL(k_check_flags, dim3(grid_o(n)), dim3(256), 0, s, dpos.as<u32>(), side.as<unsigned char>(), n,
                       posid.as<u32>());
    TL_HIP(hipGetLastError());
    scan_u32_to_u64(posid.as<u32>(), bpre.as<u64>(), n, s);
    hipLaunchKernelGGL(k_check_rank, dim3(grid_o(n)), dim3(256), 0, s, dpos.as<u32>(), side.as<unsigned char>(),
                       bpre.as<u64>(), g->inv, n, rank);
    TL_HIP(hipGetLastError());
}

void order_impl(const tl_csr *g, int kind, u32 *rank, hipStream_t s) {
    TL_REQUIRE(kind >= 0 && kind <= 3, TL_EINVAL, "unknown ordering");
    const u32 n = g->n;
    if (n == 0) return;
    TL_REQUIRE(rank, TL_EINVAL, "rank is NULL");
    PhaseTimer timer(TL_PHASE_ORDER, s);
    DevBuf deg((u64)n * 4, s), ids((u64)n * 4, s), sorted((u64)n * 4, s), mx(4, s);
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
    // stable LSD radix sort (radix.hip) of the (degree, id) pairs on the
    // degree field: the pairs start in increasing id order, so ties keep it
    {
        DevBuf keys((u64)n * 8, s), ktmp((u64)n * 8, s);
        hipLaunchKernelGGL(k_pack_keys, dim3(grid_o(n)), dim3(256), 0, s, deg.as<u32>(), ids.as<u32>(), n,
                           keys.as<u64>());
        TL_HIP(hipGetLastError());
        const u64 *sk = radix_sort_u64(keys.as<u64>(), ktmp.as<u64>(), n, 32, bits, s);
        hipLaunchKernelGGL(k_low32, dim3(grid_o(n)), dim3(256), 0, s, sk, n, sorted.as<u32>());
        TL_HIP(hipGetLastError());
    }
    if (kind == 3) {
        check_ranks(g, sorted.as<u32>(), rank, s);
    } else {
        hipLaunchKernelGGL(k_rank_of, dim3(grid_o(n)), dim3(256), 0, s, sorted.as<u32>(), n, kind == 1 ? 1 : 0,
                           rank);
        TL_HIP(hipGetLastError());
    }
    timer.stop();
    TL_HIP(hipStreamSynchronize(s));
}
