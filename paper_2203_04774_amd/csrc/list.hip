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
// side of x).  The plan step computes that window per seed edge, compacts
// the non-empty ones and prefix-sums their lengths; the probe step then
// gives every lane exactly one scanned element (perfect load balance over
// the flattened work), which it looks up in T by binary search.
#include "tl_internal.h"
#include "dev_util.h"
#include "timing.h"

namespace {

struct GView {
    const u64 *off_f, *off_b;
    const u32 *adj_f, *adj_b, *row_f, *row_b, *inv;
    u64 m;
};

// Seed-edge geometry for the three forms.
template <int ALGO>
struct Seed {
    u32 p, x;          // pivot and the seed edge's other endpoint
    const u32 *S;      // scanned list base (S[s_lo .. s_hi))
    u64 s_lo, s_hi;
    const u32 *T;      // target array, candidates T[t_lo .. t_hi)
    u64 t_lo, t_hi;
    __device__ __forceinline__ Seed(const GView &g, u64 e) {
        if (ALGO == 0) {
            p = g.row_b[e]; x = g.adj_b[e];
            S = g.adj_f; s_lo = g.off_f[x]; s_hi = g.off_f[x + 1];
            T = g.adj_b; t_lo = e + 1; t_hi = g.off_b[p + 1];
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

constexpr int PB = 256;

template <int ALGO>
__global__ __launch_bounds__(PB) void k_plan(GView g, u32 plo, u32 phi, u32 *len, u32 *start, u32 *flag,
                                             u64 *acc) {
    __shared__ u64 lds[PB / WAVE];
    u64 work = 0;
    GRID_STRIDE(e, g.m) {
        Seed<ALGO> sd(g, e);
        u32 l = 0, st = 0;
        if (sd.p >= plo && sd.p < phi) {
            work += sd.s_hi - sd.s_lo;
            if (sd.t_lo < sd.t_hi && sd.s_lo < sd.s_hi) {
                u32 tmin = sd.T[sd.t_lo], tmax = sd.T[sd.t_hi - 1];
                u64 a = lower_bound_dev<u32>(sd.S, sd.s_lo, sd.s_hi, tmin);
                u64 b = upper_bound_dev<u32>(sd.S, a, sd.s_hi, tmax);
                l = (u32)(b - a);
                st = (u32)(a - sd.s_lo);
            }
        }
        len[e] = l;
        start[e] = st;
        flag[e] = l ? 1u : 0u;
    }
    u64 tot = block_sum_u64<PB>(work, lds);
    if (threadIdx.x == 0 && tot) atomicAdd((unsigned long long *)&acc[2], (unsigned long long)tot);
}

__global__ void k_compact_seeds(const u32 *len, const u32 *start, const u64 *pos, u64 m, u32 *cseed, u32 *cstart,
                                u32 *clen) {
    GRID_STRIDE(e, m) {
        u32 l = len[e];
        if (l) {
            u64 p = pos[e];
            cseed[p] = (u32)e;
            cstart[p] = start[e];
            clen[p] = l;
        }
    }
}

// acc: [0] count, [1] digest, [2] paper work, [3] output cursor
template <int ALGO, bool EMIT>
__global__ __launch_bounds__(PB) void k_probe(GView g, const u32 *cseed, const u32 *cstart, const u64 *cpre,
                                              u64 ncap, u64 k0, u64 k1, u32 *tri, u64 cap, u64 *acc) {
    const int lane = lane_id();
    const u64 gw = ((u64)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const u64 nw = ((u64)gridDim.x * blockDim.x) / WAVE;
    const u64 span = k1 - k0;
    const u64 per = (((span + nw - 1) / nw) + WAVE - 1) & ~(u64)(WAVE - 1);
    const u64 wb = k0 + gw * per;
    const u64 we = (wb + per < k1) ? wb + per : k1;
    u64 cnt = 0, hsh = 0;
    if (wb < we) {
        // seed of the wave's first item: last c with cpre[c] <= wb
        u64 c_lo = upper_bound_dev<u64>(cpre, 0, ncap + 1, wb) - 1;
        for (u64 kb = wb; kb < we; kb += WAVE) {
            const u64 k = kb + lane;
            const bool act = k < we;
            const u64 P = (c_lo + lane <= ncap) ? cpre[c_lo + lane] : ~0ull;
            int lo = 0;
#pragma unroll
            for (int st = 32; st > 0; st >>= 1) {
                u64 pv = shfl_u64(P, lo + st);
                if (pv <= k) lo += st;
            }
            const u64 c = c_lo + lo;
            const u64 rel = k - shfl_u64(P, lo);
            bool hit = false;
            u32 a = 0, b = 0, cc = 0;
            if (act) {
                const u64 e = cseed[c];
                Seed<ALGO> sd(g, e);
                const u32 y = sd.S[sd.s_lo + cstart[c] + rel];
                const u64 j = lower_bound_dev<u32>(sd.T, sd.t_lo, sd.t_hi, y);
                if (j < sd.t_hi && sd.T[j] == y) {
                    hit = true;
                    a = g.inv[sd.p]; b = g.inv[sd.x]; cc = g.inv[y];
                    canon3(a, b, cc);
                    cnt += 1;
                    hsh += tri_digest(a, b, cc);
                }
            }
            if (EMIT) {
                const u64 bal = __ballot(hit);
                if (bal) {
                    u64 base = 0;
                    if (lane == 0) base = atomicAdd((unsigned long long *)&acc[3], (unsigned long long)__popcll(bal));
                    base = shfl_u64(base, 0);
                    if (hit) {
                        const u64 pos = base + __popcll(bal & lanemask_lt());
                        if (pos < cap) {
                            tri[3 * pos + 0] = a;
                            tri[3 * pos + 1] = b;
                            tri[3 * pos + 2] = cc;
                        }
                    }
                }
            }
            // seed of the next chunk's first item
            const u64 c_last = shfl_u64(c, WAVE - 1);
            const u64 nk = kb + WAVE;
            if (nk < we) {
                c_lo = c_last;
                if (c_lo + 1 <= ncap && cpre[c_lo + 1] <= nk) c_lo++;
            }
        }
    }
    cnt = wave_sum_u64(cnt);
    hsh = wave_sum_u64(hsh);
    if (lane == 0 && cnt) {
        atomicAdd((unsigned long long *)&acc[0], (unsigned long long)cnt);
        atomicAdd((unsigned long long *)&acc[1], (unsigned long long)hsh);
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

GView view_of(const tl_csr *g) {
    return GView{g->off_f, g->off_b, g->adj_f, g->adj_b, g->row_f, g->row_b, g->inv, g->m};
}

template <int ALGO>
void launch_plan(const GView &v, u32 plo, u32 phi, u32 *len, u32 *start, u32 *flag, u64 *acc, hipStream_t s) {
    hipLaunchKernelGGL((k_plan<ALGO>), dim3(grid_for(v.m, PB, (unsigned)tl_num_cus() * 16)), dim3(PB), 0, s, v, plo,
                       phi, len, start, flag, acc);
    TL_HIP(hipGetLastError());
}

template <int ALGO>
void launch_probe(const GView &v, const u32 *cseed, const u32 *cstart, const u64 *cpre, u64 k0, u64 k1, u32 *tri,
                  u64 cap, bool emit, u64 *acc, hipStream_t s) {
    const u64 waves_needed = (k1 - k0 + WAVE - 1) / WAVE;
    const unsigned max_blocks = (unsigned)tl_num_cus() * 8;
    u64 blocks = (waves_needed + (PB / WAVE) - 1) / (PB / WAVE);
    if (blocks > max_blocks) blocks = max_blocks;
    if (blocks < 1) blocks = 1;
    if (emit)
        hipLaunchKernelGGL((k_probe<ALGO, true>), dim3((unsigned)blocks), dim3(PB), 0, s, v, cseed, cstart, cpre,
                           v.m, k0, k1, tri, cap, acc);
    else
        hipLaunchKernelGGL((k_probe<ALGO, false>), dim3((unsigned)blocks), dim3(PB), 0, s, v, cseed, cstart, cpre,
                           v.m, k0, k1, tri, cap, acc);
    TL_HIP(hipGetLastError());
}

}  // namespace

u64 chunk_triangles() { return g_chunk_triangles; }
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
    TL_HIP(hipMemcpyAsync(&h, out.p, sizeof(u64), hipMemcpyDeviceToHost, s));
    TL_HIP(hipStreamSynchronize(s));
    return h;
}

int list_impl(const tl_csr *g, int algo, u32 plo, u32 phi, u32 *tri, u64 cap, tl_chunk_fn cb, void *user,
              hipStream_t s, tl_summary *out) {
    *out = tl_summary{0, 0, 0, 0};
    const u64 m = g->m;
    if (phi > g->n) phi = g->n;
    if (m == 0 || plo >= phi) return TL_OK;
    const GView v = view_of(g);

    DevBuf acc(4 * sizeof(u64), s);
    TL_HIP(hipMemsetAsync(acc.p, 0, 4 * sizeof(u64), s));
    u64 *d_acc = acc.as<u64>();

    // ---- plan: window per seed edge, compaction, work prefix
    PhaseTimer plan_timer(TL_PHASE_PLAN, s);
    DevBuf len(m * sizeof(u32), s), start(m * sizeof(u32), s), flag(m * sizeof(u32), s);
    DevBuf pos((m + 1) * sizeof(u64), s);
    if (algo == 0) launch_plan<0>(v, plo, phi, len.as<u32>(), start.as<u32>(), flag.as<u32>(), d_acc, s);
    else if (algo == 1) launch_plan<1>(v, plo, phi, len.as<u32>(), start.as<u32>(), flag.as<u32>(), d_acc, s);
    else launch_plan<2>(v, plo, phi, len.as<u32>(), start.as<u32>(), flag.as<u32>(), d_acc, s);
    scan_u32_to_u64(flag.as<u32>(), pos.as<u64>(), m, s);
    DevBuf cseed(m * sizeof(u32), s), cstart(m * sizeof(u32), s);
    u32 *clen = flag.as<u32>();  // flags are consumed by the scan above; reuse as compacted lengths
    TL_HIP(hipMemsetAsync(clen, 0, m * sizeof(u32), s));
    hipLaunchKernelGGL(k_compact_seeds, dim3(grid_for(m, 256, (unsigned)tl_num_cus() * 16)), dim3(256), 0, s,
                       len.as<u32>(), start.as<u32>(), pos.as<u64>(), m, cseed.as<u32>(), cstart.as<u32>(), clen);
    TL_HIP(hipGetLastError());
    DevBuf cpre((m + 1) * sizeof(u64), s);
    scan_u32_to_u64(clen, cpre.as<u64>(), m, s);
    plan_timer.stop();
    u64 h_total = 0, h_work = 0;
    TL_HIP(hipMemcpyAsync(&h_total, cpre.as<u64>() + m, sizeof(u64), hipMemcpyDeviceToHost, s));
    TL_HIP(hipMemcpyAsync(&h_work, d_acc + 2, sizeof(u64), hipMemcpyDeviceToHost, s));
    TL_HIP(hipStreamSynchronize(s));
    out->work = h_work;
    out->scanned = h_total;

    auto probe = [&](u64 k0, u64 k1, u32 *dst, u64 dcap, bool emit) {
        PhaseTimer t(TL_PHASE_PROBE, s);
        if (algo == 0) launch_probe<0>(v, cseed.as<u32>(), cstart.as<u32>(), cpre.as<u64>(), k0, k1, dst, dcap, emit, d_acc, s);
        else if (algo == 1) launch_probe<1>(v, cseed.as<u32>(), cstart.as<u32>(), cpre.as<u64>(), k0, k1, dst, dcap, emit, d_acc, s);
        else launch_probe<2>(v, cseed.as<u32>(), cstart.as<u32>(), cpre.as<u64>(), k0, k1, dst, dcap, emit, d_acc, s);
    };

    int rc = TL_OK;
    u64 h_acc[4] = {0, 0, 0, 0};
    if (h_total == 0) {
        // nothing to scan
    } else if (tri) {
        probe(0, h_total, tri, cap, true);
        TL_HIP(hipMemcpyAsync(h_acc, d_acc, sizeof h_acc, hipMemcpyDeviceToHost, s));
        TL_HIP(hipStreamSynchronize(s));
        if (h_acc[0] > cap) rc = TL_ECAPACITY;
    } else if (cb) {
        // each scanned element yields at most one triangle, so a slice of K
        // work items always fits a chunk of K triangles
        const u64 K = g_chunk_triangles;
        DevBuf chunk(K * 3 * sizeof(u32), s);
        for (u64 k0 = 0; k0 < h_total; k0 += K) {
            const u64 k1 = (h_total - k0 > K) ? k0 + K : h_total;
            TL_HIP(hipMemsetAsync(d_acc + 3, 0, sizeof(u64), s));
            probe(k0, k1, chunk.as<u32>(), K, true);
            u64 got = 0;
            TL_HIP(hipMemcpyAsync(&got, d_acc + 3, sizeof(u64), hipMemcpyDeviceToHost, s));
            TL_HIP(hipStreamSynchronize(s));
            if (got && cb(chunk.as<u32>(), got, user) != 0) { rc = TL_EABORT; break; }
        }
        TL_HIP(hipMemcpyAsync(h_acc, d_acc, sizeof h_acc, hipMemcpyDeviceToHost, s));
        TL_HIP(hipStreamSynchronize(s));
    } else {
        probe(0, h_total, nullptr, 0, false);
        TL_HIP(hipMemcpyAsync(h_acc, d_acc, sizeof h_acc, hipMemcpyDeviceToHost, s));
        TL_HIP(hipStreamSynchronize(s));
    }
    out->count = h_acc[0];
    out->hash = h_acc[1];
    return rc;
}
