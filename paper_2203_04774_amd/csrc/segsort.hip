// Row-wise sort + deduplication of a CSR whose rows hold vertex ranks.
//
// Rows are binned by length: rows of at most 64 entries are sorted inside a
// wavefront with a bitonic network over lanes (several short rows share a
// wavefront, one aligned lane segment each); longer rows are sorted by one
// workgroup with a stable LSD radix sort (8-bit digits, LDS histograms,
// ballot-based ranking), ping-ponging through a scratch copy of the row.
// In both cases the distinct values are packed at the start of the row and
// the distinct count is written to uniq[row].
#include "tl_internal.h"
#include "dev_util.h"

namespace {

constexpr int NBINS = 8;  // 0: len<=1, 1..6: segment 2..64, 7: long rows
constexpr int SORT_BLOCK = 256;

__device__ __forceinline__ int bin_of(u64 len) {
    if (len <= 1) return 0;
    if (len <= 2) return 1;
    if (len <= 4) return 2;
    if (len <= 8) return 3;
    if (len <= 16) return 4;
    if (len <= 32) return 5;
    if (len <= 64) return 6;
    return 7;
}

__global__ void k_bin_count(const u64 *off, u32 nrows, u32 *counts, u32 *uniq) {
    __shared__ u32 c[NBINS];
    if (threadIdx.x < NBINS) c[threadIdx.x] = 0;
    __syncthreads();
    GRID_STRIDE(r, nrows) {
        u64 len = off[r + 1] - off[r];
        int b = bin_of(len);
        if (b == 0) uniq[r] = (u32)len;
        else atomicAdd(&c[b], 1u);
    }
    __syncthreads();
    if (threadIdx.x < NBINS && c[threadIdx.x]) atomicAdd(&counts[threadIdx.x], c[threadIdx.x]);
}

// Block-aggregated: one global atomic per bin per block.
__global__ __launch_bounds__(256) void k_bin_fill(const u64 *off, u32 nrows, const u32 *bin_start, u32 *cursor,
                                                  u32 *rows) {
    __shared__ u32 cnt[NBINS], base[NBINS];
    const u64 stride = (u64)gridDim.x * blockDim.x;
    for (u64 r0 = (u64)blockIdx.x * blockDim.x; r0 < nrows; r0 += stride) {  // block-uniform
        if (threadIdx.x < NBINS) cnt[threadIdx.x] = 0;
        __syncthreads();
        const u64 r = r0 + threadIdx.x;
        int b = 0;
        u32 local = 0;
        if (r < nrows) {
            b = bin_of(off[r + 1] - off[r]);
            if (b) local = atomicAdd(&cnt[b], 1u);
        }
        __syncthreads();
        if (threadIdx.x < NBINS && cnt[threadIdx.x])
            base[threadIdx.x] = atomicAdd(&cursor[threadIdx.x], cnt[threadIdx.x]);
        __syncthreads();
        if (r < nrows && b) rows[bin_start[b] + base[b] + local] = (u32)r;
        __syncthreads();
    }
}

// One wavefront sorts 64/S rows at a time, S lanes per row.
template <int S>
__global__ __launch_bounds__(256) void k_sort_wave(const u32 *rows, u32 nrows, const u64 *off, u32 *adj,
                                                   u32 *uniq) {
    constexpr int R = WAVE / S;
    const int lane = lane_id();
    const int seg = lane / S, l = lane % S;
    const u64 wave = ((u64)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const u64 nwaves = ((u64)gridDim.x * blockDim.x) / WAVE;
    const u64 segmask = (S == 64 ? ~0ull : ((1ull << S) - 1)) << (seg * S);
    for (u64 base = wave * R; base < nrows; base += nwaves * R) {
        const u64 ri = base + seg;
        const bool has = ri < nrows;
        const u32 r = has ? rows[ri] : 0;
        const u64 s0 = has ? off[r] : 0;
        const u32 len = has ? (u32)(off[r + 1] - s0) : 0;
        u32 v = (l < (int)len) ? adj[s0 + l] : 0xffffffffu;
#pragma unroll
        for (int k = 2; k <= S; k <<= 1) {
#pragma unroll
            for (int j = k >> 1; j > 0; j >>= 1) {
                u32 p = __shfl_xor(v, j, WAVE);
                bool up = (l & k) == 0;
                bool lower = (l & j) == 0;
                u32 mn = v < p ? v : p, mx = v < p ? p : v;
                v = (lower == up) ? mn : mx;
            }
        }
        u32 prev = __shfl_up(v, 1, WAVE);
        bool keep = (l < (int)len) && (l == 0 || v != prev);
        u64 bal = __ballot(keep);
        u32 idx = __popcll(bal & segmask & lanemask_lt());
        if (keep) adj[s0 + idx] = v;
        if (has && l == 0) uniq[r] = __popcll(bal & segmask);
    }
}

// One workgroup per long row: stable LSD radix sort, then in-place unique.
__global__ __launch_bounds__(SORT_BLOCK) void k_sort_block(const u32 *rows, u32 nrows, const u64 *off, u32 *adj,
                                                           u32 *tmp, u32 *uniq, int bits) {
    constexpr int NW = SORT_BLOCK / WAVE;
    __shared__ u32 hist[256];
    __shared__ u32 base[256];
    __shared__ u32 wcnt[NW][256];
    __shared__ u64 lds64[NW];
    const int t = threadIdx.x, lane = lane_id(), wid = t / WAVE;
    for (u32 bi = blockIdx.x; bi < nrows; bi += gridDim.x) {
        const u32 r = rows[bi];
        const u64 s0 = off[r];
        const u32 len = (u32)(off[r + 1] - s0);
        u32 *src = adj + s0, *dst = tmp + s0;
        for (int sh = 0; sh < bits; sh += 8) {
            hist[t] = 0;
            __syncthreads();
            for (u32 i = t; i < len; i += SORT_BLOCK) atomicAdd(&hist[(src[i] >> sh) & 255u], 1u);
            __syncthreads();
            u64 tot;
            u64 ex = block_excl_scan_u64<SORT_BLOCK>(hist[t], lds64, tot);
            base[t] = (u32)ex;
            __syncthreads();
            for (u32 t0 = 0; t0 < len; t0 += SORT_BLOCK) {
                const u32 i = t0 + t;
                const bool valid = i < len;
                const u32 v = valid ? src[i] : 0u;
                const u32 d = (v >> sh) & 255u;
                u64 mask = __ballot(valid);
#pragma unroll
                for (int b = 0; b < 8; b++) {
                    u64 bb = __ballot((d >> b) & 1u);
                    mask &= ((d >> b) & 1u) ? bb : ~bb;
                }
                const u32 rk = __popcll(mask & lanemask_lt());
#pragma unroll
                for (int w = 0; w < NW; w++) wcnt[w][t] = 0;
                __syncthreads();
                if (valid && rk == 0) wcnt[wid][d] = __popcll(mask);
                __syncthreads();
                if (valid) {
                    u32 o = base[d] + rk;
                    for (int w = 0; w < wid; w++) o += wcnt[w][d];
                    dst[o] = v;
                }
                __syncthreads();
                u32 add = 0;
#pragma unroll
                for (int w = 0; w < NW; w++) add += wcnt[w][t];
                base[t] += add;
                __syncthreads();
            }
            u32 *sw = src; src = dst; dst = sw;
        }
        // sorted values are in src; pack distinct ones at adj + s0
        u32 *out = adj + s0;
        u32 run = 0;
        for (u32 t0 = 0; t0 < len; t0 += SORT_BLOCK) {
            const u32 i = t0 + t;
            const bool valid = i < len;
            const u32 v = valid ? src[i] : 0u;
            const bool keep = valid && (i == 0 || v != src[i - 1]);
            u64 tot;
            u64 ex = block_excl_scan_u64<SORT_BLOCK>(keep ? 1 : 0, lds64, tot);  // synchronises
            if (keep) out[run + ex] = v;
            run += (u32)tot;
            __syncthreads();
        }
        if (t == 0) uniq[r] = run;
        __syncthreads();
    }
}

template <int S>
void launch_wave(const u32 *rows, u32 cnt, const u64 *off, u32 *adj, u32 *uniq, hipStream_t s) {
    if (!cnt) return;
    const u64 waves = (cnt + (WAVE / S) - 1) / (WAVE / S);
    const unsigned blocks = grid_for(waves * WAVE, 256, (unsigned)tl_num_cus() * 16);
    hipLaunchKernelGGL((k_sort_wave<S>), dim3(blocks), dim3(256), 0, s, rows, cnt, off, adj, uniq);
    TL_HIP(hipGetLastError());
}

}  // namespace

void segmented_sort_unique(const u64 *off, u32 nrows, u32 *adj, u64 nnz, u32 n_values, u32 *uniq,
                           hipStream_t s) {
    if (nrows == 0) return;
    DevBuf counts(2 * NBINS * sizeof(u32), s);
    TL_HIP(hipMemsetAsync(counts.p, 0, 2 * NBINS * sizeof(u32), s));
    u32 *d_counts = counts.as<u32>(), *d_cursor = d_counts + NBINS;
    const unsigned g = grid_for(nrows, 256, (unsigned)tl_num_cus() * 8);
    hipLaunchKernelGGL(k_bin_count, dim3(g), dim3(256), 0, s, off, nrows, d_counts, uniq);
    TL_HIP(hipGetLastError());
    u32 h_counts[NBINS];
    d2h_sync(s, {{h_counts, d_counts, sizeof h_counts}});
    u32 h_start[NBINS];
    u64 total = 0;
    for (int b = 0; b < NBINS; b++) { h_start[b] = (u32)total; total += h_counts[b]; }
    if (total == 0) return;
    DevBuf rows(total * sizeof(u32), s), starts(NBINS * sizeof(u32), s);
    h2d_sync(starts.p, h_start, sizeof h_start, s);
    hipLaunchKernelGGL(k_bin_fill, dim3(g), dim3(256), 0, s, off, nrows, starts.as<u32>(), d_cursor,
                       rows.as<u32>());
    TL_HIP(hipGetLastError());
    const u32 *R = rows.as<u32>();
    launch_wave<2>(R + h_start[1], h_counts[1], off, adj, uniq, s);
    launch_wave<4>(R + h_start[2], h_counts[2], off, adj, uniq, s);
    launch_wave<8>(R + h_start[3], h_counts[3], off, adj, uniq, s);
    launch_wave<16>(R + h_start[4], h_counts[4], off, adj, uniq, s);
    launch_wave<32>(R + h_start[5], h_counts[5], off, adj, uniq, s);
    launch_wave<64>(R + h_start[6], h_counts[6], off, adj, uniq, s);
    if (h_counts[7]) {
        int bits = 1;
        while (bits < 32 && (1ull << bits) < (u64)n_values) bits++;
        DevBuf tmp(nnz * sizeof(u32), s);
        const unsigned blocks = h_counts[7] < (u32)tl_num_cus() * 8 ? h_counts[7] : (u32)tl_num_cus() * 8;
        hipLaunchKernelGGL(k_sort_block, dim3(blocks), dim3(SORT_BLOCK), 0, s, R + h_start[7], h_counts[7], off,
                           adj, tmp.as<u32>(), uniq, bits);
        TL_HIP(hipGetLastError());
    }
}
