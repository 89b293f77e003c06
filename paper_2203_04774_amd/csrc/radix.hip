// Device-wide stable LSD radix sort of 64-bit keys, 8-bit digits.
//
// Each pass: every tile of RT keys counts its digits in LDS (k_rs_hist,
// counts stored digit-major so that one exclusive scan gives every tile's
// global offset per digit); then each wavefront of the tile ranks its own
// contiguous run of keys by digit with ballots against per-wavefront digit
// counters (stable: key order is kept within a digit), the counters become
// offsets, the tile's keys are staged sorted in LDS and each digit's run is
// written to its global segment, so that consecutive lanes write
// consecutive addresses.
#include "tl_internal.h"
#include "dev_util.h"

namespace {

#ifndef TL_RS_THREADS
#define TL_RS_THREADS 512
#endif
constexpr int RB = TL_RS_THREADS;  // threads per tile (512: 8,192 keys, 32 per digit on average, so
                                   // longer runs per output line; RMAT-26 orientation 178 -> 173 ms)
constexpr int RI = 16;             // keys per thread
constexpr u32 RT = RB * RI;        // keys per tile
constexpr int RD = 256;            // digit values
constexpr int RNW = RB / WAVE;
static_assert(RB >= RD && RB % RD == 0, "radix tile: at least one thread per digit");

__global__ __launch_bounds__(RB) void k_rs_hist(const u64 *keys, u64 n, int sh, u32 *counts, u64 ntiles) {
    __shared__ u32 h[RD];
    const int t = threadIdx.x;
    if (t < RD) h[t] = 0;
    __syncthreads();
    const u64 base = (u64)blockIdx.x * RT;
#pragma unroll
    for (int j = 0; j < RI; j++) {
        const u64 i = base + (u64)j * RB + t;
        if (i < n) atomicAdd(&h[(keys[i] >> sh) & 255u], 1u);
    }
    __syncthreads();
    if (t < RD) counts[(u64)t * ntiles + blockIdx.x] = h[t];
}

__global__ __launch_bounds__(RB) void k_rs_scatter(const u64 *in, u64 *out, u64 n, int sh, const u32 *counts,
                                                   const u64 *offs, u64 ntiles) {
    __shared__ u64 stage[RT];
    __shared__ u32 tbase[RD];
    __shared__ u32 wcnt[RNW][RD];  // per wavefront: keys of each digit seen so far, then its offset
    __shared__ u64 gbase[RD];
    __shared__ u64 lds64[RNW];
    const int t = threadIdx.x, lane = lane_id(), wid = t / WAVE;
    const u64 tile = blockIdx.x;
    const u64 base = tile * RT;
    const u32 cnt = (u32)(n - base < RT ? n - base : RT);
    {
        const u32 c = t < RD ? counts[(u64)t * ntiles + tile] : 0u;
        u64 tot;
        const u32 tb = (u32)block_excl_scan_u64<RB>(c, lds64, tot);
        if (t < RD) {
            tbase[t] = tb;
            gbase[t] = offs[(u64)t * ntiles + tile];
#pragma unroll
            for (int w = 0; w < RNW; w++) wcnt[w][t] = 0;
        }
    }
    __syncthreads();
    // Each wavefront takes a contiguous run of RI * 64 keys (coalesced
    // loads) and ranks them round by round against its own digit counters;
    // one wavefront's LDS operations run in order, so no barrier is needed.
    const u64 wbase = base + (u64)wid * (RI * WAVE);
    u64 k[RI];
    u32 rk[RI];
#pragma unroll
    for (int r = 0; r < RI; r++) {
        const u64 i = wbase + (u64)r * WAVE + lane;
        const bool valid = i < n;
        k[r] = valid ? in[i] : 0ull;
        const u32 d = (u32)(k[r] >> sh) & 255u;
        u64 mask = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            const u64 bb = __ballot((d >> b) & 1u);
            mask &= ((d >> b) & 1u) ? bb : ~bb;
        }
        const u32 below = __popcll(mask & lanemask_lt());
        wave_lds_fence();
        const u32 seen = wcnt[wid][d];
        rk[r] = seen + below;
        wave_lds_fence();
        if (valid && below == 0) wcnt[wid][d] = seen + (u32)__popcll(mask);
        wave_lds_fence();
    }
    __syncthreads();
    // offset of each wavefront's block of digit d inside the tile's run of d
    if (t < RD) {
        u32 acc = tbase[t];
#pragma unroll
        for (int w = 0; w < RNW; w++) {
            const u32 c = wcnt[w][t];
            wcnt[w][t] = acc;
            acc += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RI; r++) {
        const u64 i = wbase + (u64)r * WAVE + lane;
        if (i < n) {
            const u32 d = (u32)(k[r] >> sh) & 255u;
            stage[wcnt[wid][d] + rk[r]] = k[r];
        }
    }
    __syncthreads();
    for (u32 j = t; j < cnt; j += RB) {
        const u64 key = stage[j];
        const u32 d = (u32)(key >> sh) & 255u;
        out[gbase[d] + (j - tbase[d])] = key;
    }
}

}  // namespace

u64 *radix_sort_u64(u64 *keys, u64 *tmp, u64 n, int lo_bit, int bits, hipStream_t s) {
    if (n <= 1 || bits <= 0) return keys;
    const u64 ntiles = (n + RT - 1) / RT;
    TL_REQUIRE(ntiles < (1ull << 31), TL_EINVAL, "radix sort: too many keys");
    DevBuf counts((u64)RD * ntiles * sizeof(u32), s), offs(((u64)RD * ntiles + 1) * sizeof(u64), s);
    DevBuf ws((scan_workspace_words((u64)RD * ntiles) + 1) * sizeof(u64), s);
    u64 *src = keys, *dst = tmp;
    for (int sh = lo_bit; sh < lo_bit + bits; sh += 8) {
        hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)ntiles), dim3(RB), 0, s, src, n, sh, counts.as<u32>(), ntiles);
        TL_HIP(hipGetLastError());
        scan_u32_to_u64(counts.as<u32>(), offs.as<u64>(), (u64)RD * ntiles, s, ws.as<u64>());
        hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)ntiles), dim3(RB), 0, s, src, dst, n, sh, counts.as<u32>(),
                           offs.as<u64>(), ntiles);
        TL_HIP(hipGetLastError());
        u64 *sw = src;
        src = dst;
        dst = sw;
    }
    return src;
}
