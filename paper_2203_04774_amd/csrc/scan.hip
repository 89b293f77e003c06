// Device-wide exclusive prefix sums (reduce, scan the block sums, scan
// again with the block offset).  Used for CSR offsets and work prefixes.
#include "tl_internal.h"
#include "dev_util.h"

namespace {

constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 8;
constexpr u64 SCAN_TILE = (u64)SCAN_BLOCK * SCAN_ITEMS;

template <class T>
__global__ __launch_bounds__(SCAN_BLOCK) void k_tile_sums(const T *in, u64 n, u64 *sums) {
    __shared__ u64 lds[SCAN_BLOCK / WAVE];
    const u64 base = (u64)blockIdx.x * SCAN_TILE;
    u64 v = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; j++) {
        u64 i = base + (u64)j * SCAN_BLOCK + threadIdx.x;  // coalesced
        if (i < n) v += (u64)in[i];
    }
    u64 t = block_sum_u64<SCAN_BLOCK>(v, lds);
    if (threadIdx.x == 0) sums[blockIdx.x] = t;
}

// `add` (may be NULL) holds one offset per tile.
template <class T>
__global__ __launch_bounds__(SCAN_BLOCK) void k_tile_scan(const T *in, u64 n, const u64 *add, u64 *out) {
    __shared__ u64 lds[SCAN_BLOCK / WAVE];
    const u64 base = (u64)blockIdx.x * SCAN_TILE + (u64)threadIdx.x * SCAN_ITEMS;  // blocked
    u64 x[SCAN_ITEMS];
    u64 local = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; j++) {
        u64 i = base + j;
        x[j] = (i < n) ? (u64)in[i] : 0;
        local += x[j];
    }
    u64 total;
    u64 run = block_excl_scan_u64<SCAN_BLOCK>(local, lds, total);
    if (add) run += add[blockIdx.x];
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; j++) {
        u64 i = base + j;
        if (i < n) out[i] = run;
        run += x[j];
    }
    // the thread holding the last element also writes out[n]
    if (n > 0 && base <= n - 1 && n - 1 < base + SCAN_ITEMS) out[n] = run;
}

__global__ void k_set_zero(u64 *p) { *p = 0; }

// Scratch (u64 words) a scan of n elements needs for its tile sums.
u64 scan_ws_words(u64 n) {
    u64 tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (tiles <= 1) return 0;
    return tiles + (tiles + 1) + scan_ws_words(tiles);
}

// ws: caller scratch of scan_ws_words(n) words, or NULL to take it from the
// pool (a scan into caller scratch allocates nothing and can be captured).
template <class T>
void scan_impl(const T *in, u64 *out, u64 n, hipStream_t s, u64 *ws) {
    if (n == 0) {
        hipLaunchKernelGGL(k_set_zero, dim3(1), dim3(1), 0, s, out);
        TL_HIP(hipGetLastError());
        return;
    }
    u64 tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    TL_REQUIRE(tiles < (1ull << 31), TL_EINVAL, "scan: input too large");
    if (tiles == 1) {
        hipLaunchKernelGGL((k_tile_scan<T>), dim3(1), dim3(SCAN_BLOCK), 0, s, in, n, (const u64 *)nullptr, out);
        TL_HIP(hipGetLastError());
        return;
    }
    DevBuf own;
    if (!ws) {
        own = DevBuf(scan_ws_words(n) * sizeof(u64), s);
        ws = own.as<u64>();
    }
    u64 *sums = ws, *offs = ws + tiles, *rest = ws + tiles + (tiles + 1);
    hipLaunchKernelGGL((k_tile_sums<T>), dim3((unsigned)tiles), dim3(SCAN_BLOCK), 0, s, in, n, sums);
    TL_HIP(hipGetLastError());
    scan_impl<u64>(sums, offs, tiles, s, rest);
    hipLaunchKernelGGL((k_tile_scan<T>), dim3((unsigned)tiles), dim3(SCAN_BLOCK), 0, s, in, n, (const u64 *)offs,
                       out);
    TL_HIP(hipGetLastError());
}

}  // namespace

void scan_u32_to_u64(const u32 *in, u64 *out, u64 n, hipStream_t s, u64 *ws) { scan_impl<u32>(in, out, n, s, ws); }
void scan_u64_to_u64(const u64 *in, u64 *out, u64 n, hipStream_t s, u64 *ws) { scan_impl<u64>(in, out, n, s, ws); }
u64 scan_workspace_words(u64 n) { return scan_ws_words(n); }
