// Internal declarations shared by the HIP translation units of libtl.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <initializer_list>
#include <string>

#include "tl.h"

typedef uint64_t u64;
typedef uint32_t u32;

// ------------------------------------------------------------ error plumbing

struct TlError {
    int code;
    std::string msg;
};

void tl_set_error(const std::string &msg);

#define TL_HIP(call)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            throw TlError{TL_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)};   \
        } while (0)

#define TL_REQUIRE(cond, code, text)                                                     \
    do {                                                                                 \
        if (!(cond)) throw TlError{(code), (text)};                                      \
    } while (0)

// ------------------------------------------------------------ device memory

// Device memory comes from a caching pool with one free list per stream: a
// block returned while kernels on stream s may still use it is only handed
// out again to work on the same stream, which runs after those kernels.
// Blocks are released to the driver only by tl_release_cached_memory().
void *pool_get(size_t bytes, hipStream_t s);
void pool_put(void *p);
void pool_trim();

// Scratch owned by one library call, returned to the pool at scope exit.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    hipStream_t s = nullptr;
    DevBuf() = default;
    DevBuf(size_t b, hipStream_t st) : bytes(b), s(st) { alloc(); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p(o.p), bytes(o.bytes), s(o.s) { o.p = nullptr; }
    DevBuf &operator=(DevBuf &&o) noexcept {
        release();
        p = o.p; bytes = o.bytes; s = o.s; o.p = nullptr;
        return *this;
    }
    ~DevBuf() { release(); }
    void alloc() { if (bytes) p = pool_get(bytes, s); }
    void release() { if (p) pool_put(p); p = nullptr; }
    template <class T> T *as() const { return static_cast<T *>(p); }
};

// A device arena installed on the calling thread for the length of one
// library call: while one is installed, pool_get carves 256-byte aligned
// blocks from it in order (blocks are not reused within the call) and throws
// TL_ECAPACITY once it is exhausted, pool_put leaves its blocks alone, and
// d2h_sync / h2d_sync copy directly instead of through the pinned staging
// buffer (whose first use allocates).  Used by the entry point that
// allocates nothing.
struct ScratchArena {
    char *base;
    size_t size;
    size_t used;
};
ScratchArena *&thread_arena();
struct ArenaScope {
    ScratchArena *prev;
    explicit ArenaScope(ScratchArena *a) : prev(thread_arena()) { thread_arena() = a; }
    ~ArenaScope() { thread_arena() = prev; }
    ArenaScope(const ArenaScope &) = delete;
    ArenaScope &operator=(const ArenaScope &) = delete;
};
// Bytes of every device block a count-only listing of a graph with n
// vertices and m edges takes from the pool, heavy tasks excepted (their
// number is known only after the plan; they are taken after a host wait).
u64 list_count_scratch_bytes(u64 n, u64 m);

// Long-lived allocation (graph storage), also pooled.
void *tl_dev_alloc(size_t bytes, hipStream_t s);
void tl_dev_free(void *p);

// Small host<->device transfers through a pinned staging area.
struct D2H {
    void *host;
    const void *dev;
    size_t bytes;
};
// Enqueue the copies on s, wait for the stream, then fill the host buffers.
void d2h_sync(hipStream_t s, std::initializer_list<D2H> copies);
// Copy host bytes to the device through pinned staging (waits for s).
void h2d_sync(void *dev, const void *host, size_t bytes, hipStream_t s);

// ------------------------------------------------------------ the handle

struct tl_csr {
    u32 n = 0;
    u64 m = 0;
    int device = 0;
    u64 *off_f = nullptr;  // n+1: forward CSR offsets (rank space)
    u32 *adj_f = nullptr;  // m:   successor ranks, rows ascending
    u32 *row_f = nullptr;  // m:   row (source rank) of each forward entry
    u64 *off_b = nullptr;  // n+1: backward CSR offsets
    u32 *adj_b = nullptr;  // m:   predecessor ranks, rows ascending
    u32 *row_b = nullptr;  // m:   row (target rank) of each backward entry
    u32 *twin_b = nullptr; // m:   index in adj_f of each backward entry's edge
    u32 *inv = nullptr;    // n:   inv[r] = vertex of rank r
};

// ------------------------------------------------------------ launch helpers

int tl_num_cus();

inline unsigned grid_for(u64 items, unsigned block, unsigned max_blocks = 65535u * 4u) {
    u64 g = (items + block - 1) / block;
    if (g < 1) g = 1;
    if (g > max_blocks) g = max_blocks;
    return (unsigned)g;
}

// exclusive scan: out[i] = sum_{j<i} in[j] for i in [0, n]; out[n] = total.
// ws: scratch of scan_workspace_words(n) u64, or NULL to use the pool.
void scan_u32_to_u64(const u32 *in, u64 *out, u64 n, hipStream_t s, u64 *ws = nullptr);
void scan_u64_to_u64(const u64 *in, u64 *out, u64 n, hipStream_t s, u64 *ws = nullptr);
u64 scan_workspace_words(u64 n);

// Stable ascending sort of n 64-bit keys by bits [lo_bit, lo_bit + bits)
// (radix.hip); tmp holds n keys of scratch; returns whichever of keys/tmp
// holds the result.
u64 *radix_sort_u64(u64 *keys, u64 *tmp, u64 n, int lo_bit, int bits, hipStream_t s);

// Sort every row of a CSR ascending and drop repeated values inside a row;
// uniq[r] receives the row's distinct count and the distinct values are
// packed at the start of the row.  Values must be < n_values.
void segmented_sort_unique(const u64 *off, u32 nrows, u32 *adj, u64 nnz, u32 n_values, u32 *uniq,
                           hipStream_t s);

// Orientation and listing drivers (orient.hip, list.hip).
bool orient_by_sort();  // tuning key orient_sort
tl_csr *orient_impl(u32 n, const u32 *src, const u32 *dst, u64 m_in, const u32 *rank, hipStream_t s);
u64 cost_impl(const tl_csr *g, int algo, hipStream_t s);
int list_impl(const tl_csr *g, int algo, u32 plo, u32 phi, u32 *tri, u64 cap, tl_chunk_fn cb, void *user,
              hipStream_t s, tl_summary *out);
u64 chunk_triangles();
int set_tuning(const char *key, u64 value);
tl_list_stats &last_stats();
int get_tuning(const char *key, u64 *value);
void set_chunk_triangles(u64 k);

// Batched listing (batch.hip).
tl_batch *batch_orient_impl(u32 k, const u32 *n, const u64 *m, const u32 *src, const u32 *dst, const u32 *rank,
                            hipStream_t s);
// A batch whose union is built from k graphs already oriented (their arrays
// copied with shifted ranks and indices; the graphs stay the caller's).
tl_batch *batch_from_csrs_impl(u32 k, const tl_csr *const *gs, hipStream_t s);
void batch_list_impl(tl_batch *b, int algo, hipStream_t s, int use_graph, u64 *per_graph_host, u64 *per_graph_dev);
// device_sync: wait for the whole device first (else the caller has
// synchronised every stream that used the batch).
void batch_free_impl(tl_batch *b, bool device_sync);
const tl_csr *batch_csr(const tl_batch *b);
// Launch parameters of the batched pass (keys batch_*).
int batch_set_tuning(const std::string &key, u64 value);
int batch_get_tuning(const std::string &key, u64 *value);
void batch_sizes(const tl_batch *b, u32 *k, u32 *n, u64 *m);

// Listing server (serve.hip).
tl_server *server_create_impl(const tl_server_config *cfg);
u64 server_submit_impl(tl_server *S, const tl_job *job);
int server_poll_impl(tl_server *S, u64 id, int64_t wait_us, tl_job_result *out);
int server_cancel_impl(tl_server *S, u64 id);
void server_pause_impl(tl_server *S, bool paused);
void server_stats_impl(tl_server *S, tl_server_stats *out);
void server_destroy_impl(tl_server *S);
u64 job_bytes(u64 n, u64 m);

// Cached device bytes (in use and free) of the current device's pool, and a
// trim of its free blocks when that total exceeds `limit`.
u64 pool_total_bytes();
void pool_trim_above(u64 limit);

// Orderings from an oriented graph (order.hip): kind 0 degree, 1 Split.
void order_impl(const tl_csr *g, int kind, u32 *rank, hipStream_t s);
void neigh_impl(const tl_csr *g, double eps, u32 max_passes, u32 max_visits, u32 *rank_dev, tl_neigh_result *res,
                hipStream_t s);
