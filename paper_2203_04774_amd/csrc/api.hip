// C-ABI entry points of libtl (declared in include/tl.h).  Each call
// validates its arguments on the host, runs the HIP pipeline on the
// caller's stream and converts every failure into a status code.
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "tl_internal.h"

namespace {

thread_local std::string g_last_error;

int g_num_cus = 0;

template <class F>
int guarded(F &&f) {
    try {
        return f();
    } catch (const TlError &e) {
        g_last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return TL_ENOMEM;
    } catch (...) {
        g_last_error = "unexpected exception";
        return TL_EHIP;
    }
}

}  // namespace

void tl_set_error(const std::string &msg) { g_last_error = msg; }

int tl_num_cus() {
    if (!g_num_cus) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            g_num_cus = cus;
        else
            g_num_cus = 256;
    }
    return g_num_cus;
}

// ---------------------------------------------------------------- pool

namespace {

struct Pool {
    std::mutex mu;
    std::map<hipStream_t, std::multimap<size_t, void *>> free_;   // per stream, by size
    std::unordered_map<void *, std::pair<size_t, hipStream_t>> live_;
    std::vector<std::pair<void *, size_t>> all_;
};

Pool &pool_of(int dev) {
    static std::mutex mu;
    static std::map<int, Pool *> pools;
    std::lock_guard<std::mutex> lk(mu);
    Pool *&p = pools[dev];
    if (!p) p = new Pool();  // lives until process exit
    return *p;
}

size_t round_bytes(size_t b) {
    const size_t g = b < (1u << 20) ? 256 : (size_t)2 << 20;
    return (b + g - 1) / g * g;
}

}  // namespace

ScratchArena *&thread_arena() {
    thread_local ScratchArena *a = nullptr;
    return a;
}

void *pool_get(size_t bytes, hipStream_t s) {
    if (ScratchArena *a = thread_arena()) {
        const size_t b = ((bytes ? bytes : 1) + 255) & ~(size_t)255;
        TL_REQUIRE(b <= a->size - a->used, TL_ECAPACITY,
                   "no-allocation scratch exhausted: " + std::to_string(a->used + b) + " bytes needed, " +
                       std::to_string(a->size) + " available");
        void *p = a->base + a->used;
        a->used += b;
        return p;
    }
    int dev = 0;
    TL_HIP(hipGetDevice(&dev));
    Pool &P = pool_of(dev);
    bytes = round_bytes(bytes ? bytes : 1);
    std::lock_guard<std::mutex> lk(P.mu);
    auto &fl = P.free_[s];
    auto it = fl.lower_bound(bytes);
    if (it != fl.end() && it->first <= 2 * bytes) {
        void *p = it->second;
        P.live_[p] = {it->first, s};
        fl.erase(it);
        return p;
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        // give cached blocks of every stream back to the driver and retry
        (void)hipGetLastError();
        (void)hipDeviceSynchronize();
        for (auto &kv : P.free_)
            for (auto &blk : kv.second) {
                (void)hipFree(blk.second);
                for (size_t i = 0; i < P.all_.size(); i++)
                    if (P.all_[i].first == blk.second) { P.all_.erase(P.all_.begin() + i); break; }
            }
        P.free_.clear();
        e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            throw TlError{TL_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed"};
        }
    }
    P.live_[p] = {bytes, s};
    P.all_.push_back({p, bytes});
    return p;
}

void pool_put(void *p) {
    if (!p) return;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    Pool &P = pool_of(dev);
    std::lock_guard<std::mutex> lk(P.mu);
    auto it = P.live_.find(p);
    if (it == P.live_.end()) return;
    P.free_[it->second.second].insert({it->second.first, p});
    P.live_.erase(it);
}

void pool_trim() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    Pool &P = pool_of(dev);
    std::lock_guard<std::mutex> lk(P.mu);
    (void)hipDeviceSynchronize();
    for (auto &kv : P.free_)
        for (auto &blk : kv.second) {
            (void)hipFree(blk.second);
            for (size_t i = 0; i < P.all_.size(); i++)
                if (P.all_[i].first == blk.second) { P.all_.erase(P.all_.begin() + i); break; }
        }
    P.free_.clear();
}

u64 pool_total_bytes() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    Pool &P = pool_of(dev);
    std::lock_guard<std::mutex> lk(P.mu);
    u64 t = 0;
    for (auto &a : P.all_) t += a.second;
    return t;
}

void pool_trim_above(u64 limit) {
    if (pool_total_bytes() > limit) pool_trim();
}

void *tl_dev_alloc(size_t bytes, hipStream_t s) { return pool_get(bytes, s); }
void tl_dev_free(void *p) { pool_put(p); }

// ------------------------------------------------------- pinned staging

namespace {
constexpr size_t STAGE_BYTES = 4u << 20;

// One pinned buffer per thread, released when the thread ends.
struct Stage {
    char *buf = nullptr;
    ~Stage() {
        if (buf) (void)hipHostFree(buf);
    }
};

char *stage_buffer() {
    thread_local Stage st;
    if (!st.buf) {
        void *p = nullptr;
        if (hipHostMalloc(&p, STAGE_BYTES, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            throw TlError{TL_ENOMEM, "pinned staging allocation failed"};
        }
        st.buf = static_cast<char *>(p);
    }
    return st.buf;
}
}  // namespace

void d2h_sync(hipStream_t s, std::initializer_list<D2H> copies) {
    size_t total = 0;
    for (const D2H &c : copies) total += (c.bytes + 15) & ~size_t(15);
    if (total > STAGE_BYTES || thread_arena()) {
        for (const D2H &c : copies)
            if (c.bytes) TL_HIP(hipMemcpyAsync(c.host, c.dev, c.bytes, hipMemcpyDeviceToHost, s));
        TL_HIP(hipStreamSynchronize(s));
        return;
    }
    char *st = stage_buffer();
    size_t off = 0;
    for (const D2H &c : copies) {
        if (c.bytes) TL_HIP(hipMemcpyAsync(st + off, c.dev, c.bytes, hipMemcpyDeviceToHost, s));
        off += (c.bytes + 15) & ~size_t(15);
    }
    TL_HIP(hipStreamSynchronize(s));
    off = 0;
    for (const D2H &c : copies) {
        if (c.bytes) memcpy(c.host, st + off, c.bytes);
        off += (c.bytes + 15) & ~size_t(15);
    }
}

void h2d_sync(void *dev, const void *host, size_t bytes, hipStream_t s) {
    if (!bytes) return;
    if (bytes > STAGE_BYTES || thread_arena()) {
        TL_HIP(hipMemcpyAsync(dev, host, bytes, hipMemcpyHostToDevice, s));
        TL_HIP(hipStreamSynchronize(s));
        return;
    }
    char *st = stage_buffer();
    TL_HIP(hipStreamSynchronize(s));  // staging may still feed an earlier copy
    memcpy(st, host, bytes);
    TL_HIP(hipMemcpyAsync(dev, st, bytes, hipMemcpyHostToDevice, s));
    TL_HIP(hipStreamSynchronize(s));
}

extern "C" {

int tl_orient(uint32_t n, const uint32_t *src, const uint32_t *dst, uint64_t m_in, const uint32_t *rank,
              void *stream, tl_csr **out) {
    return guarded([&] {
        TL_REQUIRE(out, TL_EINVAL, "out is NULL");
        *out = nullptr;
        *out = orient_impl(n, src, dst, m_in, rank, (hipStream_t)stream);
        return TL_OK;
    });
}

int tl_cost(const tl_csr *g, tl_algo a, void *stream, uint64_t *cost) {
    return guarded([&] {
        TL_REQUIRE(g && cost, TL_EINVAL, "NULL argument");
        TL_REQUIRE(a == TL_APP || a == TL_APM || a == TL_AMM, TL_EINVAL, "unknown algorithm");
        *cost = cost_impl(g, (int)a, (hipStream_t)stream);
        return TL_OK;
    });
}

int tl_list_range(const tl_csr *g, tl_algo a, uint32_t pivot_lo, uint32_t pivot_hi, uint32_t *tri_dev,
                  uint64_t cap_triangles, tl_chunk_fn cb, void *user, void *stream, tl_summary *out) {
    return guarded([&] {
        TL_REQUIRE(g && out, TL_EINVAL, "NULL argument");
        TL_REQUIRE(a == TL_APP || a == TL_APM || a == TL_AMM, TL_EINVAL, "unknown algorithm");
        TL_REQUIRE(!(tri_dev && cb), TL_EINVAL, "give either an output buffer or a chunk callback");
        return list_impl(g, (int)a, pivot_lo, pivot_hi, tri_dev, cap_triangles, cb, user, (hipStream_t)stream, out);
    });
}

int tl_list(const tl_csr *g, tl_algo a, uint32_t *tri_dev, uint64_t cap_triangles, tl_chunk_fn cb, void *user,
            void *stream, tl_summary *out) {
    return tl_list_range(g, a, 0u, 0xffffffffu, tri_dev, cap_triangles, cb, user, stream, out);
}

int tl_csr_size(const tl_csr *g, uint32_t *n, uint64_t *m) {
    return guarded([&] {
        TL_REQUIRE(g, TL_EINVAL, "NULL handle");
        if (n) *n = g->n;
        if (m) *m = g->m;
        return TL_OK;
    });
}

int tl_csr_copy_to_host(const tl_csr *g, uint64_t *off_fwd, uint32_t *adj_fwd, uint64_t *off_bwd, uint32_t *adj_bwd,
                        uint32_t *inv) {
    return guarded([&] {
        TL_REQUIRE(g, TL_EINVAL, "NULL handle");
        TL_HIP(hipDeviceSynchronize());
        const size_t no = ((size_t)g->n + 1) * sizeof(uint64_t), na = (size_t)g->m * sizeof(uint32_t);
        if (off_fwd) TL_HIP(hipMemcpy(off_fwd, g->off_f, no, hipMemcpyDeviceToHost));
        if (off_bwd) TL_HIP(hipMemcpy(off_bwd, g->off_b, no, hipMemcpyDeviceToHost));
        if (adj_fwd && na) TL_HIP(hipMemcpy(adj_fwd, g->adj_f, na, hipMemcpyDeviceToHost));
        if (adj_bwd && na) TL_HIP(hipMemcpy(adj_bwd, g->adj_b, na, hipMemcpyDeviceToHost));
        if (inv && g->n) TL_HIP(hipMemcpy(inv, g->inv, (size_t)g->n * sizeof(uint32_t), hipMemcpyDeviceToHost));
        return TL_OK;
    });
}

void tl_csr_free(tl_csr *g) {
    if (!g) return;
    tl_dev_free(g->off_f);
    tl_dev_free(g->adj_f);
    tl_dev_free(g->row_f);
    tl_dev_free(g->off_b);
    tl_dev_free(g->adj_b);
    tl_dev_free(g->row_b);
    tl_dev_free(g->twin_b);
    tl_dev_free(g->inv);
    delete g;
}

int tl_set_tuning(const char *key, uint64_t value) {
    return guarded([&] {
        TL_REQUIRE(key, TL_EINVAL, "NULL key");
        const int rc = set_tuning(key, value);
        TL_REQUIRE(rc == TL_OK, TL_EINVAL, std::string("unknown tuning key or value out of range: ") + key);
        return TL_OK;
    });
}

int tl_get_tuning(const char *key, uint64_t *value) {
    return guarded([&] {
        TL_REQUIRE(key && value, TL_EINVAL, "NULL argument");
        const int rc = get_tuning(key, value);
        TL_REQUIRE(rc == TL_OK, TL_EINVAL, std::string("unknown tuning key: ") + key);
        return TL_OK;
    });
}

int tl_last_list_stats(tl_list_stats *out) {
    if (!out) return TL_EINVAL;
    *out = last_stats();
    return TL_OK;
}

int tl_release_cached_memory(void) {
    return guarded([&] {
        pool_trim();
        return TL_OK;
    });
}

int tl_set_chunk_triangles(uint64_t k) {
    if (k == 0 || k > (1ull << 32)) {
        g_last_error = "chunk size must be in [1, 2^32]";
        return TL_EINVAL;
    }
    set_chunk_triangles(k);
    return TL_OK;
}

const char *tl_strerror(int code) {
    switch (code) {
        case TL_OK: return "ok";
        case TL_EINVAL: return "invalid argument";
        case TL_ENOMEM: return "out of device memory";
        case TL_ECAPACITY: return "output buffer too small";
        case TL_EHIP: return "HIP runtime error";
        case TL_EABORT: return "aborted by chunk callback";
        default: return "unknown error code";
    }
}

const char *tl_last_error(void) { return g_last_error.c_str(); }

int tl_order(const tl_csr *g, tl_order_kind kind, uint32_t *rank_dev, void *stream) {
    return guarded([&] {
        TL_REQUIRE(g, TL_EINVAL, "NULL handle");
        order_impl(g, (int)kind, rank_dev, (hipStream_t)stream);
        return TL_OK;
    });
}

int tl_order_neigh(const tl_csr *g, double eps, uint32_t max_passes, uint32_t max_visits, uint32_t *rank_dev,
                   tl_neigh_result *out, void *stream) {
    return guarded([&] {
        TL_REQUIRE(g, TL_EINVAL, "NULL handle");
        TL_REQUIRE(rank_dev || g->n == 0, TL_EINVAL, "rank is NULL");
        neigh_impl(g, eps, max_passes, max_visits, rank_dev, out, (hipStream_t)stream);
        return TL_OK;
    });
}

int tl_batch_orient(uint32_t k, const uint32_t *n, const uint64_t *m, const uint32_t *src, const uint32_t *dst,
                    const uint32_t *rank, void *stream, tl_batch **out) {
    return guarded([&] {
        TL_REQUIRE(out, TL_EINVAL, "out is NULL");
        *out = nullptr;
        *out = batch_orient_impl(k, n, m, src, dst, rank, (hipStream_t)stream);
        return TL_OK;
    });
}

int tl_batch_from_graphs(uint32_t k, const tl_csr *const *gs, void *stream, tl_batch **out) {
    return guarded([&] {
        TL_REQUIRE(out, TL_EINVAL, "out is NULL");
        *out = nullptr;
        *out = batch_from_csrs_impl(k, gs, (hipStream_t)stream);
        return TL_OK;
    });
}

int tl_batch_list(tl_batch *b, tl_algo a, int use_graph, uint64_t *per_graph, uint64_t *per_graph_dev,
                  void *stream) {
    return guarded([&] {
        TL_REQUIRE(b, TL_EINVAL, "NULL handle");
        TL_REQUIRE(a == TL_APP || a == TL_APM || a == TL_AMM, TL_EINVAL, "unknown algorithm");
        batch_list_impl(b, (int)a, (hipStream_t)stream, use_graph ? 1 : 0, per_graph, per_graph_dev);
        return TL_OK;
    });
}

int tl_batch_size(const tl_batch *b, uint32_t *k, uint32_t *n, uint64_t *m) {
    return guarded([&] {
        TL_REQUIRE(b, TL_EINVAL, "NULL handle");
        batch_sizes(b, k, n, m);
        return TL_OK;
    });
}

void tl_batch_free(tl_batch *b) {
    if (!b) return;
    (void)guarded([&] {
        batch_free_impl(b, true);
        return TL_OK;
    });
}

int tl_server_create(const tl_server_config *cfg, tl_server **out) {
    return guarded([&] {
        TL_REQUIRE(out, TL_EINVAL, "out is NULL");
        *out = nullptr;
        *out = server_create_impl(cfg);
        return TL_OK;
    });
}

int tl_server_submit(tl_server *s, const tl_job *job, uint64_t *id) {
    return guarded([&] {
        TL_REQUIRE(s && id, TL_EINVAL, "NULL argument");
        *id = server_submit_impl(s, job);
        return TL_OK;
    });
}

int tl_server_poll(tl_server *s, uint64_t id, int64_t wait_us, tl_job_result *out) {
    return guarded([&] {
        TL_REQUIRE(s && out, TL_EINVAL, "NULL argument");
        return server_poll_impl(s, id, wait_us, out);
    });
}

int tl_server_cancel(tl_server *s, uint64_t id) {
    return guarded([&] {
        TL_REQUIRE(s, TL_EINVAL, "NULL handle");
        return server_cancel_impl(s, id);
    });
}

int tl_server_pause(tl_server *s, int paused) {
    return guarded([&] {
        TL_REQUIRE(s, TL_EINVAL, "NULL handle");
        server_pause_impl(s, paused != 0);
        return TL_OK;
    });
}

int tl_server_get_stats(tl_server *s, tl_server_stats *out) {
    return guarded([&] {
        TL_REQUIRE(s && out, TL_EINVAL, "NULL argument");
        server_stats_impl(s, out);
        return TL_OK;
    });
}

uint64_t tl_server_job_bytes(uint32_t n, uint64_t m) { return job_bytes(n, m); }

void tl_server_destroy(tl_server *s) {
    if (!s) return;
    (void)guarded([&] {
        server_destroy_impl(s);
        return TL_OK;
    });
}

}  // extern "C"
