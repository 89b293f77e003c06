// Listing server: jobs arrive one by one, are admitted against a device
// memory budget, batched with whatever else is waiting, and listed while
// the next batch is uploaded and oriented on a second stream.
//
// Three threads own the device work, each on its own stream.  The upload
// thread admits waiting jobs in arrival order while their modelled
// footprint fits the budget and copies their edges and orderings to the
// device; a job whose graph is large forms a batch of its own.  The orient
// thread orients each uploaded batch as one disjoint union (batch.hip).
// The list threads (eight by default, each on its own stream) take oriented
// batches in order: a union of small graphs is listed by the batched pass
// (per-graph rows), a batch of one by the plain listing (light and heavy
// pivots).  So the copy of one batch, the orientation of the next and the
// listing of others overlap, and one batch's host waits are covered by
// another's kernels.  A batch
// whose union fails validation is split and its jobs are oriented one by
// one, so a malformed job fails alone.
//
// Keyed jobs keep their oriented graph resident: the first job of a key is
// uploaded and oriented alone (inside a keyed batch), its graph is kept in
// a cache under the key, and later jobs of the key skip the upload and the
// orientation: a keyed batch is listed from a union built by copying the
// resident graphs (batch_from_csrs_impl).  Resident bytes count against the
// budget; entries not in use are dropped, least recently used first, when a
// job needs the room.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "tl_internal.h"

namespace {

u64 now_ns() {
    return (u64)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// Host-to-device upload through two page-locked staging buffers: copier
// threads fill one buffer from the caller's (pageable) arrays while the
// copy engine drains the other, so the upload runs near the link's rate
// instead of the single-threaded pageable path's.
class Uploader {
  public:
    static constexpr u64 CHUNK = 16ull << 20;  // bytes per staging buffer
    static constexpr int COPIERS = 4;

    explicit Uploader(hipStream_t s) : s_(s) {
        bool ok = true;
        for (int b = 0; b < 2; b++) {
            if (hipHostMalloc(reinterpret_cast<void **>(&pin_[b]), CHUNK, hipHostMallocDefault) != hipSuccess) {
                pin_[b] = nullptr;
                ok = false;
            }
            if (hipEventCreateWithFlags(&ev_[b], hipEventDisableTiming) != hipSuccess) {
                ev_[b] = nullptr;
                ok = false;
            }
        }
        if (!ok) {
            release();
            throw TlError{TL_ENOMEM, "cannot allocate the page-locked upload staging buffers"};
        }
        for (int t = 0; t < COPIERS; t++) th_.emplace_back([this] { copier(); });
    }
    ~Uploader() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto &t : th_) t.join();
        (void)hipStreamSynchronize(s_);
        release();
    }
    // bytes from host memory h to device memory d, enqueued on the stream
    void copy(void *d, const void *h, u64 bytes) {
        if (bytes < (1ull << 20)) {  // small: the ordinary path
            TL_HIP(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, s_));
            return;
        }
        for (u64 off = 0; off < bytes; off += CHUNK) {
            const int b = (int)(n_++ & 1);
            if (used_[b]) TL_HIP(hipEventSynchronize(ev_[b]));  // its previous copy has left the buffer
            const u64 len = bytes - off < CHUNK ? bytes - off : CHUNK;
            fill(pin_[b], static_cast<const char *>(h) + off, len);
            TL_HIP(hipMemcpyAsync(static_cast<char *>(d) + off, pin_[b], len, hipMemcpyHostToDevice, s_));
            TL_HIP(hipEventRecord(ev_[b], s_));
            used_[b] = true;
        }
    }

  private:
    void release() {
        for (int b = 0; b < 2; b++) {
            if (ev_[b]) (void)hipEventDestroy(ev_[b]);
            if (pin_[b]) (void)hipHostFree(pin_[b]);
            ev_[b] = nullptr;
            pin_[b] = nullptr;
        }
    }
    // the copier threads copy one part each of [src, src + len)
    void fill(char *dst, const char *src, u64 len) {
        std::unique_lock<std::mutex> lk(mu_);
        dst_ = dst;
        src_ = src;
        len_ = len;
        taken_ = 0;
        finished_ = 0;
        gen_++;
        cv_.notify_all();
        cv_done_.wait(lk, [&] { return finished_ == COPIERS; });
    }
    void copier() {
        u64 seen = 0;
        for (;;) {
            char *dst;
            const char *src;
            u64 lo, hi;
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
                if (stop_) return;
                seen = gen_;
                const u64 part = (len_ + COPIERS - 1) / COPIERS;
                const u64 k = taken_++;
                lo = k * part < len_ ? k * part : len_;
                hi = lo + part < len_ ? lo + part : len_;
                dst = dst_;
                src = src_;
            }
            if (hi > lo) std::memcpy(dst + lo, src + lo, hi - lo);
            {
                std::lock_guard<std::mutex> lk(mu_);
                if (++finished_ == COPIERS) cv_done_.notify_one();
            }
        }
    }

    hipStream_t s_;
    char *pin_[2] = {nullptr, nullptr};
    hipEvent_t ev_[2] = {nullptr, nullptr};
    bool used_[2] = {false, false};
    u64 n_ = 0;
    std::vector<std::thread> th_;
    std::mutex mu_;
    std::condition_variable cv_, cv_done_;
    char *dst_ = nullptr;
    const char *src_ = nullptr;
    u64 len_ = 0, taken_ = 0, gen_ = 0;
    int finished_ = 0;
    bool stop_ = false;
};

struct Job {
    u64 id = 0;
    tl_job in{};
    u64 bytes = 0;  // modelled device footprint
    tl_job_result res{};
    bool solo = false;
    // keyed jobs: the resident graph listed (pinned while the job is in flight)
    bool resident = false;   // its graph was resident when it was admitted
    u64 keep_bytes = 0;      // a graph to be made resident: its bytes, reserved with the job's
    tl_csr *csr = nullptr;
    bool owns_csr = false;   // a duplicate of a graph made resident meanwhile: freed after listing
};

struct Ready {
    tl_batch *b = nullptr;   // the union (null for a keyed job listed alone from its graph)
    std::vector<Job *> jobs;
    u64 bytes = 0;
    u64 batch_id = 0;
    bool keyed = false;
};

// A resident oriented graph (keyed jobs).
struct Resident {
    tl_csr *g = nullptr;
    u64 bytes = 0;
    u32 refs = 0;    // jobs in flight that list it
    u64 last = 0;    // use tick, for least-recently-used dropping
};

// Device bytes of a resident oriented graph: offsets, adjacency, rows,
// forward indices and the inverse permutation.
u64 resident_bytes(u64 n, u64 m) { return 20 * m + 20 * n + 4096; }

// A batch whose edges and orderings are on the device, waiting to be oriented.
struct Uploaded {
    std::vector<Job *> jobs;
    u64 bytes = 0;
    DevBuf src, dst, rank;
    bool keyed = false;
    std::vector<u64> eo, vo;  // each job's offset in src/dst and in rank (uploaded jobs only)
};

}  // namespace

struct tl_server {
    tl_server_config cfg{};
    int device = 0;
    hipStream_t s_copy = nullptr, s_up = nullptr;
    std::vector<hipStream_t> s_list;  // one per list thread

    std::mutex mu;
    std::condition_variable cv_pending;  // upload waits: new jobs, freed budget, stop
    std::condition_variable cv_ready;    // list waits: oriented batches, stop
    std::condition_variable cv_space;    // orient waits: room in the ready queue
    std::condition_variable cv_uploaded; // orient waits: uploaded batches, stop
    std::condition_variable cv_upspace;  // upload waits: room in the uploaded queue
    std::condition_variable cv_done;     // pollers wait
    std::deque<Job *> pending;
    std::deque<Job *> solo_retry;        // jobs of a union that failed validation
    std::deque<Ready> ready;
    std::deque<std::unique_ptr<Uploaded>> uploaded;
    u32 in_flight = 0;                   // batches between admission and the end of their listing
    std::unordered_map<u64, std::unique_ptr<Job>> jobs;
    std::unordered_map<u64, Resident> cache;  // resident graphs by key
    u64 cache_bytes = 0, tick = 0;
    u64 next_id = 1, next_batch = 1;
    u64 reserved = 0;  // admitted jobs' footprints plus the resident graphs
    bool stop = false, paused = false;
    tl_server_stats st{};

    std::unique_ptr<Uploader> up;  // staging pipeline of the upload thread
    std::thread uploader, orienter;
    std::vector<std::thread> listers;
};

namespace {

void finish(tl_server *S, Job *j, int status) {
    j->res.status = status;
    j->res.t_done_ns = now_ns();
}

// Called with S->mu held.
void release_bytes(tl_server *S, u64 bytes) {
    S->reserved -= bytes;
    S->cv_pending.notify_all();
}

// Copies the jobs' arrays to the device on the copy stream; throws on failure.
// Resident jobs of a keyed batch need no copy.
std::unique_ptr<Uploaded> upload_jobs(tl_server *S, const std::vector<Job *> &js, bool keyed) {
    u64 N = 0, M = 0;
    for (Job *j : js) {
        if (j->resident) continue;
        N += j->in.n;
        M += j->in.m;
    }
    const u64 t0 = now_ns();
    auto U = std::make_unique<Uploaded>();
    U->jobs = js;
    U->keyed = keyed;
    U->src = DevBuf((M ? M : 1) * 4, S->s_copy);
    U->dst = DevBuf((M ? M : 1) * 4, S->s_copy);
    U->rank = DevBuf((N ? N : 1) * 4, S->s_copy);
    u64 eo = 0, vo = 0;
    for (Job *j : js) {
        U->eo.push_back(eo);
        U->vo.push_back(vo);
        if (j->resident) continue;
        const tl_job &J = j->in;
        if (J.m) {
            S->up->copy(U->src.as<u32>() + eo, J.src, J.m * 4);
            S->up->copy(U->dst.as<u32>() + eo, J.dst, J.m * 4);
        }
        if (J.n) S->up->copy(U->rank.as<u32>() + vo, J.rank, (u64)J.n * 4);
        eo += J.m;
        vo += J.n;
    }
    TL_HIP(hipStreamSynchronize(S->s_copy));
    std::lock_guard<std::mutex> lk(S->mu);
    S->st.upload_ns += now_ns() - t0;
    return U;
}

// Orients an uploaded batch as one union on the orient stream; throws on failure.
tl_batch *orient_uploaded(tl_server *S, Uploaded &U) {
    const u32 k = (u32)U.jobs.size();
    std::vector<u32> n(k);
    std::vector<u64> m(k);
    for (u32 i = 0; i < k; i++) {
        n[i] = U.jobs[i]->in.n;
        m[i] = U.jobs[i]->in.m;
    }
    const u64 t0 = now_ns();
    tl_batch *b = batch_orient_impl(k, n.data(), m.data(), U.src.as<u32>(), U.dst.as<u32>(), U.rank.as<u32>(),
                                    S->s_up);
    std::lock_guard<std::mutex> lk(S->mu);
    S->st.orient_ns += now_ns() - t0;
    return b;
}

// Drops the least recently used resident graph not in use (called with
// S->mu held); false if there is none.
bool drop_resident(tl_server *S) {
    auto victim = S->cache.end();
    for (auto it = S->cache.begin(); it != S->cache.end(); ++it)
        if (it->second.refs == 0 && (victim == S->cache.end() || it->second.last < victim->second.last)) victim = it;
    if (victim == S->cache.end()) return false;
    tl_csr_free(victim->second.g);
    S->cache_bytes -= victim->second.bytes;
    S->reserved -= victim->second.bytes;
    S->cache.erase(victim);
    S->st.resident_dropped++;
    return true;
}

// Picks the next batch (called with S->mu held).  Returns false to wait.
// A batch holds either keyed jobs only or unkeyed jobs only; keyed is set.
bool pick(tl_server *S, std::vector<Job *> &out, u64 &bytes, bool &keyed) {
    out.clear();
    bytes = 0;
    keyed = false;
    if (!S->solo_retry.empty()) {
        Job *j = S->solo_retry.front();
        S->solo_retry.pop_front();
        j->solo = true;
        out.push_back(j);
        return true;  // its bytes are still reserved
    }
    u64 edges = 0;
    while (!S->paused && !S->pending.empty()) {
        Job *j = S->pending.front();
        const bool jk = j->in.key != 0;
        if (!out.empty() && jk != keyed) break;  // keyed and unkeyed jobs are not batched together
        auto hit = jk ? S->cache.find(j->in.key) : S->cache.end();
        const bool res = hit != S->cache.end();
        // a graph to be made resident is reserved with the job; a resident
        // one is listed from a union built by copying it, no upload or sort
        const u64 keep = jk && !res ? resident_bytes(j->in.n, j->in.m) : 0;
        const u64 need = j->bytes + keep;
        const bool big = j->in.m >= S->cfg.solo_edges;
        if (!out.empty() && (big || out.size() >= S->cfg.max_batch_jobs || edges + j->in.m > S->cfg.max_batch_edges))
            break;
        if (need > S->cfg.hbm_budget) {  // can never fit: refuse it
            S->pending.pop_front();
            finish(S, j, TL_ENOMEM);
            S->st.rejected++;
            S->cv_done.notify_all();
            continue;
        }
        if (res) hit->second.refs++;  // pinned: room is not made by dropping its own graph
        while (S->reserved + bytes + need > S->cfg.hbm_budget && drop_resident(S)) {
        }
        if (S->reserved + bytes + need > S->cfg.hbm_budget) {  // wait for memory, keep the order
            if (res) hit->second.refs--;
            break;
        }
        S->pending.pop_front();
        keyed = jk;
        j->resident = res;
        if (res) {
            hit->second.last = ++S->tick;
            j->csr = hit->second.g;
            S->st.resident_hits++;
        } else {
            j->keep_bytes = keep;
        }
        out.push_back(j);
        bytes += j->bytes + j->keep_bytes;
        edges += j->in.m;
        if (big) {
            j->solo = true;
            break;
        }
    }
    if (out.empty()) return false;
    S->reserved += bytes;
    S->st.peak_reserved = std::max(S->st.peak_reserved, S->reserved);
    return true;
}

// A keyed batch's graphs: resident ones as they are, the others oriented one
// by one (each made resident unless its key became resident meanwhile); a
// job whose graph fails validation finishes alone.  Then the union is built
// by copying, or, for one job alone, its graph is listed directly.  Throws on
// device failures.
bool orient_keyed(tl_server *S, Uploaded &U, Ready &r) {
    const u64 t0 = now_ns();
    std::vector<Job *> ok;
    std::vector<const tl_csr *> gs;
    for (size_t i = 0; i < U.jobs.size(); i++) {
        Job *j = U.jobs[i];
        if (!j->resident) {
            tl_csr *g = nullptr;
            try {
                g = orient_impl(j->in.n, U.src.as<u32>() + U.eo[i], U.dst.as<u32>() + U.eo[i], j->in.m,
                                U.rank.as<u32>() + U.vo[i], S->s_up);
                TL_HIP(hipStreamSynchronize(S->s_up));
            } catch (const TlError &e) {
                if (e.code != TL_EINVAL) throw;
                std::lock_guard<std::mutex> lk(S->mu);
                finish(S, j, TL_EINVAL);
                release_bytes(S, j->bytes + j->keep_bytes);
                U.bytes -= j->bytes + j->keep_bytes;
                S->cv_done.notify_all();
                continue;
            }
            std::lock_guard<std::mutex> lk(S->mu);
            j->csr = g;
            auto it = S->cache.find(j->in.key);
            if (it == S->cache.end()) {
                // made resident: its bytes move from the job to the cache
                Resident rs;
                rs.g = g;
                rs.bytes = j->keep_bytes;
                rs.refs = 1;
                rs.last = ++S->tick;
                S->cache.emplace(j->in.key, rs);
                S->cache_bytes += j->keep_bytes;
                U.bytes -= j->keep_bytes;
                j->resident = true;
            } else {
                j->owns_csr = true;  // listed from its own copy, freed afterwards
            }
            j->keep_bytes = 0;
        }
        ok.push_back(j);
        gs.push_back(j->csr);
    }
    r.jobs = ok;
    r.bytes = U.bytes;
    r.keyed = true;
    if (!ok.empty() && !(ok.size() == 1 && ok[0]->solo)) r.b = batch_from_csrs_impl((u32)gs.size(), gs.data(), S->s_up);
    std::lock_guard<std::mutex> lk(S->mu);
    S->st.orient_ns += now_ns() - t0;
    return !ok.empty();
}

// After a keyed batch is listed (called with S->mu held): unpins the
// resident graphs, frees duplicates.
void release_keyed(tl_server *S, const std::vector<Job *> &js) {
    for (Job *j : js) {
        if (j->owns_csr) {
            tl_csr_free(j->csr);
        } else if (j->csr) {
            auto it = S->cache.find(j->in.key);
            if (it != S->cache.end() && it->second.g == j->csr && it->second.refs) it->second.refs--;
        }
        j->csr = nullptr;
        j->owns_csr = false;
    }
}

// Called with S->mu held: a failed batch either splits (a malformed job
// among several: each is retried alone) or fails its jobs.
void fail_batch(tl_server *S, const std::vector<Job *> &js, u64 bytes, int err) {
    S->in_flight--;
    if (err == TL_EINVAL && js.size() > 1 && js[0]->in.key == 0) {  // (keyed jobs fail alone already)
        for (Job *j : js) S->solo_retry.push_back(j);
        S->st.split_batches++;
        S->cv_pending.notify_all();
        return;  // the bytes stay reserved for the retries
    }
    release_keyed(S, js);
    for (Job *j : js) finish(S, j, err);
    release_bytes(S, bytes);
    S->cv_done.notify_all();
}

void upload_loop(tl_server *S) {
    (void)hipSetDevice(S->device);
    std::vector<Job *> js;
    for (;;) {
        u64 bytes = 0;
        bool keyed = false;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            // without pipelining a batch is admitted only when the previous one is listed
            S->cv_pending.wait(lk, [&] {
                return S->stop || ((S->cfg.pipeline || S->in_flight == 0) && pick(S, js, bytes, keyed));
            });
            if (S->stop) return;
            S->in_flight++;
            const u64 t = now_ns();
            for (Job *j : js)
                if (!j->res.t_admit_ns) j->res.t_admit_ns = t;
        }
        if (js.size() == 1 && js[0]->solo && bytes == 0) bytes = js[0]->bytes;  // a retry: reserved already
        std::unique_ptr<Uploaded> U;
        int err = TL_OK;
        try {
            U = upload_jobs(S, js, keyed);
        } catch (const TlError &e) {
            err = e.code;
        } catch (...) {
            err = TL_EHIP;
        }
        std::unique_lock<std::mutex> lk(S->mu);
        if (err != TL_OK) {
            fail_batch(S, js, bytes, err);
            continue;
        }
        U->bytes = bytes;
        S->cv_upspace.wait(lk, [&] { return S->stop || S->uploaded.size() < 1; });
        if (S->stop) return;
        S->uploaded.push_back(std::move(U));
        S->cv_uploaded.notify_all();
    }
}

void orient_loop(tl_server *S) {
    (void)hipSetDevice(S->device);
    for (;;) {
        std::unique_ptr<Uploaded> U;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_uploaded.wait(lk, [&] { return S->stop || !S->uploaded.empty(); });
            if (S->stop) return;
            U = std::move(S->uploaded.front());
            S->uploaded.pop_front();
            S->cv_upspace.notify_all();
        }
        Ready r;
        int err = TL_OK;
        bool any = true;
        try {
            if (U->keyed) {
                any = orient_keyed(S, *U, r);
            } else {
                r.b = orient_uploaded(S, *U);
                r.jobs = U->jobs;
                r.bytes = U->bytes;
            }
        } catch (const TlError &e) {
            err = e.code;
        } catch (...) {
            err = TL_EHIP;
        }
        const std::vector<Job *> js = U->jobs;
        const u64 bytes = U->bytes;
        U.reset();  // the copies are no longer needed (the orient stream has finished with them)
        std::unique_lock<std::mutex> lk(S->mu);
        if (err != TL_OK) {
            if (r.b) {
                lk.unlock();
                batch_free_impl(r.b, true);
                lk.lock();
            }
            // jobs of a keyed batch that already failed alone are final
            std::vector<Job *> left;
            for (Job *j : js)
                if (j->res.status == TL_JOB_PENDING) left.push_back(j);
            fail_batch(S, left, bytes, err);
            continue;
        }
        if (!any) {  // every job of a keyed batch failed alone
            S->in_flight--;
            release_bytes(S, r.bytes);
            S->cv_pending.notify_all();
            continue;
        }
        S->cv_space.wait(lk, [&] { return S->stop || S->ready.size() < 2u; });
        if (S->stop) {
            lk.unlock();
            if (r.b) batch_free_impl(r.b, true);
            return;
        }
        r.batch_id = S->next_batch++;
        S->ready.push_back(std::move(r));
        S->cv_ready.notify_all();
    }
}

void list_loop(tl_server *S, u32 li) {
    (void)hipSetDevice(S->device);
    const hipStream_t stream = S->s_list[li];
    std::vector<u64> table;
    for (;;) {
        Ready r;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_ready.wait(lk, [&] { return S->stop || !S->ready.empty(); });
            if (S->stop) return;
            r = std::move(S->ready.front());
            S->ready.pop_front();  // taken: another list thread may start on the next
            S->cv_space.notify_all();
        }
        const u32 k = (u32)r.jobs.size();
        const u64 t_start = now_ns();
        int err = TL_OK;
        std::vector<tl_summary> solo_out;
        try {
            if (k == 1 && r.jobs[0]->solo) {
                // a graph alone: the plain listing with light and heavy pivots
                tl_summary sm{};
                list_impl(r.b ? batch_csr(r.b) : r.jobs[0]->csr, (int)r.jobs[0]->in.algo, 0u, 0xffffffffu, nullptr,
                          0, nullptr, nullptr, stream, &sm);
                solo_out.push_back(sm);
            } else {
                table.assign(3ull * k, 0);
                std::vector<u64> t2(3ull * k);
                bool have[3] = {false, false, false};
                for (Job *j : r.jobs) have[(int)j->in.algo] = true;
                for (int a = 0; a < 3; a++) {
                    if (!have[a]) continue;
                    batch_list_impl(r.b, a, stream, 0, t2.data(), nullptr);
                    for (u32 i = 0; i < k; i++)
                        if ((int)r.jobs[i]->in.algo == a)
                            for (int c = 0; c < 3; c++) table[3ull * i + c] = t2[3ull * i + c];
                }
            }
        } catch (const TlError &e) {
            err = e.code;
        } catch (...) {
            err = TL_EHIP;
        }
        if (r.b) batch_free_impl(r.b, false);  // the list stream has finished with it
        pool_trim_above(S->cfg.hbm_budget + S->cfg.hbm_budget / 2);
        std::unique_lock<std::mutex> lk(S->mu);
        if (r.keyed) release_keyed(S, r.jobs);
        S->in_flight--;
        S->cv_space.notify_all();
        S->cv_pending.notify_all();
        for (u32 i = 0; i < k; i++) {
            Job *j = r.jobs[i];
            j->res.t_start_ns = t_start;
            j->res.batch_id = r.batch_id;
            j->res.batch_jobs = k;
            if (err == TL_OK) {
                if (!solo_out.empty()) {
                    j->res.count = solo_out[0].count;
                    j->res.hash = solo_out[0].hash;
                    j->res.work = solo_out[0].work;
                } else {
                    j->res.count = table[3ull * i];
                    j->res.hash = table[3ull * i + 1];
                    j->res.work = table[3ull * i + 2];
                }
            }
            finish(S, j, err);
        }
        S->st.batches++;
        S->st.jobs_done += k;
        S->st.max_batch_jobs_seen = std::max<u64>(S->st.max_batch_jobs_seen, k);
        S->st.list_ns += now_ns() - t_start;
        release_bytes(S, r.bytes);
        S->cv_done.notify_all();
    }
}

}  // namespace

// Modelled device bytes of one job from admission to completion: the
// uploaded edges and ranks, the union's copies, the orientation's
// temporaries, the oriented CSR with its inverse, and the listing scratch.
u64 job_bytes(u64 n, u64 m) { return 72 * m + 64 * n + (2ull << 20); }

tl_server *server_create_impl(const tl_server_config *cfg) {
    TL_REQUIRE(cfg, TL_EINVAL, "NULL config");
    TL_REQUIRE(cfg->hbm_budget > 0, TL_EINVAL, "hbm_budget must be > 0");
    auto S = std::make_unique<tl_server>();
    S->cfg = *cfg;
    if (!S->cfg.max_batch_jobs) S->cfg.max_batch_jobs = 4096;
    if (!S->cfg.max_batch_edges) S->cfg.max_batch_edges = 1ull << 27;
    if (!S->cfg.solo_edges) S->cfg.solo_edges = 1ull << 21;
    if (!S->cfg.list_threads) S->cfg.list_threads = 8;
    TL_REQUIRE(S->cfg.list_threads <= 8, TL_EINVAL, "list_threads must be at most 8");
    TL_HIP(hipGetDevice(&S->device));
    TL_HIP(hipStreamCreateWithFlags(&S->s_copy, hipStreamNonBlocking));
    TL_HIP(hipStreamCreateWithFlags(&S->s_up, hipStreamNonBlocking));
    S->s_list.assign(S->cfg.list_threads, nullptr);
    for (auto &st : S->s_list) TL_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    S->up = std::make_unique<Uploader>(S->s_copy);
    tl_server *p = S.release();
    p->uploader = std::thread(upload_loop, p);
    p->orienter = std::thread(orient_loop, p);
    for (u32 li = 0; li < p->cfg.list_threads; li++) p->listers.emplace_back(list_loop, p, li);
    return p;
}

u64 server_submit_impl(tl_server *S, const tl_job *job) {
    TL_REQUIRE(job, TL_EINVAL, "NULL job");
    TL_REQUIRE(job->algo == TL_APP || job->algo == TL_APM || job->algo == TL_AMM, TL_EINVAL, "unknown algorithm");
    TL_REQUIRE(job->m == 0 || (job->src && job->dst), TL_EINVAL, "src/dst is NULL");
    TL_REQUIRE(job->n == 0 || job->rank, TL_EINVAL, "rank is NULL");
    TL_REQUIRE(job->m < (1ull << 32) && job->n < 0xffffffffu, TL_EINVAL, "job too large");
    auto j = std::make_unique<Job>();
    j->in = *job;
    j->bytes = job_bytes(job->n, job->m);
    j->res.status = TL_JOB_PENDING;
    j->res.t_submit_ns = now_ns();
    std::lock_guard<std::mutex> lk(S->mu);
    TL_REQUIRE(!S->stop, TL_EINVAL, "server is stopping");
    j->id = S->next_id++;
    const u64 id = j->id;
    S->pending.push_back(j.get());
    S->jobs.emplace(id, std::move(j));
    S->st.submitted++;
    S->cv_pending.notify_all();
    return id;
}

int server_poll_impl(tl_server *S, u64 id, int64_t wait_us, tl_job_result *out) {
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->jobs.find(id);
    TL_REQUIRE(it != S->jobs.end(), TL_EINVAL, "unknown job id (or its result was already taken)");
    Job *j = it->second.get();
    auto done = [&] { return j->res.status != TL_JOB_PENDING; };
    if (!done() && wait_us != 0) {
        if (wait_us < 0) S->cv_done.wait(lk, done);
        else S->cv_done.wait_for(lk, std::chrono::microseconds(wait_us), done);
    }
    *out = j->res;
    if (done()) S->jobs.erase(it);  // a final result is handed out once
    return TL_OK;
}

int server_cancel_impl(tl_server *S, u64 id) {
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->jobs.find(id);
    TL_REQUIRE(it != S->jobs.end(), TL_EINVAL, "unknown job id");
    Job *j = it->second.get();
    auto q = std::find(S->pending.begin(), S->pending.end(), j);
    if (q == S->pending.end()) return TL_EINVAL;  // admitted already: it runs to completion
    S->pending.erase(q);
    finish(S, j, TL_EABORT);
    S->st.cancelled++;
    S->cv_done.notify_all();
    S->cv_pending.notify_all();
    return TL_OK;
}

void server_pause_impl(tl_server *S, bool paused) {
    std::lock_guard<std::mutex> lk(S->mu);
    S->paused = paused;
    S->cv_pending.notify_all();
}

void server_stats_impl(tl_server *S, tl_server_stats *out) {
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->st;
    out->reserved = S->reserved;
    out->pending = S->pending.size();
    out->resident_graphs = S->cache.size();
    out->resident_bytes = S->cache_bytes;
}

void server_destroy_impl(tl_server *S) {
    {
        std::unique_lock<std::mutex> lk(S->mu);
        // let admitted work finish; jobs still waiting are cancelled
        for (Job *j : S->pending) finish(S, j, TL_EABORT);
        S->cv_done.notify_all();
        S->pending.clear();
        S->cv_done.wait(lk, [&] {
            return S->in_flight == 0 && S->ready.empty() && S->uploaded.empty() && S->reserved == S->cache_bytes &&
                   S->solo_retry.empty();
        });
        for (auto &kv : S->cache) tl_csr_free(kv.second.g);
        S->cache.clear();
        S->reserved -= S->cache_bytes;
        S->cache_bytes = 0;
        S->stop = true;
        S->cv_pending.notify_all();
        S->cv_uploaded.notify_all();
        S->cv_upspace.notify_all();
        S->cv_ready.notify_all();
        S->cv_space.notify_all();
    }
    S->uploader.join();
    S->orienter.join();
    for (std::thread &t : S->listers) t.join();
    S->up.reset();
    std::vector<hipStream_t> streams = S->s_list;
    streams.push_back(S->s_copy);
    streams.push_back(S->s_up);
    for (hipStream_t st : streams) {
        if (!st) continue;
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    delete S;
}
