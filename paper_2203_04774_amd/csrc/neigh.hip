// Neigh (Algorithm 3, Section 3.3.1): a local search that moves each vertex
// to the place among its neighbours that gives the lowest C+-.  It is
// sequential (every move changes the costs of the next), so it runs on the
// host over a copy of the oriented graph.  The order is a doubly linked
// list with 64-bit order labels (a vertex moves in O(1), two vertices
// compare by label; labels are spread out again when a gap closes), and the
// candidates' costs come from the neighbours' current in- and out-degrees
// in Θ(d) per vertex, as the paper describes:
//
//   with N_u sorted by the order as v_1 .. v_d, candidate p puts u after
//   v_1 .. v_p and before the rest.  Let (a_i, b_i) be v_i's out- and
//   in-degree not counting u.  Moving from p - 1 to p puts v_p before u:
//   v_p's share goes from a_p (b_p + 1) to (a_p + 1) b_p and u's from
//   (p - 1)(d - p + 1) to p (d - p), so
//     C(p) - C(p - 1) = (b_p - a_p) + (d - 2p + 1).
//
// Readings: a pass visits vertices by increasing id; a vertex whose current
// place is among the cheapest stays put, otherwise it goes to the smallest
// cheapest p (right before v_1 for p = 0, right after v_p otherwise); passes
// repeat while one brings C+- below (1 - eps) times its value at the pass's
// start, at most max_passes times.
#include <algorithm>
#include <chrono>
#include <utility>
#include <vector>

#include "tl_internal.h"
#include "timing.h"

namespace {

struct OrderList {
    // nodes 0..n-1 are vertices (in g's rank space), n is the head, n+1 the tail
    std::vector<u32> prev, next;
    std::vector<u64> label;
    u32 n;
    u64 gap;

    explicit OrderList(u32 nv) : prev(nv + 2), next(nv + 2), label(nv + 2), n(nv) {
        int bits = 1;
        while (bits < 40 && (1ull << bits) < (u64)nv + 2) bits++;
        gap = 1ull << (62 - bits);
        for (u32 r = 0; r < nv; r++) {
            prev[r] = r == 0 ? head() : r - 1;
            next[r] = r + 1 == nv ? tail() : r + 1;
        }
        next[head()] = nv ? 0 : tail();
        prev[tail()] = nv ? nv - 1 : head();
        relabel();
    }
    u32 head() const { return n; }
    u32 tail() const { return n + 1; }
    void relabel() {
        u64 l = 0;
        for (u32 x = head();; x = next[x]) {
            label[x] = l;
            l += gap;
            if (x == tail()) break;
        }
    }
    void unlink(u32 x) {
        next[prev[x]] = next[x];
        prev[next[x]] = prev[x];
    }
    // x goes between a and next[a]
    void insert_after(u32 a, u32 x) {
        const u32 b = next[a];
        prev[x] = a;
        next[x] = b;
        next[a] = x;
        prev[b] = x;
        if (label[b] - label[a] < 2) relabel();
        else label[x] = label[a] + (label[b] - label[a]) / 2;
    }
};

}  // namespace

void neigh_impl(const tl_csr *g, double eps, u32 max_passes, u32 max_visits, u32 *rank_dev, tl_neigh_result *res,
                hipStream_t s) {
    TL_REQUIRE(eps >= 0.0 && eps < 1.0, TL_EINVAL, "eps must lie in [0, 1)");
    const u32 n = g->n;
    const u64 m = g->m;
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<u64> off_f((u64)n + 1), off_b((u64)n + 1);
    std::vector<u32> adj_f(m), adj_b(m), inv(n);
    if (n) {
        TL_HIP(hipMemcpyAsync(off_f.data(), g->off_f, ((u64)n + 1) * 8, hipMemcpyDeviceToHost, s));
        TL_HIP(hipMemcpyAsync(off_b.data(), g->off_b, ((u64)n + 1) * 8, hipMemcpyDeviceToHost, s));
        TL_HIP(hipMemcpyAsync(inv.data(), g->inv, (u64)n * 4, hipMemcpyDeviceToHost, s));
        if (m) {
            TL_HIP(hipMemcpyAsync(adj_f.data(), g->adj_f, m * 4, hipMemcpyDeviceToHost, s));
            TL_HIP(hipMemcpyAsync(adj_b.data(), g->adj_b, m * 4, hipMemcpyDeviceToHost, s));
        }
        TL_HIP(hipStreamSynchronize(s));
    }
    // starting order: g's own ranks, so out-degree = successors, in-degree = predecessors
    std::vector<u32> rank_of(n);
    std::vector<u64> dplus(n), dminus(n);
    u64 c = 0;
    for (u32 r = 0; r < n; r++) {
        rank_of[inv[r]] = r;
        dplus[r] = off_f[r + 1] - off_f[r];
        dminus[r] = off_b[r + 1] - off_b[r];
        c += dplus[r] * dminus[r];
    }
    const u64 c_start = c;
    OrderList L(n);
    std::vector<std::pair<u64, u32>> nb;
    std::vector<long long> f;
    u32 passes = 0, visits = 0;
    u64 moves = 0;
    bool stop = false;
    while (!stop && passes < max_passes) {
        const u64 c0 = c;
        for (u32 u = 0; u < n; u++) {
            if (max_visits && visits == max_visits) {
                stop = true;
                break;
            }
            visits++;
            const u32 r = rank_of[u];
            const u64 d = (off_f[r + 1] - off_f[r]) + (off_b[r + 1] - off_b[r]);
            if (d == 0) continue;
            nb.clear();
            for (u64 j = off_f[r]; j < off_f[r + 1]; j++) nb.emplace_back(L.label[adj_f[j]], adj_f[j]);
            for (u64 j = off_b[r]; j < off_b[r + 1]; j++) nb.emplace_back(L.label[adj_b[j]], adj_b[j]);
            std::sort(nb.begin(), nb.end());
            const u64 lr = L.label[r];
            u64 pcur = 0;
            while (pcur < d && nb[pcur].first < lr) pcur++;
            // relative costs f[p] = C(p) - C(0)
            f.assign(d + 1, 0);
            long long best = 0;
            for (u64 p = 1; p <= d; p++) {
                const u32 v = nb[p - 1].second;
                const bool before = p <= pcur;  // v precedes u now
                const long long a = (long long)dplus[v] - (before ? 1 : 0);
                const long long b = (long long)dminus[v] - (before ? 0 : 1);
                f[p] = f[p - 1] + (b - a) + ((long long)d - 2 * (long long)p + 1);
                best = std::min(best, f[p]);
            }
            if (f[pcur] == best) continue;
            u64 ps = 0;
            while (f[ps] != best) ps++;
            L.unlink(r);
            if (ps == 0) L.insert_after(L.prev[nb[0].second], r);
            else L.insert_after(nb[ps - 1].second, r);
            // neighbours that changed sides
            if (ps > pcur) {
                for (u64 i = pcur; i < ps; i++) {
                    const u32 v = nb[i].second;
                    dminus[v]--;
                    dplus[v]++;
                }
            } else {
                for (u64 i = ps; i < pcur; i++) {
                    const u32 v = nb[i].second;
                    dplus[v]--;
                    dminus[v]++;
                }
            }
            dminus[r] = ps;
            dplus[r] = d - ps;
            c = (u64)((long long)c + (best - f[pcur]));
            moves++;
        }
        if (stop) break;
        passes++;
        if (!((double)c < (1.0 - eps) * (double)c0)) break;
    }
    std::vector<u32> rank(n);
    {
        u32 i = 0;
        for (u32 x = L.next[L.head()]; x != L.tail(); x = L.next[x]) rank[inv[x]] = i++;
    }
    if (n) {
        TL_HIP(hipMemcpyAsync(rank_dev, rank.data(), (u64)n * 4, hipMemcpyHostToDevice, s));
        TL_HIP(hipStreamSynchronize(s));
    }
    if (res) {
        res->cpm_start = c_start;
        res->cpm = c;
        res->passes = passes;
        res->visits = visits;
        res->moves = moves;
        res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
}
