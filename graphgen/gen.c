/*
 * Seeded synthetic graph and ordering generators.
 *
 * These produce the inputs that both the oracle and the GPU library consume:
 * undirected edge lists (RMAT, Chung-Lu) and vertex orderings (degree, core,
 * uniform random).  Nothing here lists triangles or evaluates a cost; the
 * graph-model definitions follow the standard published generators:
 *
 *   RMAT      Chakrabarti, Zhan, Faloutsos, "R-MAT: A Recursive Model for
 *             Graph Mining", SDM 2004: each edge descends `scale` levels of
 *             the adjacency matrix, choosing quadrant a/b/c/d at each level.
 *   Chung-Lu  Chung & Lu, "Connected components in random graphs with given
 *             expected degree sequences", 2002: endpoints drawn independently
 *             with probability proportional to a weight w_i; here
 *             w_i = (i + i0)^(-1/(gamma-1)) (a power law of exponent gamma).
 *   core      Batagelj & Zaversnik, "An O(m) algorithm for cores
 *             decomposition of networks", 2003: repeatedly remove a vertex of
 *             minimum current degree.  Ties are broken by smallest vertex id,
 *             which makes the peeling order (and hence the rank) unique.
 *
 * Random numbers come from a counter-based stream built on the splitmix64
 * output function (Steele, Lea, Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014; Vigna's public splitmix64.c):
 *   rnd(key, i) = mix64(key + (i + 1) * 0x9e3779b97f4a7c15)
 * so any element of any stream can be produced independently, in parallel.
 *
 * Every generated graph is returned simple: self-loops removed and each
 * undirected edge reported once as (min id, max id), sorted by that pair.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

typedef uint64_t u64;
typedef uint32_t u32;

static inline u64 mix64(u64 z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}
static inline u64 rnd(u64 key, u64 i) { return mix64(key + (i + 1) * 0x9e3779b97f4a7c15ULL); }
static inline u64 stream_key(u64 seed, u64 tag) { return mix64(mix64(seed) ^ (tag * 0xd1b54a32d192ed03ULL)); }
/* uniform double in [0,1) from the top 53 bits */
static inline double u01(u64 r) { return (double)(r >> 11) * (1.0 / 9007199254740992.0); }

int gg_num_threads(void) { return omp_get_max_threads(); }

/* ---------------------------------------------------------------- sorting */

/* LSD radix sort of 64-bit keys, 16-bit digits, parallel histogram/scatter.
 * Only the digits that can be non-zero (given max_key) are processed. */
static void radix_sort_u64(u64 *a, u64 *tmp, u64 n, u64 max_key) {
    int nbits = 0;
    while (nbits < 64 && (max_key >> nbits)) nbits++;
    int passes = (nbits + 15) / 16;
    int nt = omp_get_max_threads();
    u64 *hist = (u64 *)calloc((size_t)nt * 65536, sizeof(u64));
    u64 *src = a, *dst = tmp;
    for (int p = 0; p < passes; p++) {
        int sh = 16 * p;
        memset(hist, 0, (size_t)nt * 65536 * sizeof(u64));
#pragma omp parallel num_threads(nt)
        {
            int t = omp_get_thread_num();
            u64 lo = n * (u64)t / nt, hi = n * (u64)(t + 1) / nt;
            u64 *h = hist + (size_t)t * 65536;
            for (u64 i = lo; i < hi; i++) h[(src[i] >> sh) & 0xffff]++;
#pragma omp barrier
#pragma omp single
            {
                u64 run = 0;
                for (int d = 0; d < 65536; d++)
                    for (int tt = 0; tt < nt; tt++) {
                        u64 c = hist[(size_t)tt * 65536 + d];
                        hist[(size_t)tt * 65536 + d] = run;
                        run += c;
                    }
            }
            for (u64 i = lo; i < hi; i++) {
                u64 k = src[i];
                dst[h[(k >> sh) & 0xffff]++] = k;
            }
        }
        u64 *sw = src; src = dst; dst = sw;
    }
    if (src != a) memcpy(a, src, n * sizeof(u64));
    free(hist);
}

/* keys hold (min<<32 | max) with loops already removed (or UINT64_MAX
 * sentinels); sort, deduplicate, split into src/dst.  Returns edge count. */
static u64 finish_simple(u64 *keys, u64 nk, u32 n, u32 *src, u32 *dst) {
    u64 *tmp = (u64 *)malloc(nk * sizeof(u64) + 8);
    u64 maxk = ((u64)(n ? n - 1 : 0) << 32) | (u64)(n ? n - 1 : 0);
    /* sentinels are removed before sorting so max_key bounds every key */
    u64 w = 0;
    for (u64 i = 0; i < nk; i++) if (keys[i] != UINT64_MAX) keys[w++] = keys[i];
    radix_sort_u64(keys, tmp, w, maxk);
    free(tmp);
    u64 m = 0;
    for (u64 i = 0; i < w; i++) {
        if (i && keys[i] == keys[i - 1]) continue;
        src[m] = (u32)(keys[i] >> 32);
        dst[m] = (u32)(keys[i] & 0xffffffffu);
        m++;
    }
    return m;
}

static inline u64 pack_edge(u32 a, u32 b) {
    if (a == b) return UINT64_MAX;
    return a < b ? (((u64)a << 32) | b) : (((u64)b << 32) | a);
}

/* ------------------------------------------------------------------ RMAT */

/* Draws `samples` RMAT edges over 2^scale vertices with quadrant
 * probabilities a, b, c (d = 1-a-b-c), no label scrambling, then simplifies.
 * src/dst must hold `samples` entries; returns the simple edge count m. */
u64 gg_rmat(int scale, u64 samples, double a, double b, double c, u64 seed, u32 *src, u32 *dst) {
    u64 key = stream_key(seed, 0x524d4154ULL /* "RMAT" */);
    u64 *keys = (u64 *)malloc(samples * sizeof(u64) + 8);
    /* thresholds on 32-bit uniforms */
    double ta = a, tb = a + b, tc = a + b + c;
    u64 TA = (u64)(ta * 4294967296.0), TB = (u64)(tb * 4294967296.0), TC = (u64)(tc * 4294967296.0);
    int words = (scale + 1) / 2; /* two 32-bit draws per 64-bit word */
#pragma omp parallel for schedule(static)
    for (long long i = 0; i < (long long)samples; i++) {
        u32 u = 0, v = 0;
        u64 base = (u64)i * (u64)words;
        u64 r = 0;
        for (int lvl = 0; lvl < scale; lvl++) {
            if ((lvl & 1) == 0) r = rnd(key, base + (u64)(lvl >> 1));
            u64 x = (lvl & 1) ? (r >> 32) : (r & 0xffffffffULL);
            u32 bit = 1u << (scale - 1 - lvl);
            if (x < TA) {
            } else if (x < TB) {
                v |= bit;
            } else if (x < TC) {
                u |= bit;
            } else {
                u |= bit; v |= bit;
            }
        }
        keys[i] = pack_edge(u, v);
    }
    u32 n = (u32)(1ULL << scale);
    u64 m = finish_simple(keys, samples, n, src, dst);
    free(keys);
    return m;
}

/* -------------------------------------------------------------- Chung-Lu */

/* Draws `samples` endpoint pairs, each endpoint independently with
 * probability proportional to w_i = (i + i0)^(-1/(gamma-1)), i in [0,n),
 * then simplifies.  Returns m. */
/* Chung-Lu endpoint pairs: each endpoint is vertex i with probability
 * proportional to (i + i0)^(-1/(gamma-1)); keys[i] = packed pair (loops as
 * sentinels).  Threads split the samples when `parallel` is set; the keys do
 * not depend on it. */
static void chung_lu_keys(u32 n, double gamma, double i0, u64 samples, u64 seed, u64 *keys, int parallel) {
    u64 key = stream_key(seed, 0x43484c55ULL /* "CHLU" */);
    double *cdf = (double *)malloc((size_t)n * sizeof(double) + 8);
    double ex = -1.0 / (gamma - 1.0), run = 0.0;
    for (u32 i = 0; i < n; i++) { run += pow((double)i + i0, ex); cdf[i] = run; }
    for (u32 i = 0; i < n; i++) cdf[i] /= run;
    cdf[n - 1] = 1.0;
#pragma omp parallel for schedule(static) if (parallel)
    for (long long i = 0; i < (long long)samples; i++) {
        u32 e[2];
        for (int s = 0; s < 2; s++) {
            double x = u01(rnd(key, 2 * (u64)i + (u64)s));
            /* first index with cdf > x */
            u32 lo = 0, hi = n - 1;
            while (lo < hi) {
                u32 mid = lo + (hi - lo) / 2;
                if (cdf[mid] > x) hi = mid; else lo = mid + 1;
            }
            e[s] = lo;
        }
        keys[i] = pack_edge(e[0], e[1]);
    }
    free(cdf);
}

u64 gg_chung_lu(u32 n, double gamma, double i0, u64 samples, u64 seed, u32 *src, u32 *dst) {
    u64 *keys = (u64 *)malloc(samples * sizeof(u64) + 8);
    chung_lu_keys(n, gamma, i0, samples, seed, keys, 1);
    u64 m = finish_simple(keys, samples, n, src, dst);
    free(keys);
    return m;
}

static int cmp_u32(const void *a, const void *b) {
    u32 x = *(const u32 *)a, y = *(const u32 *)b;
    return x < y ? -1 : x > y;
}

void gg_degrees(u32 n, u64 m, const u32 *src, const u32 *dst, u32 *deg);
void gg_degree_order(u32 n, const u32 *deg, u32 *rank);

/* Single-threaded finish_simple: bucket the pairs by smaller endpoint,
 * sort and deduplicate each bucket.  Same output as finish_simple. */
static u64 finish_simple_serial(const u64 *keys, u64 nk, u32 n, u32 *src, u32 *dst) {
    u64 *off = (u64 *)calloc((size_t)n + 1, sizeof(u64));
    u32 *col = (u32 *)malloc(nk * sizeof(u32) + 4);
    for (u64 i = 0; i < nk; i++) if (keys[i] != UINT64_MAX) off[(keys[i] >> 32) + 1]++;
    for (u32 v = 0; v < n; v++) off[v + 1] += off[v];
    u64 *fill = (u64 *)malloc(((size_t)n + 1) * sizeof(u64));
    memcpy(fill, off, ((size_t)n + 1) * sizeof(u64));
    for (u64 i = 0; i < nk; i++)
        if (keys[i] != UINT64_MAX) col[fill[keys[i] >> 32]++] = (u32)(keys[i] & 0xffffffffu);
    free(fill);
    u64 m = 0;
    for (u32 v = 0; v < n; v++) {
        u32 *r = col + off[v];
        u64 len = off[v + 1] - off[v];
        if (len > 1) qsort(r, len, sizeof(u32), cmp_u32);
        for (u64 j = 0; j < len; j++) {
            if (j && r[j] == r[j - 1]) continue;
            src[m] = v;
            dst[m] = r[j];
            m++;
        }
    }
    free(col);
    free(off);
    return m;
}

/* k Chung-Lu graphs generated side by side (one thread per graph), each the
 * same as gg_chung_lu(n[i], gamma[i], i0, samples[i], seed[i]), followed by
 * its degree order.  Graph i's edges (local ids, src < dst, sorted) go to
 * [ebase[i], ebase[i+1]) of src/dst, which must hold sum(samples) entries;
 * its ranks go to rank[vbase[i] .. + n[i]) with vbase the prefix of n. */
void gg_chung_lu_batch(u32 k, const u32 *n, const double *gamma, const u64 *samples, const u64 *seed, double i0,
                       u64 *ebase, u32 *src, u32 *dst, u32 *rank) {
    u64 *cap = (u64 *)malloc(((size_t)k + 1) * sizeof(u64));
    u64 *vb = (u64 *)malloc(((size_t)k + 1) * sizeof(u64));
    u64 *mm = (u64 *)malloc(((size_t)k + 1) * sizeof(u64));
    cap[0] = 0;
    vb[0] = 0;
    for (u32 i = 0; i < k; i++) {
        cap[i + 1] = cap[i] + samples[i];
        vb[i + 1] = vb[i] + n[i];
    }
#pragma omp parallel
    {
        u64 kcap = 0;
        u64 *keys = NULL;
        u32 *deg = NULL;
        u32 dcap = 0;
#pragma omp for schedule(dynamic, 1)
        for (long long ii = 0; ii < (long long)k; ii++) {
            u32 i = (u32)ii;
            if (samples[i] + 1 > kcap) {
                free(keys);
                kcap = samples[i] + 1;
                keys = (u64 *)malloc(kcap * sizeof(u64));
            }
            if (n[i] + 1 > dcap) {
                free(deg);
                dcap = n[i] + 1;
                deg = (u32 *)malloc((size_t)dcap * sizeof(u32));
            }
            u64 m = 0;
            if (n[i] && samples[i]) {
                chung_lu_keys(n[i], gamma[i], i0, samples[i], seed[i], keys, 0);
                m = finish_simple_serial(keys, samples[i], n[i], src + cap[i], dst + cap[i]);
            }
            mm[i] = m;
            if (n[i]) {
                gg_degrees(n[i], m, src + cap[i], dst + cap[i], deg);
                gg_degree_order(n[i], deg, rank + vb[i]);
            }
        }
        free(keys);
        free(deg);
    }
    /* close the gaps between graphs (each moves toward lower addresses) */
    ebase[0] = 0;
    for (u32 i = 0; i < k; i++) {
        ebase[i + 1] = ebase[i] + mm[i];
        if (mm[i] && ebase[i] != cap[i]) {
            memmove(src + ebase[i], src + cap[i], mm[i] * sizeof(u32));
            memmove(dst + ebase[i], dst + cap[i], mm[i] * sizeof(u32));
        }
    }
    free(cap);
    free(vb);
    free(mm);
}

/* Simplifies an arbitrary edge list (drops loops, dedups undirected pairs).
 * Output arrays may alias the inputs.  Returns m. */
u64 gg_simplify(u32 n, u64 m_in, const u32 *s, const u32 *d, u32 *src, u32 *dst) {
    u64 *keys = (u64 *)malloc(m_in * sizeof(u64) + 8);
    for (u64 i = 0; i < m_in; i++) keys[i] = pack_edge(s[i], d[i]);
    u64 m = finish_simple(keys, m_in, n, src, dst);
    free(keys);
    return m;
}

/* ------------------------------------------------------------- orderings */

void gg_degrees(u32 n, u64 m, const u32 *src, const u32 *dst, u32 *deg) {
    memset(deg, 0, (size_t)n * sizeof(u32));
    for (u64 i = 0; i < m; i++) { deg[src[i]]++; deg[dst[i]]++; }
}

/* rank[u] = position of u when vertices are sorted by (degree ascending,
 * id ascending).  Stable counting sort. */
void gg_degree_order(u32 n, const u32 *deg, u32 *rank) {
    u32 maxd = 0;
    for (u32 u = 0; u < n; u++) if (deg[u] > maxd) maxd = deg[u];
    u64 *cnt = (u64 *)calloc((size_t)maxd + 2, sizeof(u64));
    for (u32 u = 0; u < n; u++) cnt[deg[u] + 1]++;
    for (u32 d = 1; d <= maxd + 1; d++) cnt[d] += cnt[d - 1];
    for (u32 u = 0; u < n; u++) rank[u] = (u32)(cnt[deg[u]]++);
    free(cnt);
}

/* Uniform random permutation (Fisher-Yates driven by the counter stream). */
void gg_random_order(u32 n, u64 seed, u32 *rank) {
    u64 key = stream_key(seed, 0x5045524dULL /* "PERM" */);
    u32 *perm = (u32 *)malloc((size_t)n * sizeof(u32) + 4);
    for (u32 i = 0; i < n; i++) perm[i] = i;
    for (u32 i = n; i > 1; i--) {
        u64 r = rnd(key, i);
        u32 j = (u32)(((unsigned __int128)r * i) >> 64); /* uniform in [0,i) */
        u32 t = perm[i - 1]; perm[i - 1] = perm[j]; perm[j] = t;
    }
    for (u32 i = 0; i < n; i++) rank[perm[i]] = i;
    free(perm);
}

/* Core (degeneracy) order: peel a vertex of minimum current degree, smallest
 * id first; rank = removal index.  Uses a binary heap with lazy deletion. */
typedef struct { u32 d, v; } hent;
static inline int hless(hent x, hent y) { return x.d < y.d || (x.d == y.d && x.v < y.v); }
static void hpush(hent *h, u64 *sz, hent e) {
    u64 i = (*sz)++;
    h[i] = e;
    while (i) {
        u64 p = (i - 1) / 2;
        if (!hless(h[i], h[p])) break;
        hent t = h[i]; h[i] = h[p]; h[p] = t; i = p;
    }
}
static hent hpop(hent *h, u64 *sz) {
    hent top = h[0];
    h[0] = h[--(*sz)];
    u64 i = 0;
    for (;;) {
        u64 l = 2 * i + 1, r = l + 1, s = i;
        if (l < *sz && hless(h[l], h[s])) s = l;
        if (r < *sz && hless(h[r], h[s])) s = r;
        if (s == i) break;
        hent t = h[i]; h[i] = h[s]; h[s] = t; i = s;
    }
    return top;
}
void gg_core_order(u32 n, u64 m, const u32 *src, const u32 *dst, u32 *rank, u32 *core) {
    u32 *deg = (u32 *)calloc((size_t)n + 1, sizeof(u32));
    for (u64 i = 0; i < m; i++) { deg[src[i]]++; deg[dst[i]]++; }
    u64 *off = (u64 *)calloc((size_t)n + 1, sizeof(u64));
    for (u32 u = 0; u < n; u++) off[u + 1] = off[u] + deg[u];
    u32 *adj = (u32 *)malloc(2 * m * sizeof(u32) + 4);
    u64 *cur = (u64 *)malloc(((size_t)n + 1) * sizeof(u64));
    memcpy(cur, off, ((size_t)n + 1) * sizeof(u64));
    for (u64 i = 0; i < m; i++) { adj[cur[src[i]]++] = dst[i]; adj[cur[dst[i]]++] = src[i]; }
    free(cur);
    unsigned char *gone = (unsigned char *)calloc((size_t)n + 1, 1);
    hent *h = (hent *)malloc((2 * m + n + 1) * sizeof(hent));
    u64 sz = 0;
    for (u32 u = 0; u < n; u++) hpush(h, &sz, (hent){deg[u], u});
    u32 next = 0, kcore = 0;
    while (sz) {
        hent e = hpop(h, &sz);
        if (gone[e.v] || e.d != deg[e.v]) continue;
        gone[e.v] = 1;
        if (e.d > kcore) kcore = e.d;
        if (core) core[e.v] = kcore;
        rank[e.v] = next++;
        for (u64 j = off[e.v]; j < off[e.v + 1]; j++) {
            u32 w = adj[j];
            if (!gone[w]) { deg[w]--; hpush(h, &sz, (hent){deg[w], w}); }
        }
    }
    free(h); free(gone); free(adj); free(off); free(deg);
}
