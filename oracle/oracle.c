/*
 * CPU ORACLE -- test infrastructure only.
 *
 * A plain, single-threaded, deliberately unoptimised statement of what the
 * GPU triangle-listing path computes.  Only the test-suite, the smoke check
 * and the benchmark's CPU-baseline leg may load it; the product path never
 * does.  It shares no code, header or table with the GPU library.
 *
 * Paper: Lecuyer, Jachiet, Magnien, Tabourier, "Tailored vertex ordering for
 * faster triangle listing in large graphs" (arXiv 2203.04774).
 *
 *   graph model        Section 1.3 (Notations): simple undirected G=(V,E),
 *                      ordering pi, DAG G_pi with (u,v) in E_pi iff
 *                      pi_u < pi_v, successors N+ and predecessors N-.
 *                      Input loops and duplicate pairs are dropped, as the
 *                      experimental setup does with its datasets (Sec. 4.1.1).
 *   listing            each triangle of G exactly once, found from the
 *                      definition (an edge and a vertex adjacent to both of
 *                      its ends) rather than by the paper's marking scheme;
 *                      the forms A++ (Algorithm 1), A+- (Algorithm 2) and
 *                      A-- (Section 2.1's footnote) fix which vertex of a
 *                      triangle is the outer-loop pivot, which matters only
 *                      when the pivots are restricted to a rank range.
 *   cost               Definition 1: C++ = sum_u d+_u d+_u,
 *                      C+- = sum_u d+_u d-_u.
 *   work               one unit per element scanned in the innermost loop of
 *                      Algorithms 1/2, taken from Property 1's count (each
 *                      seed edge scans one whole list); summed over all
 *                      pivots it equals C++ (A++) or C+- (A+-), which the
 *                      tests check against the costs computed separately.
 *
 * Output convention (not fixed by the paper): a triangle is reported as its
 * three original vertex ids sorted ascending, a < b < c.  The 64-bit
 * order-independent digest is the wrapping sum over triangles of
 *   h(a,b,c) = f(f((a << 32) | b) + c),
 * f = the splitmix64 output function (Steele, Lea, Flood, OOPSLA 2014).
 * Parity of the digest is unpinned by the paper; the tests pin f against
 * splitmix64's published output sequence and the sum against hashing the
 * brute-force triangle set.
 *
 * Orderings (degree, Split, coreness and core ordering, Check, Neigh) are stated
 * beside their functions below, each with the passage it follows.
 *
 * Restricting the outer loop to pivots whose rank lies in [lo, hi) lists
 * exactly the triangles whose pivot (w for A++, u for A+-, v for A--) has
 * such a rank;
 * the outer iterations are independent (Section 4.1.2), so ranges partition
 * the output.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef uint64_t u64;
typedef uint32_t u32;

enum { ORC_APP = 0, ORC_APM = 1, ORC_AMM = 2 };

static u64 orc_f(u64 z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

u64 orc_mix64(u64 z) { return orc_f(z); }

u64 orc_triangle_hash(u32 a, u32 b, u32 c) {
    return orc_f(orc_f(((u64)a << 32) | (u64)b) + (u64)c);
}

/* ------------------------------------------------------------ the graph */

/* Undirected simple graph as adjacency lists in original ids, plus the
 * oriented lists N+ and N- under a given rank. */
typedef struct {
    u32 n;
    u64 m;         /* undirected edges after dropping loops and duplicates */
    u64 *off;      /* n+1, into adj */
    u32 *adj;      /* 2m neighbour ids, each list sorted by id, no repeats */
    const u32 *rank;
    u64 *poff, *moff;  /* n+1 each */
    u32 *plus, *minus; /* N+_u and N-_u, in id order */
} graph;

static int cmp_u32(const void *a, const void *b) {
    u32 x = *(const u32 *)a, y = *(const u32 *)b;
    return (x > y) - (x < y);
}

static void graph_free(graph *g) {
    free(g->off); free(g->adj); free(g->poff); free(g->moff); free(g->plus); free(g->minus);
    memset(g, 0, sizeof *g);
}

/* Returns 0 on success, -1 on bad input (id >= n, rank not a permutation),
 * -2 on allocation failure. */
static int graph_build(graph *g, u32 n, u64 m_in, const u32 *src, const u32 *dst, const u32 *rank) {
    memset(g, 0, sizeof *g);
    g->n = n;
    g->rank = rank;
    /* rank must be a permutation of [0, n) */
    unsigned char *seen = (unsigned char *)calloc((size_t)n + 1, 1);
    if (!seen) return -2;
    for (u32 u = 0; u < n; u++) {
        if (rank[u] >= n || seen[rank[u]]) { free(seen); return -1; }
        seen[rank[u]] = 1;
    }
    free(seen);
    for (u64 i = 0; i < m_in; i++)
        if (src[i] >= n || dst[i] >= n) return -1;

    /* symmetric adjacency with loops removed */
    u64 *cnt = (u64 *)calloc((size_t)n + 1, sizeof(u64));
    if (!cnt) return -2;
    for (u64 i = 0; i < m_in; i++) {
        if (src[i] == dst[i]) continue;
        cnt[src[i]]++;
        cnt[dst[i]]++;
    }
    u64 *raw_off = (u64 *)calloc((size_t)n + 1, sizeof(u64));
    for (u32 u = 0; u < n; u++) raw_off[u + 1] = raw_off[u] + cnt[u];
    u32 *raw = (u32 *)malloc(raw_off[n] * sizeof(u32) + 4);
    if (!raw_off || !raw) { free(cnt); free(raw_off); free(raw); return -2; }
    memset(cnt, 0, ((size_t)n + 1) * sizeof(u64));
    for (u64 i = 0; i < m_in; i++) {
        u32 a = src[i], b = dst[i];
        if (a == b) continue;
        raw[raw_off[a] + cnt[a]++] = b;
        raw[raw_off[b] + cnt[b]++] = a;
    }
    /* sort each list and drop repeated neighbours (duplicate edges) */
    g->off = (u64 *)calloc((size_t)n + 1, sizeof(u64));
    u64 w = 0;
    for (u32 u = 0; u < n; u++) {
        u32 *row = raw + raw_off[u];
        u64 len = raw_off[u + 1] - raw_off[u];
        qsort(row, len, sizeof(u32), cmp_u32);
        g->off[u] = w;
        for (u64 j = 0; j < len; j++)
            if (j == 0 || row[j] != row[j - 1]) raw[w++] = row[j];
    }
    g->off[n] = w;
    g->adj = raw; /* compacted in place */
    g->m = w / 2;
    free(raw_off);
    free(cnt);

    /* orientation by rank: N+_u = {v : pi_v > pi_u}, N-_u = {v : pi_v < pi_u} */
    g->poff = (u64 *)calloc((size_t)n + 1, sizeof(u64));
    g->moff = (u64 *)calloc((size_t)n + 1, sizeof(u64));
    g->plus = (u32 *)malloc(g->m * sizeof(u32) + 4);
    g->minus = (u32 *)malloc(g->m * sizeof(u32) + 4);
    if (!g->off || !g->poff || !g->moff || !g->plus || !g->minus) { graph_free(g); return -2; }
    u64 pw = 0, mw = 0;
    for (u32 u = 0; u < n; u++) {
        g->poff[u] = pw;
        g->moff[u] = mw;
        for (u64 j = g->off[u]; j < g->off[u + 1]; j++) {
            u32 v = g->adj[j];
            if (rank[v] > rank[u]) g->plus[pw++] = v;
            else g->minus[mw++] = v;
        }
    }
    g->poff[n] = pw;
    g->moff[n] = mw;
    return 0;
}

#define DPLUS(g, u) ((g)->poff[(u) + 1] - (g)->poff[(u)])
#define DMINUS(g, u) ((g)->moff[(u) + 1] - (g)->moff[(u)])

/* ============================================================ listing
 *
 * What is listed has a plain definition (Section 1.3): a triangle is a set
 * of three vertices joined pairwise by edges, and the task is to report each
 * one exactly once.  Under the ordering pi the three vertices of a triangle
 * have distinct ranks r1 < r2 < r3, and in the DAG G_pi its edges are
 * r1 -> r2, r1 -> r3 and r2 -> r3 (Figure 1): one source, one middle
 * vertex, one sink.  Reporting a triangle once is reporting it under one of
 * these roles, and the three forms of Section 2.1 differ only in which role
 * their outer loop runs over (the pivot):
 *   A++ (Algorithm 1)  the sink r3     (outer vertex w)
 *   A+- (Algorithm 2)  the source r1   (outer vertex u)
 *   A--                the middle r2   (outer vertex v)
 * Listing "with pivots of rank in [lo, hi)" is therefore the set of
 * triangles whose vertex in the form's pivot role has a rank in [lo, hi).
 *
 * This file finds them from the definition, not by the paper's marking
 * scheme: a triangle is an edge together with a vertex adjacent to both of
 * its ends.  For a pivot p and each edge of p in the direction that keeps p
 * in its role, the third vertex ranges over the common part of the two
 * endpoint lists that the role allows, found by intersecting two sorted
 * lists:
 *   sink p:    for q in N-(p), third in N-(q) & N-(p)   (ranks third < q < p)
 *   source p:  for q in N+(p), third in N+(p) & N+(q)   (ranks p < q < third)
 *   middle p:  for q in N-(p), third in N+(q) & N+(p)   (ranks q < p < third)
 * Each triangle of the role appears exactly once: its other two vertices are
 * told apart by rank, the smaller-or-middle one being q.
 *
 * The paper's work (one unit per element of the innermost scan of
 * Algorithms 1/2) is taken from its counting instead of from a scan: for
 * each seed edge the form scans one whole list (Property 1):
 *   A++  pivot w, seeds u in N-(w), each scanning N+(u):  sum d+(u)
 *   A+-  pivot u, seeds v in N+(u), each scanning N+(v):  sum d+(v)
 *   A--  pivot v, seeds w in N+(v), each scanning N-(w):  sum d-(w)
 * Summed over all pivots these are Definition 1's costs by double counting,
 * which the tests check against the costs computed separately.
 */

/* The oriented graph in rank space: vertex r is the vertex of rank r, its
 * successor list P(r) and predecessor list M(r) hold ranks, ascending. */
typedef struct {
    u32 n;
    u64 m;
    u32 *inv;          /* inv[r] = original id of rank r */
    u64 *poff, *moff;  /* n+1 each */
    u32 *P, *M;
} dag;

static void dag_free(dag *d) {
    free(d->inv); free(d->poff); free(d->moff); free(d->P); free(d->M);
    memset(d, 0, sizeof *d);
}

/* Builds the DAG of the simple graph underlying (src, dst): loops and
 * repeated pairs (in either direction) are dropped.  Returns 0, -1 on bad
 * input (id >= n, rank not a permutation), -2 when out of memory. */
static int dag_build(dag *d, u32 n, u64 m_in, const u32 *src, const u32 *dst, const u32 *rank) {
    memset(d, 0, sizeof *d);
    d->n = n;
    d->inv = (u32 *)malloc((size_t)n * sizeof(u32) + 4);
    d->poff = (u64 *)calloc((size_t)n + 1, sizeof(u64));
    d->moff = (u64 *)calloc((size_t)n + 1, sizeof(u64));
    if (!d->inv || !d->poff || !d->moff) { dag_free(d); return -2; }
    for (u32 r = 0; r < n; r++) d->inv[r] = 0xffffffffu;
    for (u32 u = 0; u < n; u++) {
        if (rank[u] >= n || d->inv[rank[u]] != 0xffffffffu) { dag_free(d); return -1; }
        d->inv[rank[u]] = u;
    }
    for (u64 i = 0; i < m_in; i++)
        if (src[i] >= n || dst[i] >= n) { dag_free(d); return -1; }
    /* each edge, once per input pair, in the successor list of its lower end */
    for (u64 i = 0; i < m_in; i++) {
        if (src[i] == dst[i]) continue;
        u32 a = rank[src[i]], b = rank[dst[i]];
        d->poff[(a < b ? a : b) + 1]++;
    }
    for (u32 r = 0; r < n; r++) d->poff[r + 1] += d->poff[r];
    d->P = (u32 *)malloc(d->poff[n] * sizeof(u32) + 4);
    u64 *fill = (u64 *)calloc((size_t)n + 1, sizeof(u64));
    if (!d->P || !fill) { free(fill); dag_free(d); return -2; }
    for (u64 i = 0; i < m_in; i++) {
        if (src[i] == dst[i]) continue;
        u32 a = rank[src[i]], b = rank[dst[i]];
        u32 lo = a < b ? a : b, hi = a < b ? b : a;
        d->P[d->poff[lo] + fill[lo]++] = hi;
    }
    /* sort each list and keep one copy of each successor */
    u64 w = 0;
    for (u32 r = 0; r < n; r++) {
        u64 b0 = d->poff[r], b1 = d->poff[r + 1];
        qsort(d->P + b0, b1 - b0, sizeof(u32), cmp_u32);
        d->poff[r] = w;
        for (u64 j = b0; j < b1; j++)
            if (j == b0 || d->P[j] != d->P[j - 1]) d->P[w++] = d->P[j];
    }
    d->poff[n] = w;
    d->m = w;
    /* predecessor lists: walking the rows in rank order appends to each
     * list in ascending order */
    memset(fill, 0, ((size_t)n + 1) * sizeof(u64));
    for (u64 j = 0; j < w; j++) d->moff[d->P[j] + 1]++;
    for (u32 r = 0; r < n; r++) d->moff[r + 1] += d->moff[r];
    d->M = (u32 *)malloc(w * sizeof(u32) + 4);
    if (!d->M) { free(fill); dag_free(d); return -2; }
    for (u32 r = 0; r < n; r++)
        for (u64 j = d->poff[r]; j < d->poff[r + 1]; j++) {
            u32 s = d->P[j];
            d->M[d->moff[s] + fill[s]++] = r;
        }
    free(fill);
    return 0;
}

#define PLEN(d, r) ((d)->poff[(r) + 1] - (d)->poff[(r)])
#define MLEN(d, r) ((d)->moff[(r) + 1] - (d)->moff[(r)])

typedef struct {
    u64 count, hash;
    u32 *tri;      /* optional: 3*cap slots */
    u64 cap;
} sink;

/* A triangle found in rank space: reported as its three original ids sorted
 * ascending (the output convention), counted and hashed. */
static void found(const dag *d, sink *s, u32 ra, u32 rb, u32 rc) {
    u32 x = d->inv[ra], y = d->inv[rb], z = d->inv[rc], t;
    if (x > y) { t = x; x = y; y = t; }
    if (y > z) { t = y; y = z; z = t; }
    if (x > y) { t = x; x = y; y = t; }
    if (s->tri && s->count < s->cap) {
        s->tri[3 * s->count + 0] = x;
        s->tri[3 * s->count + 1] = y;
        s->tri[3 * s->count + 2] = z;
    }
    s->count++;
    s->hash += orc_triangle_hash(x, y, z);
}

/* Position of the first element >= key in the ascending list a[0..len). */
static u64 first_at_least(const u32 *a, u64 len, u32 key) {
    u64 lo = 0, hi = len;
    while (lo < hi) {
        u64 mid = lo + (hi - lo) / 2;
        if (a[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

/* The elements common to the ascending lists a[0..la) and b[0..lb), in
 * ascending order, written to out (room for min(la, lb)); returns how many.
 * Lists of similar length are merged; when one is more than 16 times longer
 * each element of the shorter is looked up in it by binary search. */
static u64 intersect(const u32 *a, u64 la, const u32 *b, u64 lb, u32 *out) {
    u64 k = 0;
    if (la > lb) { const u32 *t = a; a = b; b = t; u64 tl = la; la = lb; lb = tl; }
    if (la * 16 < lb) {
        for (u64 i = 0; i < la; i++) {
            u64 j = first_at_least(b, lb, a[i]);
            if (j < lb && b[j] == a[i]) out[k++] = a[i];
        }
        return k;
    }
    u64 i = 0, j = 0;
    while (i < la && j < lb) {
        if (a[i] < b[j]) i++;
        else if (a[i] > b[j]) j++;
        else { out[k++] = a[i]; i++; j++; }
    }
    return k;
}

/* Triangles in which vertex p has the pivot role of the form (see above). */
static void triangles_at(const dag *d, int algo, u32 p, u32 *scratch, sink *s) {
    if (algo == ORC_APP) {             /* p is the sink */
        const u32 *Mp = d->M + d->moff[p];
        for (u64 j = 0; j < MLEN(d, p); j++) {
            u32 q = Mp[j];
            u64 k = intersect(d->M + d->moff[q], MLEN(d, q), Mp, MLEN(d, p), scratch);
            for (u64 i = 0; i < k; i++) found(d, s, scratch[i], q, p);
        }
    } else if (algo == ORC_APM) {      /* p is the source */
        const u32 *Pp = d->P + d->poff[p];
        for (u64 j = 0; j < PLEN(d, p); j++) {
            u32 q = Pp[j];
            u64 k = intersect(Pp, PLEN(d, p), d->P + d->poff[q], PLEN(d, q), scratch);
            for (u64 i = 0; i < k; i++) found(d, s, p, q, scratch[i]);
        }
    } else {                           /* p is the middle vertex */
        const u32 *Mp = d->M + d->moff[p];
        for (u64 j = 0; j < MLEN(d, p); j++) {
            u32 q = Mp[j];
            u64 k = intersect(d->P + d->poff[q], PLEN(d, q), d->P + d->poff[p], PLEN(d, p), scratch);
            for (u64 i = 0; i < k; i++) found(d, s, q, p, scratch[i]);
        }
    }
}

/* The paper's work for pivot p (Property 1's count; see above). */
static u64 work_at(const dag *d, int algo, u32 p) {
    u64 w = 0;
    if (algo == ORC_APP)
        for (u64 j = d->moff[p]; j < d->moff[p + 1]; j++) w += PLEN(d, d->M[j]);
    else if (algo == ORC_APM)
        for (u64 j = d->poff[p]; j < d->poff[p + 1]; j++) w += PLEN(d, d->P[j]);
    else
        for (u64 j = d->poff[p]; j < d->poff[p + 1]; j++) w += MLEN(d, d->P[j]);
    return w;
}

static u32 *scratch_for(const dag *d) {
    u64 mx = 1;
    for (u32 r = 0; r < d->n; r++) {
        if (PLEN(d, r) > mx) mx = PLEN(d, r);
        if (MLEN(d, r) > mx) mx = MLEN(d, r);
    }
    return (u32 *)malloc(mx * sizeof(u32));
}

/* Triangles whose pivot (the form's role) has rank in [lo, hi), and the
 * paper's work over those pivots.  out[0..3] = count, hash, work, m. */
static int dag_list(const dag *d, int algo, u32 lo, u32 hi, u32 *tri, u64 cap, u64 *out) {
    if (algo != ORC_APP && algo != ORC_APM && algo != ORC_AMM) return -1;
    if (hi > d->n) hi = d->n;
    u32 *scratch = scratch_for(d);
    if (!scratch) return -2;
    sink s = {0, 0, tri, cap};
    u64 work = 0;
    for (u32 p = lo; p < hi; p++) {
        triangles_at(d, algo, p, scratch, &s);
        work += work_at(d, algo, p);
    }
    free(scratch);
    out[0] = s.count;
    out[1] = s.hash;
    out[2] = work;
    out[3] = d->m;
    return 0;
}

/* ================================================================ ABI */

/*
 * Lists the triangles of the simple graph underlying (src, dst) under the
 * ordering `rank` whose pivot for the form (0: A++, Algorithm 1; 1: A+-,
 * Algorithm 2; 2: A--) has rank in [lo, hi).
 * out[0..2] = count, hash, work; out[3] = m after simplification.
 * If tri != NULL, the first min(count, cap) canonical triangles are written
 * there (3 ids each) in the order found.
 * Returns 0, -1 (invalid input) or -2 (out of memory).
 */
int orc_list(u32 n, u64 m_in, const u32 *src, const u32 *dst, const u32 *rank, int algo,
             u32 lo, u32 hi, u32 *tri, u64 cap, u64 *out) {
    dag d;
    int rc = dag_build(&d, n, m_in, src, dst, rank);
    if (rc) return rc;
    rc = dag_list(&d, algo, lo, hi, tri, cap, out);
    dag_free(&d);
    return rc;
}

/*
 * As orc_list, for nr pivot ranges [lo[i], hi[i]) over one graph build.
 * tri[i] (may be NULL) receives up to cap[i] triangles of range i;
 * out[4*i .. 4*i+3] = count, hash, work, m for range i.
 */
int orc_list_ranges(u32 n, u64 m_in, const u32 *src, const u32 *dst, const u32 *rank, int algo, u32 nr,
                    const u32 *lo, const u32 *hi, u32 **tri, const u64 *cap, u64 *out) {
    dag d;
    int rc = dag_build(&d, n, m_in, src, dst, rank);
    if (rc) return rc;
    for (u32 i = 0; i < nr && !rc; i++)
        rc = dag_list(&d, algo, lo[i], hi[i], tri ? tri[i] : 0, cap ? cap[i] : 0, out + 4 * i);
    dag_free(&d);
    return rc;
}

/* A graph built once (for listing many pivot ranges). */
void *orc_graph_new(u32 n, u64 m_in, const u32 *src, const u32 *dst, const u32 *rank, int *rc) {
    dag *d = (dag *)calloc(1, sizeof(dag));
    if (!d) { *rc = -2; return 0; }
    *rc = dag_build(d, n, m_in, src, dst, rank);
    if (*rc) { free(d); return 0; }
    return d;
}

int orc_graph_list(void *h, int algo, u32 lo, u32 hi, u32 *tri, u64 cap, u64 *out) {
    return dag_list((const dag *)h, algo, lo, hi, tri, cap, out);
}

/*
 * Every triangle whose source (smallest rank) lies in [src_lo, src_hi),
 * sorted into bins by the rank of its pivot for the form: bin i holds the
 * triangles whose pivot rank lies in [cut[i], cut[i+1]), for nb bins over
 * ascending cuts (cut has nb+1 entries; triangles outside [cut[0], cut[nb])
 * are not counted).  out[2*i], out[2*i+1] += count, hash of bin i.
 * Source ranges partition the triangles, so summing this over a partition of
 * [0, n) gives each bin's (count, hash) for the whole graph: one pass over
 * all triangles for many pivot ranges at once.
 */
int orc_graph_bin(void *h, int algo, u32 src_lo, u32 src_hi, u32 nb, const u32 *cut, u64 *out) {
    const dag *d = (const dag *)h;
    if (algo != ORC_APP && algo != ORC_APM && algo != ORC_AMM) return -1;
    for (u32 i = 0; i < nb; i++)
        if (cut[i] > cut[i + 1]) return -1;
    if (src_hi > d->n) src_hi = d->n;
    u32 *scratch = scratch_for(d);
    if (!scratch) return -2;
    for (u32 p = src_lo; p < src_hi; p++) {
        const u32 *Pp = d->P + d->poff[p];
        for (u64 j = 0; j < PLEN(d, p); j++) {
            u32 q = Pp[j];
            u64 k = intersect(Pp, PLEN(d, p), d->P + d->poff[q], PLEN(d, q), scratch);
            for (u64 i = 0; i < k; i++) {
                u32 t = scratch[i];  /* ranks p < q < t */
                u32 piv = algo == ORC_APP ? t : (algo == ORC_APM ? p : q);
                if (piv < cut[0] || piv >= cut[nb]) continue;
                u64 lo = 0, hi = nb;  /* the bin with cut[b] <= piv < cut[b+1] */
                while (hi - lo > 1) {
                    u64 mid = (lo + hi) / 2;
                    if (cut[mid] <= piv) lo = mid; else hi = mid;
                }
                sink s = {0, 0, 0, 0};
                found(d, &s, p, q, t);
                out[2 * lo] += 1;
                out[2 * lo + 1] += s.hash;
            }
        }
    }
    free(scratch);
    return 0;
}

/* The paper's work of the form over pivots of rank in [lo, hi). */
u64 orc_graph_work(void *h, int algo, u32 lo, u32 hi) {
    const dag *d = (const dag *)h;
    u64 w = 0;
    if (hi > d->n) hi = d->n;
    for (u32 p = lo; p < hi; p++) w += work_at(d, algo, p);
    return w;
}

u64 orc_graph_m(void *h) { return ((const dag *)h)->m; }

void orc_graph_free(void *h) {
    dag *d = (dag *)h;
    if (!d) return;
    dag_free(d);
    free(d);
}

/*
 * Definition 1 costs.  out[0] = C++ = sum d+ d+, out[1] = C+- = sum d+ d-,
 * out[2] = sum d- d-, out[3] = m, out[4] = sum d+, out[5] = sum d-.
 */
int orc_cost(u32 n, u64 m_in, const u32 *src, const u32 *dst, const u32 *rank, u64 *out) {
    graph g;
    int rc = graph_build(&g, n, m_in, src, dst, rank);
    if (rc) return rc;
    u64 cpp = 0, cpm = 0, cmm = 0, sp = 0, sm = 0;
    for (u32 u = 0; u < n; u++) {
        u64 dp = DPLUS(&g, u), dm = DMINUS(&g, u);
        cpp += dp * dp;
        cpm += dp * dm;
        cmm += dm * dm;
        sp += dp;
        sm += dm;
    }
    out[0] = cpp; out[1] = cpm; out[2] = cmm; out[3] = g.m; out[4] = sp; out[5] = sm;
    graph_free(&g);
    return 0;
}

/*
 * The oriented graph in rank space, for comparing CSR arrays: row r holds
 * the ranks of the successors of the vertex of rank r, ascending.
 * fwd_off has n+1 entries, fwd_adj m entries (caller sizes it with m from
 * orc_cost); bwd_* likewise hold the predecessors.  inv[r] = vertex of rank r.
 */
int orc_oriented_csr(u32 n, u64 m_in, const u32 *src, const u32 *dst, const u32 *rank,
                     u64 *fwd_off, u32 *fwd_adj, u64 *bwd_off, u32 *bwd_adj, u32 *inv) {
    graph g;
    int rc = graph_build(&g, n, m_in, src, dst, rank);
    if (rc) return rc;
    for (u32 u = 0; u < n; u++) inv[rank[u]] = u;
    u64 pw = 0, mw = 0;
    for (u32 r = 0; r < n; r++) {
        u32 u = inv[r];
        fwd_off[r] = pw;
        for (u64 j = g.poff[u]; j < g.poff[u + 1]; j++) fwd_adj[pw++] = rank[g.plus[j]];
        qsort(fwd_adj + fwd_off[r], pw - fwd_off[r], sizeof(u32), cmp_u32);
        bwd_off[r] = mw;
        for (u64 j = g.moff[u]; j < g.moff[u + 1]; j++) bwd_adj[mw++] = rank[g.minus[j]];
        qsort(bwd_adj + bwd_off[r], mw - bwd_off[r], sizeof(u32), cmp_u32);
    }
    fwd_off[n] = pw;
    bwd_off[n] = mw;
    graph_free(&g);
    return 0;
}

/* ============================================================ orderings */

/*
 * Degree ordering (Section 2.2): vertices by non-decreasing degree in the
 * simple graph, ties by increasing id; rank[u] = position of u.
 */
typedef struct {
    u32 deg, id;
} degkey;

static int cmp_degkey(const void *a, const void *b) {
    const degkey *x = (const degkey *)a, *y = (const degkey *)b;
    if (x->deg != y->deg) return (x->deg > y->deg) - (x->deg < y->deg);
    return (x->id > y->id) - (x->id < y->id);
}

static int degree_positions(u32 n, u64 m_in, const u32 *src, const u32 *dst, u32 *order) {
    u32 *ident = (u32 *)malloc((size_t)n * sizeof(u32) + 4);
    degkey *k = (degkey *)malloc((size_t)n * sizeof(degkey) + 8);
    if (!ident || !k) { free(ident); free(k); return -2; }
    for (u32 u = 0; u < n; u++) ident[u] = u;
    graph g;
    int rc = graph_build(&g, n, m_in, src, dst, ident);
    if (rc) { free(ident); free(k); return rc; }
    for (u32 u = 0; u < n; u++) {
        k[u].deg = (u32)(g.off[u + 1] - g.off[u]);
        k[u].id = u;
    }
    qsort(k, n, sizeof(degkey), cmp_degkey);
    for (u32 i = 0; i < n; i++) order[i] = k[i].id;
    graph_free(&g);
    free(ident);
    free(k);
    return 0;
}

int orc_degree_order(u32 n, u64 m_in, const u32 *src, const u32 *dst, u32 *rank) {
    u32 *order = (u32 *)malloc((size_t)n * sizeof(u32) + 4);
    if (!order) return -2;
    int rc = degree_positions(n, m_in, src, dst, order);
    if (!rc)
        for (u32 i = 0; i < n; i++) rank[order[i]] = i;
    free(order);
    return rc;
}

/*
 * Split (Section 3.3.3): take a non-increasing degree ordering delta
 * (1-based positions) -- here the degree ordering above read backwards --
 * and send the vertex at position 2i+1 to index i+1, the vertex at
 * position 2i to index n+1-i.  rank[u] = index - 1.
 */
int orc_split_order(u32 n, u64 m_in, const u32 *src, const u32 *dst, u32 *rank) {
    u32 *order = (u32 *)malloc((size_t)n * sizeof(u32) + 4);
    if (!order) return -2;
    int rc = degree_positions(n, m_in, src, dst, order);
    if (!rc) {
        for (u32 pos = 1; pos <= n; pos++) {    /* delta position, 1-based */
            u32 u = order[n - pos];             /* non-increasing degree */
            u32 index = (pos % 2 == 1) ? (pos - 1) / 2 + 1 : n + 1 - pos / 2;
            rank[u] = index - 1;
        }
    }
    free(order);
    return rc;
}

/*
 * Coreness (Section 1.3): c_u is the largest k such that u belongs to a
 * subgraph in which every vertex has degree at least k.  Computed by
 * bucket peeling in order of current degree (linear time, as Section 1.3
 * notes): repeatedly remove a vertex of minimum current degree; its
 * coreness is the largest minimum degree seen so far.
 * Core ordering: non-decreasing coreness, ties by id (Section 1.3 fixes
 * only the coreness order); rank[u] = position.
 */
int orc_coreness(u32 n, u64 m_in, const u32 *src, const u32 *dst, u32 *core) {
    u32 *ident = (u32 *)malloc((size_t)n * sizeof(u32) + 4);
    if (!ident) return -2;
    for (u32 u = 0; u < n; u++) ident[u] = u;
    graph g;
    int rc = graph_build(&g, n, m_in, src, dst, ident);
    free(ident);
    if (rc) return rc;
    u32 maxd = 0;
    u32 *deg = (u32 *)malloc((size_t)n * sizeof(u32) + 4);
    unsigned char *gone = (unsigned char *)calloc((size_t)n + 1, 1);
    for (u32 u = 0; u < n; u++) {
        deg[u] = (u32)(g.off[u + 1] - g.off[u]);
        if (deg[u] > maxd) maxd = deg[u];
    }
    /* buckets of vertices by current degree, as doubly linked lists */
    u32 *head = (u32 *)malloc(((size_t)maxd + 1) * sizeof(u32));
    u32 *next = (u32 *)malloc((size_t)n * sizeof(u32) + 4);
    u32 *prev = (u32 *)malloc((size_t)n * sizeof(u32) + 4);
    const u32 NIL = 0xffffffffu;
    for (u32 d = 0; d <= maxd; d++) head[d] = NIL;
    for (u32 u = n; u-- > 0;) {  /* so that each list starts with its smallest id */
        prev[u] = NIL;
        next[u] = head[deg[u]];
        if (head[deg[u]] != NIL) prev[head[deg[u]]] = u;
        head[deg[u]] = u;
    }
    u32 level = 0, d = 0;
    for (u32 removed = 0; removed < n; removed++) {
        while (head[d] == NIL) d++;
        u32 u = head[d];
        head[d] = next[u];
        if (next[u] != NIL) prev[next[u]] = NIL;
        gone[u] = 1;
        if (d > level) level = d;
        core[u] = level;
        for (u64 j = g.off[u]; j < g.off[u + 1]; j++) {
            u32 w = g.adj[j];
            if (gone[w]) continue;
            /* move w from bucket deg[w] to deg[w] - 1 */
            u32 dw = deg[w];
            if (prev[w] != NIL) next[prev[w]] = next[w]; else head[dw] = next[w];
            if (next[w] != NIL) prev[next[w]] = prev[w];
            deg[w] = dw - 1;
            prev[w] = NIL;
            next[w] = head[dw - 1];
            if (head[dw - 1] != NIL) prev[head[dw - 1]] = w;
            head[dw - 1] = w;
            if (dw - 1 < d) d = dw - 1;
        }
    }
    free(head); free(next); free(prev); free(deg); free(gone);
    graph_free(&g);
    return 0;
}

int orc_core_order(u32 n, u64 m_in, const u32 *src, const u32 *dst, u32 *rank) {
    u32 *core = (u32 *)malloc((size_t)n * sizeof(u32) + 4);
    degkey *k = (degkey *)malloc((size_t)n * sizeof(degkey) + 8);
    if (!core || !k) { free(core); free(k); return -2; }
    int rc = orc_coreness(n, m_in, src, dst, core);
    if (!rc) {
        for (u32 u = 0; u < n; u++) { k[u].deg = core[u]; k[u].id = u; }
        qsort(k, n, sizeof(degkey), cmp_degkey);
        for (u32 i = 0; i < n; i++) rank[k[i].id] = i;
    }
    free(core);
    free(k);
    return rc;
}

/*
 * Check (Section 3.3.2): vertices are taken by non-increasing degree (the
 * degree ordering read backwards, as for Split).  Before u is placed, its
 * neighbours split into N_b (placed at the beginning), N_e (placed at the
 * end) and N_? (not placed yet).  Placed right after the beginning block,
 * u costs C_b = |N_b| (|N_e| + |N_?|); placed right before the end block,
 * C_e = (|N_b| + |N_?|) |N_e|.  The cheaper side is taken; on equal costs
 * the beginning (a reading: the paper does not say).  Beginning positions
 * are handed out 1, 2, ... and end positions n, n-1, ...; rank[u] =
 * position - 1.  side[u] (optional) = 0 for beginning, 1 for end.
 */
int orc_check_order(u32 n, u64 m_in, const u32 *src, const u32 *dst, u32 *rank, unsigned char *side) {
    u32 *order = (u32 *)malloc((size_t)n * sizeof(u32) + 4);
    u32 *ident = (u32 *)malloc((size_t)n * sizeof(u32) + 4);
    unsigned char *where = (unsigned char *)malloc((size_t)n + 1);  /* 0 unplaced, 1 beginning, 2 end */
    if (!order || !ident || !where) { free(order); free(ident); free(where); return -2; }
    int rc = degree_positions(n, m_in, src, dst, order);
    graph g;
    if (!rc) {
        for (u32 u = 0; u < n; u++) ident[u] = u;
        rc = graph_build(&g, n, m_in, src, dst, ident);
    }
    if (!rc) {
        memset(where, 0, (size_t)n + 1);
        u32 n_begin = 0, n_end = 0;
        for (u32 i = 0; i < n; i++) {
            u32 u = order[n - 1 - i];  /* non-increasing degree */
            u64 nb = 0, ne = 0, nq = 0;
            for (u64 j = g.off[u]; j < g.off[u + 1]; j++) {
                unsigned char w = where[g.adj[j]];
                if (w == 1) nb++;
                else if (w == 2) ne++;
                else nq++;
            }
            u64 cb = nb * (ne + nq), ce = (nb + nq) * ne;
            if (cb <= ce) {
                where[u] = 1;
                n_begin++;
                rank[u] = n_begin - 1;        /* position |V_b| + 1 */
            } else {
                where[u] = 2;
                rank[u] = n - n_end - 1;      /* position n - |V_e| */
                n_end++;
            }
            if (side) side[u] = where[u] - 1;
        }
        graph_free(&g);
    }
    free(order); free(ident); free(where);
    return rc;
}

/*
 * Neigh (Algorithm 3, Section 3.3.1): a pass visits every vertex u and
 * moves it to the place among its neighbours that gives the lowest C+-:
 * with N_u sorted by the current order as v_1 .. v_d, candidate p = 1..d
 * puts u right after v_p, candidate 0 right before v_1.  Passes repeat
 * while a pass brings C+- below (1 - eps) times its value at the pass's
 * start (the algorithm's loop condition), at most max_passes times.
 * Readings (the paper leaves them open): a pass visits vertices by
 * increasing id; when u's current place is among the cheapest it stays
 * put, otherwise the smallest cheapest p is taken.
 * Every candidate's C+- is computed from scratch on the candidate order
 * (Definition 1), and the order is a plain array: slow, for small graphs.
 * max_visits > 0 stops after that many vertex visits (for checking single
 * moves).  rank_in: the starting order; rank_out: the result.
 */
static u64 cpm_of_positions(const graph *g, const u32 *pos) {
    u64 c = 0;
    for (u32 u = 0; u < g->n; u++) {
        u64 plus = 0, d = g->off[u + 1] - g->off[u];
        for (u64 j = g->off[u]; j < g->off[u + 1]; j++) plus += pos[g->adj[j]] > pos[u];
        c += plus * (d - plus);
    }
    return c;
}

/* order without u, then u inserted at index `at` of that shorter order */
static void place(const u32 *order, u32 n, u32 u, u32 at, u32 *out) {
    u32 k = 0;
    for (u32 i = 0; i < n; i++) {
        if (order[i] == u) continue;
        if (k == at) out[k++] = u;
        out[k++] = order[i];
    }
    if (k == at) out[k++] = u;
}

static int cmp_u64(const void *a, const void *b) {
    u64 x = *(const u64 *)a, y = *(const u64 *)b;
    return (x > y) - (x < y);
}

int orc_neigh_order(u32 n, u64 m_in, const u32 *src, const u32 *dst, const u32 *rank_in, double eps,
                    u32 max_passes, u32 max_visits, u32 *rank_out, u64 *cpm_out, u32 *passes_out) {
    u32 *ident = (u32 *)malloc((size_t)n * sizeof(u32) + 4);
    if (!ident) return -2;
    for (u32 u = 0; u < n; u++) ident[u] = u;
    graph g;
    int rc = graph_build(&g, n, m_in, src, dst, ident);
    free(ident);
    if (rc) return rc;
    /* rank_in must be a permutation */
    unsigned char *seen = (unsigned char *)calloc((size_t)n + 1, 1);
    u32 *order = (u32 *)malloc((size_t)n * sizeof(u32) + 4);
    u32 *cand = (u32 *)malloc((size_t)n * sizeof(u32) + 4);
    u32 *pos = (u32 *)malloc((size_t)n * sizeof(u32) + 4);
    u32 *cpos = (u32 *)malloc((size_t)n * sizeof(u32) + 4);
    u64 maxd = 0;
    for (u32 u = 0; u < n; u++)
        if (g.off[u + 1] - g.off[u] > maxd) maxd = g.off[u + 1] - g.off[u];
    u64 *nb = (u64 *)malloc((size_t)(maxd + 1) * sizeof(u64));
    u64 *cost = (u64 *)malloc((size_t)(maxd + 1) * sizeof(u64));
    if (!seen || !order || !cand || !pos || !cpos || !nb || !cost) rc = -2;
    for (u32 u = 0; !rc && u < n; u++) {
        if (rank_in[u] >= n || seen[rank_in[u]]) rc = -1;
        else { seen[rank_in[u]] = 1; pos[u] = rank_in[u]; order[rank_in[u]] = u; }
    }
    u64 c = 0;
    u32 passes = 0, visits = 0;
    int stop = 0;
    if (!rc) {
        c = cpm_of_positions(&g, pos);
        while (!stop && passes < max_passes) {
            const u64 c0 = c;
            for (u32 u = 0; u < n && !stop; u++) {
                if (max_visits && visits == max_visits) { stop = 1; break; }
                visits++;
                const u64 d = g.off[u + 1] - g.off[u];
                if (d == 0) continue;
                /* neighbours by current position */
                for (u64 j = 0; j < d; j++) {
                    u32 v = g.adj[g.off[u] + j];
                    nb[j] = ((u64)pos[v] << 32) | v;
                }
                qsort(nb, d, sizeof(u64), cmp_u64);
                u64 pcur = 0;
                for (u64 j = 0; j < d; j++) pcur += (u32)(nb[j] >> 32) < pos[u];
                /* C+- of every candidate, from scratch */
                u64 best = ~0ull;
                for (u64 p = 0; p <= d; p++) {
                    u32 at;
                    if (p == 0) {
                        u32 v1 = (u32)nb[0];
                        at = pos[v1] - (pos[u] < pos[v1] ? 1 : 0);  /* index of v_1 once u is out */
                    } else {
                        u32 vp = (u32)nb[p - 1];
                        at = pos[vp] - (pos[u] < pos[vp] ? 1 : 0) + 1;
                    }
                    place(order, n, u, at, cand);
                    for (u32 i = 0; i < n; i++) cpos[cand[i]] = i;
                    cost[p] = cpm_of_positions(&g, cpos);
                    if (cost[p] < best) best = cost[p];
                }
                u64 pstar = pcur;
                if (cost[pcur] != best) {
                    for (pstar = 0; cost[pstar] != best; pstar++) {}
                }
                if (pstar != pcur) {
                    u32 at;
                    if (pstar == 0) {
                        u32 v1 = (u32)nb[0];
                        at = pos[v1] - (pos[u] < pos[v1] ? 1 : 0);
                    } else {
                        u32 vp = (u32)nb[pstar - 1];
                        at = pos[vp] - (pos[u] < pos[vp] ? 1 : 0) + 1;
                    }
                    place(order, n, u, at, cand);
                    memcpy(order, cand, (size_t)n * sizeof(u32));
                    for (u32 i = 0; i < n; i++) pos[order[i]] = i;
                    c = best;
                }
            }
            if (stop) break;
            passes++;
            if (!((double)c < (1.0 - eps) * (double)c0)) break;
        }
        for (u32 u = 0; u < n; u++) rank_out[u] = pos[u];
        if (cpm_out) *cpm_out = c;
        if (passes_out) *passes_out = passes;
    }
    free(seen); free(order); free(cand); free(pos); free(cpos); free(nb); free(cost);
    graph_free(&g);
    return rc;
}
