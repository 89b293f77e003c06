"""Small fixture graphs with closed-form properties (test helpers).

Each returns ``(n, src, dst)`` with uint32 edge arrays.  Edges are given as
unordered pairs, possibly in either direction; the library and the oracle
both drop loops and duplicates.
"""
from __future__ import annotations

import itertools
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _pack(n, pairs):
    if len(pairs) == 0:
        return n, np.zeros(0, np.uint32), np.zeros(0, np.uint32)
    a = np.asarray(pairs, dtype=np.uint32).reshape(-1, 2)
    return n, np.ascontiguousarray(a[:, 0]), np.ascontiguousarray(a[:, 1])


def complete(n):
    return _pack(n, list(itertools.combinations(range(n), 2)))


def wheel(n):
    """Hub 0 joined to a cycle on vertices 1..n-1 (n >= 4)."""
    k = n - 1
    pairs = [(0, i) for i in range(1, n)] + [(1 + i, 1 + (i + 1) % k) for i in range(k)]
    return _pack(n, pairs)


def cycle(n):
    return _pack(n, [(i, (i + 1) % n) for i in range(n)])


def grid(r, c):
    pairs = []
    for i in range(r):
        for j in range(c):
            v = i * c + j
            if j + 1 < c:
                pairs.append((v, v + 1))
            if i + 1 < r:
                pairs.append((v, v + c))
    return _pack(r * c, pairs)


def complete_bipartite(a, b):
    return _pack(a + b, [(i, a + j) for i in range(a) for j in range(b)])


def random_bipartite(a, b, p, seed):
    rs = np.random.default_rng(seed)
    pairs = [(i, a + j) for i in range(a) for j in range(b) if rs.random() < p]
    return _pack(a + b, pairs)


def star(n):
    return _pack(n, [(0, i) for i in range(1, n)])


def erdos_renyi(n, p, seed):
    rs = np.random.default_rng(seed)
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n) if rs.random() < p]
    return _pack(n, pairs)


def ld_gadget(d):
    """L_d of Appendix B.  Ids: e_d = 0, v_i = i (1..d), K_i = d+1+i (0..d).
    Returns (n, src, dst, order) with `order` = e_d, v_1..v_d, K_d..K_0."""
    e = 0
    v = [1 + i for i in range(d)]
    K = [d + 1 + i for i in range(d + 1)]
    pairs = [(e, x) for x in v] + [(x, k) for x in v for k in K]
    pairs += list(itertools.combinations(K, 2))
    n = 2 * d + 2
    order = [e] + v + K[::-1]
    return (*_pack(n, pairs), order)


def gphi_gadget(n_vars, n_clauses, seed):
    """G_phi of Appendix A for a random satisfiable NAE3SAT+ instance.

    A truth assignment is drawn first; every clause takes three distinct
    variables that are not all equal under it.  Ids: X_i = i, and literal
    L_j^a = n_vars + 3 j + a.  Returns (n, src, dst, order_vertices) where
    the order is the one built in the proof of the forward direction: true
    variables, false literals, other literals, true literals, false variables.
    """
    rs = np.random.default_rng(seed)
    assign = rs.random(n_vars) < 0.5
    assign[0], assign[1] = True, False  # both truth values present
    clauses = []
    while len(clauses) < n_clauses:
        c = rs.choice(n_vars, size=3, replace=False)
        vals = assign[c]
        if vals.all() or (~vals).all():
            continue
        clauses.append([int(x) for x in c])
    L = lambda j, a: n_vars + 3 * j + a
    pairs = []
    for j, c in enumerate(clauses):
        pairs += [(L(j, 0), L(j, 1)), (L(j, 0), L(j, 2)), (L(j, 1), L(j, 2))]
        pairs += [(c[a], L(j, a)) for a in range(3)]
    true_vars = [i for i in range(n_vars) if assign[i]]
    false_vars = [i for i in range(n_vars) if not assign[i]]
    f_lits, a_lits, t_lits = [], [], []
    for j, c in enumerate(clauses):
        vals = [bool(assign[x]) for x in c]
        f = vals.index(False)
        t = vals.index(True)
        a = 3 - f - t
        f_lits.append(L(j, f))
        a_lits.append(L(j, a))
        t_lits.append(L(j, t))
    order = true_vars + f_lits + a_lits + t_lits + false_vars
    n = n_vars + 3 * n_clauses
    return (*_pack(n, pairs), order)


def fig2():
    """The Figure 2 graph and its printed C+- values, read from the golden
    fixture.  Returns (n, src, dst, [(order_vertices, cpm), ...], names)."""
    names, pairs, orders = None, [], []
    with open(os.path.join(GOLDEN, "fig2_worked_example.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            if tok[0] == "vertices":
                names = tok[1:]
            elif tok[0] == "edge":
                pairs.append((names.index(tok[1]), names.index(tok[2])))
            elif tok[0] == "order":
                i = tok.index("cpm")
                orders.append(([names.index(x) for x in tok[1:i]], int(tok[i + 1])))
    n, s, d = _pack(len(names), pairs)
    return n, s, d, orders, names


def order_to_rank(order):
    """Vertices listed first-to-last -> rank array (rank[u] = position)."""
    rank = np.zeros(len(order), np.uint32)
    for pos, u in enumerate(order):
        rank[u] = pos
    return rank


def ld_golden():
    out = []
    with open(os.path.join(GOLDEN, "ld_gadget.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                d, c = line.split()
                out.append((int(d), int(c)))
    return out


def brute_force_triangles(n, src, dst):
    """All {a<b<c} with the three edges present: O(n^3) enumeration."""
    adj = [set() for _ in range(n)]
    for a, b in zip(src.tolist(), dst.tolist()):
        if a != b:
            adj[a].add(b)
            adj[b].add(a)
    out = []
    for a in range(n):
        for b in range(a + 1, n):
            if b not in adj[a]:
                continue
            for c in range(b + 1, n):
                if c in adj[a] and c in adj[b]:
                    out.append((a, b, c))
    return np.asarray(out, dtype=np.uint32).reshape(-1, 3)


def trace_count(n, src, dst):
    """Triangle count as trace(A^3)/6 of the symmetric 0/1 adjacency matrix."""
    A = np.zeros((n, n), dtype=np.int64)
    for a, b in zip(src.tolist(), dst.tolist()):
        if a != b:
            A[a, b] = 1
            A[b, a] = 1
    return int(np.trace(A @ A @ A)) // 6


def simple_degrees(n, src, dst):
    """Degrees of the simple graph (loops and duplicates removed)."""
    pairs = {(min(a, b), max(a, b)) for a, b in zip(src.tolist(), dst.tolist()) if a != b}
    deg = np.zeros(n, np.int64)
    for a, b in pairs:
        deg[a] += 1
        deg[b] += 1
    return deg, pairs


def oriented_degrees(n, src, dst, rank):
    """(d+, d-) per vertex, from the edge set directly (for cost checks)."""
    _, pairs = simple_degrees(n, src, dst)
    dp = np.zeros(n, np.int64)
    dm = np.zeros(n, np.int64)
    for a, b in pairs:
        lo, hi = (a, b) if rank[a] < rank[b] else (b, a)
        dp[lo] += 1
        dm[hi] += 1
    return dp, dm
