"""Small named graphs with closed-form triangle counts, built as edge lists."""
import itertools

import numpy as np


def edges(pairs, n):
    pairs = list(pairs)
    if not pairs:
        return n, np.zeros(0, np.int32), np.zeros(0, np.int32)
    a = np.array(pairs, np.int32)
    return n, a[:, 0].copy(), a[:, 1].copy()


def complete(n):
    return edges(itertools.combinations(range(n), 2), n)


def complete_bipartite(a, b):
    return edges(((i, a + j) for i in range(a) for j in range(b)), a + b)


def complete_tripartite(a, b, c):
    parts = [range(0, a), range(a, a + b), range(a + b, a + b + c)]
    pairs = [(x, y) for p, q in itertools.combinations(parts, 2) for x in p for y in q]
    return edges(pairs, a + b + c)


def cycle(n):
    return edges(((i, (i + 1) % n) for i in range(n)), n)


def wheel(n):
    """W_n: hub 0 plus a rim cycle on nodes 1..n-1."""
    rim = n - 1
    pairs = [(0, i) for i in range(1, n)] + [(1 + i, 1 + (i + 1) % rim) for i in range(rim)]
    return edges(pairs, n)


def friendship(k):
    pairs = []
    for t in range(k):
        a, b = 1 + 2 * t, 2 + 2 * t
        pairs += [(0, a), (0, b), (a, b)]
    return edges(pairs, 2 * k + 1)


def grid(r, c):
    pairs = []
    for i in range(r):
        for j in range(c):
            v = i * c + j
            if j + 1 < c:
                pairs.append((v, v + 1))
            if i + 1 < r:
                pairs.append((v, v + c))
    return edges(pairs, r * c)


def hypercube(d):
    n = 1 << d
    return edges(((v, v ^ (1 << b)) for v in range(n) for b in range(d) if v < v ^ (1 << b)), n)


def random_tree(n, rng):
    return edges(((i, int(rng.integers(0, i))) for i in range(1, n)), n)


def random_bipartite(a, b, p, rng):
    return edges(((i, a + j) for i in range(a) for j in range(b) if rng.random() < p), a + b)


def star(k):
    return edges(((0, i) for i in range(1, k + 1)), k + 1)


def disjoint_union(*graphs):
    srcs, dsts, base = [], [], 0
    for n, s, d in graphs:
        srcs.append(s + base)
        dsts.append(d + base)
        base += n
    return base, np.concatenate(srcs).astype(np.int32), np.concatenate(dsts).astype(np.int32)


def gnp(n, p, rng):
    iu = np.triu_indices(n, 1)
    keep = rng.random(iu[0].shape[0]) < p
    return n, iu[0][keep].astype(np.int32), iu[1][keep].astype(np.int32)


def brute_force(n, src, dst):
    """Every triple of the simple graph checked directly (the naive method of
    Section III-A); pure Python, tiny n only."""
    adj = [set() for _ in range(n)]
    for u, v in zip(src.tolist(), dst.tolist()):
        if u != v:
            adj[u].add(v)
            adj[v].add(u)
    T = 0
    Tv = np.zeros(n, np.int64)
    for a, b, c in itertools.combinations(range(n), 3):
        if b in adj[a] and c in adj[a] and c in adj[b]:
            T += 1
            Tv[a] += 1
            Tv[b] += 1
            Tv[c] += 1
    return T, Tv


def dense_cube(n, src, dst):
    """trace(A^3)/6 and diag(A^3)/2 in exact int64 (textbook identity)."""
    A = np.zeros((n, n), np.int64)
    keep = src != dst
    A[src[keep], dst[keep]] = 1
    A[dst[keep], src[keep]] = 1
    A3 = A @ A @ A
    return int(np.trace(A3)) // 6, np.diag(A3) // 2
