"""Seeded tiny graph family (at most 16 nodes) for brute-force pins.

Input construction only: plain edge lists turned into symmetric CSR.
"""
from __future__ import annotations

import random

import numpy as np

from graphgen import Graph


def from_edges(n: int, edges, ew=None, nw=None, rng: random.Random | None = None, shuffle_rows=False) -> Graph:
    """Symmetric CSR from undirected edges {u, v} (u != v, no repeats)."""
    rows = [[] for _ in range(n)]
    for i, (u, v) in enumerate(edges):
        w = 1 if ew is None else ew[i]
        rows[u].append((v, w))
        rows[v].append((u, w))
    for r in rows:
        if shuffle_rows and rng is not None:
            rng.shuffle(r)
        else:
            r.sort()
    rp = np.zeros(n + 1, np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    col = np.array([v for r in rows for v, _ in r], np.int32)
    w = np.array([w for r in rows for _, w in r], np.int32)
    return Graph(rp, col, ew=None if ew is None else w,
                 nw=None if nw is None else np.asarray(nw, np.int64))


def path(n):
    return [(i, i + 1) for i in range(n - 1)]


def cycle(n):
    return path(n) + [(n - 1, 0)] if n > 2 else path(n)


def star(n, centre=0):
    return [(centre, i) for i in range(n) if i != centre]


def clique(ids):
    ids = list(ids)
    return [(ids[i], ids[j]) for i in range(len(ids)) for j in range(i + 1, len(ids))]


def kab(a, b):
    return [(i, a + j) for i in range(a) for j in range(b)]


def gnp(n, p, rng):
    return [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < p]


def family(seed: int = 7, count: int = 60):
    """Yield (name, Graph) over paths, cycles, stars, cliques, K_{a,b},
    G(n, p) and disjoint unions, unweighted and weighted, n <= 16."""
    rng = random.Random(seed)
    shapes = []
    for n in (1, 2, 3, 5, 8, 16):
        shapes.append((f"path{n}", n, path(n)))
        shapes.append((f"star{n}", n, star(n)))
    for n in (3, 4, 7, 16):
        shapes.append((f"cycle{n}", n, cycle(n)))
        shapes.append((f"clique{n}", n, clique(range(n))))
    for a, b in ((1, 3), (2, 2), (3, 5), (4, 4)):
        shapes.append((f"k{a}_{b}", a + b, kab(a, b)))
    i = 0
    while len(shapes) < count:
        n = rng.randint(2, 16)
        p = rng.choice((0.15, 0.3, 0.5, 0.8))
        shapes.append((f"gnp{i}", n, gnp(n, p, rng)))
        i += 1
    for name, n, edges in shapes:
        yield name, from_edges(n, edges)
        ew = [rng.randint(1, 5) for _ in edges]
        nw = [rng.randint(0, 4) for _ in range(n)]
        yield name + "_w", from_edges(n, edges, ew=ew, nw=nw, rng=rng, shuffle_rows=True)
