"""Brute-force checkers used to pin the oracle (pure Python / numpy, tiny inputs).

They share no code with the oracle or with the GPU library:
  triangles_brute        vertex-triple loop (the triangle set of Section 2)
  support_brute          sup(e) straight from Definition 1 on edge sets
  truss_by_peeling       Definition 2 by repeated deletion: for k = 2, 3, ...
                         delete every edge with fewer than k-2 triangles in the
                         current subgraph until none is left (the shape of
                         Algorithm 1, with supports recomputed from scratch)
  truss_literal          Definition 2 literally: T_k is the union of all edge
                         subsets in which every edge lies in >= k-2 triangles of
                         the subset (a union of such subsets is one, so the
                         largest one is their union); exhaustive for m <= 16
  kcore_numbers          core number by repeated min-degree deletion
  x_brute / psi_brute    Procedure 6 by its words: for each end vertex, try
                         every x and count the other incident edges with
                         support >= x
  clustering_brute       mean local clustering coefficient of an edge set
                         (pairs of neighbours that are adjacent, per vertex)
"""
from __future__ import annotations

import itertools

import numpy as np


def canon(edges):
    return [(min(u, v), max(u, v)) for u, v in edges]


def adjacency(n, edges):
    nb = [set() for _ in range(n)]
    for u, v in edges:
        nb[u].add(v)
        nb[v].add(u)
    return nb


def triangles_brute(n, edges):
    es = set(canon(edges))
    cnt = 0
    for a, b, c in itertools.combinations(range(n), 3):
        if (a, b) in es and (a, c) in es and (b, c) in es:
            cnt += 1
    return cnt


def support_brute(n, edges):
    nb = adjacency(n, edges)
    return np.array([len(nb[u] & nb[v]) for u, v in edges], dtype=np.int64)


def truss_by_peeling(n, edges):
    m = len(edges)
    phi = np.full(m, 2, dtype=np.int64)
    alive = set(range(m))
    k = 3
    while alive:
        while True:
            nb = [set() for _ in range(n)]
            for i in alive:
                u, v = edges[i]
                nb[u].add(v)
                nb[v].add(u)
            drop = [i for i in alive if len(nb[edges[i][0]] & nb[edges[i][1]]) < k - 2]
            if not drop:
                break
            alive.difference_update(drop)
        for i in alive:
            phi[i] = k
        k += 1
    return phi


def truss_literal(n, edges):
    m = len(edges)
    assert m <= 16, "exhaustive subset enumeration is for m <= 16"
    if m == 0:
        return np.zeros(0, dtype=np.int64)
    ce = canon(edges)
    index = {e: i for i, e in enumerate(ce)}
    # triangles as triples of edge indices
    tris = []
    for i, j in itertools.combinations(range(m), 2):
        a = set(ce[i]) | set(ce[j])
        if len(a) == 3:
            x, y, z = sorted(a)
            t = tuple(sorted((index.get((x, y), -1), index.get((x, z), -1), index.get((y, z), -1))))
            if t[0] >= 0 and t not in tris:
                tris.append(t)
    S = np.arange(1 << m, dtype=np.int64)
    member = [(S >> e) & 1 for e in range(m)]
    sup = [np.zeros(S.size, dtype=np.int64) for _ in range(m)]
    for a, b, c in tris:
        for e, f, g in ((a, b, c), (b, a, c), (c, a, b)):
            sup[e] += member[f] & member[g]
    big = np.int64(1 << 30)
    minsup = np.full(S.size, big)
    for e in range(m):
        minsup = np.minimum(minsup, np.where(member[e] == 1, sup[e], big))
    phi = np.zeros(m, dtype=np.int64)
    for e in range(m):
        phi[e] = (minsup[member[e] == 1]).max() + 2
    return phi


def kcore_numbers(n, edges):
    nb = adjacency(n, edges)
    deg = [len(x) for x in nb]
    core = [0] * n
    alive = set(range(n))
    k = 0
    while alive:
        v = min(alive, key=lambda x: deg[x])
        k = max(k, deg[v])
        core[v] = k
        alive.remove(v)
        for w in nb[v]:
            if w in alive:
                deg[w] -= 1
    return np.array(core, dtype=np.int64)


def random_graph(rng, n, p):
    edges = [(u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < p]
    return edges


def x_brute(n, edges, sup, i, w):
    """Largest x such that at least x edges incident to w, other than edge i,
    have support >= x (Procedure 6)."""
    others = [sup[j] for j, (a, b) in enumerate(edges) if j != i and (a == w or b == w)]
    best = 0
    for x in range(len(others) + 1):
        if sum(1 for s in others if s >= x) >= x:
            best = x
    return best


def psi_brute(n, edges, sup):
    """psi(e) = min{sup(e), x_u, x_v} + 2 for every edge (Procedure 6)."""
    return np.array([min(sup[i], x_brute(n, edges, sup, i, u), x_brute(n, edges, sup, i, v)) + 2
                     for i, (u, v) in enumerate(edges)], dtype=np.int64)


def clustering_brute(n, edges):
    """(vertices touching an edge, edges, mean over those vertices of
    adjacent-neighbour pairs / all neighbour pairs; 0 for degree < 2)."""
    nb = adjacency(n, edges)
    vs = [v for v in range(n) if nb[v]]
    total = 0.0
    for v in vs:
        d = len(nb[v])
        if d < 2:
            continue
        links = sum(1 for a, b in itertools.combinations(sorted(nb[v]), 2) if b in nb[a])
        total += links / (d * (d - 1) / 2)
    return len(vs), len(set(canon(edges))), (total / len(vs) if vs else 0.0)
