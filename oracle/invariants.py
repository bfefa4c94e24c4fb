"""Structural checks on a finished TMFG (test infrastructure only).

Facts fixed by the construction itself (Section 2 and Algorithms 1-2): the seed is a
4-clique with 6 edges and 4 triangular faces, and each insertion adds one vertex, three
edges and a net of two faces. A TMFG on n vertices therefore has 3n - 6 edges and 2n - 4
faces, is planar with every face a triangle (Euler: V - E + F = 2), every edge lies on
exactly two faces, and each inserted vertex is joined to exactly one face that was live
when it was inserted. The recorded gains must equal float32 ((W[x,u] + W[y,u]) + W[z,u])
for the recorded face (x < y < z).
"""
from __future__ import annotations

from collections import Counter
from typing import Dict

import numpy as np


def check_tmfg(W: np.ndarray, res: Dict[str, np.ndarray], planarity: bool = True) -> None:
    """Raise AssertionError on the first violated invariant."""
    n = W.shape[0]
    order = [int(v) for v in res["order"]]
    edges = [tuple(int(a) for a in e) for e in res["edges"]]
    steps = [tuple(int(a) for a in s) for s in res["steps"]]
    gains = np.asarray(res["step_gain"], dtype=np.float32)
    faces = [tuple(int(a) for a in f) for f in res["faces"]]

    assert sorted(order) == list(range(n)), "order must be a permutation of the vertices"
    assert len(edges) == 3 * n - 6, "a TMFG has 3n-6 edges"
    assert len(faces) == 2 * n - 4, "a TMFG has 2n-4 faces"
    assert len(steps) == n - 4 and gains.shape == (n - 4,)
    und = {frozenset(e) for e in edges}
    assert len(und) == len(edges) and all(len(e) == 2 for e in und), "edges distinct, no loops"
    assert n - len(edges) + len(faces) == 2, "Euler characteristic of a sphere"

    # Replay: rebuild faces and edges from the seed and the step records.
    v1, v2, v3, v4 = order[:4]
    assert edges[:6] == [(v1, v2), (v1, v3), (v1, v4), (v2, v3), (v2, v4), (v3, v4)]
    live = [tuple(sorted(t)) for t in ((v1, v2, v3), (v1, v2, v4), (v1, v3, v4), (v2, v3, v4))]
    seen = set(order[:4])
    for i, (f, x, y, z) in enumerate(steps):
        u = order[4 + i]
        assert u not in seen, "each vertex is inserted once"
        assert 0 <= f < len(live) and live[f] == (x, y, z), "step joins a live face"
        assert x < y < z
        assert edges[6 + 3 * i: 9 + 3 * i] == [(u, x), (u, y), (u, z)]
        g = (W[x, u] + W[y, u]) + W[z, u] + np.float32(0.0)    # -0.0 is recorded as +0.0
        assert np.float32(g).tobytes() == gains[i].tobytes(), "recorded gain matches W"
        live[f] = tuple(sorted((u, x, y)))
        live.append(tuple(sorted((u, y, z))))
        live.append(tuple(sorted((u, x, z))))
        seen.add(u)
    assert live == faces, "final faces equal the replayed faces"

    # Every face is a triangle of the edge set; every edge lies on exactly two faces.
    cnt: Counter = Counter()
    for (a, b, c) in faces:
        assert a < b < c
        for e in ((a, b), (a, c), (b, c)):
            assert frozenset(e) in und, "face sides are edges"
            cnt[frozenset(e)] += 1
    assert all(cnt[e] == 2 for e in und), "every edge borders exactly two faces"

    if planarity:
        import networkx as nx
        G = nx.Graph()
        G.add_nodes_from(range(n))
        G.add_edges_from(edges)
        ok, _ = nx.check_planarity(G)
        assert ok, "TMFG must be planar"
