"""DBHT clustering on a finished TMFG, and the ARI of a clustering (test infrastructure only).

What is computed (Section 2, Background, the DBHT paragraph; Section 5, Evaluation). The
bubble tree has one node per 4-clique ("bubble") of the TMFG and an edge between two bubbles
that share a separating triangle. Each edge points to the side (inside or outside the
triangle) whose vertices are more strongly connected to the triangle. Converging bubbles
have only incoming edges. Every vertex is assigned to a converging bubble (its group), then
inside its group to a bubble by shortest-path distances on the TMFG. Complete linkage on the
all-pairs shortest-path distances joins, in turn, the vertices of each bubble, the bubbles of
each group, and the groups, giving a dendrogram; it is cut into as many clusters as the
ground truth has, and scored by the adjusted Rand index.

The paper outlines DBHT but leaves its quantities open. Readings:
  D1 edge lengths: sqrt(2 (1 - W[i, j])) in float64 (the usual correlation distance;
     1 - W is taken as 0 if negative), on the 3n - 6 TMFG edges only. Shortest paths are
     Dijkstra's: a path's length is summed from the source outward, so the two directions of
     a pair can differ in the last bit; the distance of i and j is the one from the smaller
     id.
  D2 bubbles: the seed 4-clique is bubble 0; insertion k (k = 1..n-4) of vertex u into face
     (x, y, z) makes bubble k = {u, x, y, z}. The face belonged to the bubble that created it
     (the seed faces to bubble 0); that bubble is bubble k's parent, and (x, y, z) is their
     separating triangle. The three faces made by insertion k belong to bubble k.
  D3 edge direction: the child side is the vertices inserted by the child's subtree, the
     parent side every other vertex not on the triangle. A side's strength is the sum of
     W[i, j] over TMFG edges from a triangle vertex i to a vertex j of that side, in float64,
     i ascending, then j ascending. The edge points to the strictly stronger side; a tie
     points to the parent.
  D4 converging bubbles: no outgoing edge. A vertex's group is, among the converging
     bubbles reachable along directed edges from the bubbles that contain it, the one to which
     its TMFG edges are strongest (sum of W[v, w] over its edges to the bubble's other
     vertices, ascending w); ties go to the lowest bubble id.
  D5 a vertex's bubble: among the bubbles that contain it and reach its group, the one with
     the least sum of shortest-path distances from the vertex to the bubble's four vertices
     (ascending); ties go to the lowest bubble id.
  D6 complete linkage: the distance of two clusters is the largest distance between their
     members; the closest pair merges, ties to the lowest (smaller id, larger id); the vertices
     are clusters 0..n-1 and merge m makes cluster n + m. Level 1 joins each (group, bubble)
     cell, level 2 the cells of each group, level 3 the groups; inside a level the cells and
     groups are taken in ascending order of their bubble ids. The record is scipy's: rows of
     (smaller id, larger id, distance, size).
  D7 the cut into k clusters undoes the last k - 1 merges of that sequence; clusters are
     numbered by their smallest vertex.
  D8 ARI: the paper's formula, with every distinct ground-truth label (noise included) one
     class.

Pinned by: shortest paths against a plain Floyd-Warshall on small graphs; complete linkage
against scipy.cluster.hierarchy on tie-free inputs; the ARI against the textbook cases and
scikit-learn; the bubble tree's invariants (n - 3 bubbles, each a 4-clique of the TMFG, each
separating triangle shared by its two bubbles); and a hand-derived small case.
"""
from __future__ import annotations

import heapq
from typing import Dict, List, Sequence, Tuple

import numpy as np


# ---- D1: distances -------------------------------------------------------------------------
def edge_lengths(W: np.ndarray, edges: np.ndarray) -> np.ndarray:
    """D1 for each edge, float64."""
    w = np.asarray([float(W[a, b]) for a, b in np.asarray(edges).tolist()], dtype=np.float64)
    return np.sqrt(2.0 * np.maximum(1.0 - w, 0.0))


def adjacency(n: int, edges: np.ndarray) -> List[List[int]]:
    """Neighbour lists of the TMFG, ascending."""
    adj: List[set] = [set() for _ in range(n)]
    for a, b in np.asarray(edges).tolist():
        adj[a].add(b)
        adj[b].add(a)
    return [sorted(s) for s in adj]


def apsp(W: np.ndarray, edges: np.ndarray) -> np.ndarray:
    """All-pairs shortest paths on the TMFG (D1), one Dijkstra per source (scipy's)."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import dijkstra
    n = W.shape[0]
    e = np.asarray(edges)
    ln = edge_lengths(W, e)
    G = csr_matrix((np.concatenate([ln, ln]), (np.concatenate([e[:, 0], e[:, 1]]),
                                              np.concatenate([e[:, 1], e[:, 0]]))), shape=(n, n))
    return symmetric(dijkstra(G, directed=False))


def symmetric(D: np.ndarray) -> np.ndarray:
    """D1: the distance of i and j is the path sum from the smaller id."""
    U = np.triu(D, 1)
    return U + U.T


def apsp_plain(W: np.ndarray, edges: np.ndarray) -> np.ndarray:
    """The same by a plain heap Dijkstra per source (small n)."""
    n = W.shape[0]
    e = np.asarray(edges)
    ln = edge_lengths(W, e)
    nb: List[List[Tuple[int, float]]] = [[] for _ in range(n)]
    for (a, b), l in zip(e.tolist(), ln.tolist()):
        nb[a].append((b, l))
        nb[b].append((a, l))
    D = np.full((n, n), np.inf)
    for s in range(n):
        dist = D[s]
        dist[s] = 0.0
        h = [(0.0, s)]
        done = np.zeros(n, dtype=bool)
        while h:
            d, v = heapq.heappop(h)
            if done[v]:
                continue
            done[v] = True
            for w, l in nb[v]:
                nd = d + l
                if nd < dist[w]:
                    dist[w] = nd
                    heapq.heappush(h, (nd, w))
    return symmetric(D)


# ---- D2, D3: the bubble tree --------------------------------------------------------------
def bubble_tree(order: np.ndarray, steps: np.ndarray):
    """D2: bubbles (vertex 4-tuples, ascending), parent of each, separating triangles, and the
    bubble that inserted each vertex (the seed's vertices: bubble 0)."""
    order = np.asarray(order).tolist()
    steps = np.asarray(steps).reshape(-1, 4).tolist()
    bubbles = [tuple(sorted(order[:4]))]
    parent = [-1]
    tri = [None]
    owner = {f: 0 for f in range(4)}          # face id -> bubble that made it
    creator = {v: 0 for v in order[:4]}
    nfaces = 4
    for k, (f, x, y, z) in enumerate(steps, start=1):
        u = order[3 + k]
        bubbles.append(tuple(sorted((u, x, y, z))))
        parent.append(owner[f])
        tri.append((x, y, z))
        owner[f] = k
        owner[nfaces] = k
        owner[nfaces + 1] = k
        nfaces += 2
        creator[u] = k
    return bubbles, parent, tri, creator


def directions(W: np.ndarray, edges: np.ndarray, bubbles, parent, tri, creator) -> List[bool]:
    """D3: for each bubble k >= 1, True when the edge to its parent points to the child."""
    nb = len(bubbles)
    children: List[List[int]] = [[] for _ in range(nb)]
    for k in range(1, nb):
        children[parent[k]].append(k)
    tin, tout = [0] * nb, [0] * nb
    clock = 0
    stack = [(0, False)]
    while stack:
        k, leaving = stack.pop()
        if leaving:
            tout[k] = clock
            continue
        tin[k] = clock
        clock += 1
        stack.append((k, True))
        for c in reversed(children[k]):
            stack.append((c, False))
    adj = adjacency(W.shape[0], edges)
    to_child = [False] * nb
    for k in range(1, nb):
        t = tri[k]
        s_child = 0.0
        s_parent = 0.0
        for i in sorted(t):
            for j in adj[i]:
                if j in t:
                    continue
                b = creator[j]
                if tin[k] <= tin[b] < tout[k]:
                    s_child += float(W[i, j])
                else:
                    s_parent += float(W[i, j])
        to_child[k] = s_child > s_parent
    return to_child


def converging(bubbles, parent, to_child) -> Tuple[List[int], List[List[int]]]:
    """D4: the converging bubbles, and for each bubble the converging bubbles it reaches."""
    nb = len(bubbles)
    out: List[List[int]] = [[] for _ in range(nb)]
    for k in range(1, nb):
        if to_child[k]:
            out[parent[k]].append(k)
        else:
            out[k].append(parent[k])
    sinks = [k for k in range(nb) if not out[k]]
    reach: List[set] = [None] * nb
    # the directed tree has no cycle: resolve by depth-first search with memoisation
    for s in range(nb):
        if reach[s] is not None:
            continue
        stack = [s]
        while stack:
            k = stack[-1]
            pend = [y for y in out[k] if reach[y] is None]
            if pend:
                stack.extend(pend)
                continue
            stack.pop()
            if reach[k] is None:
                reach[k] = {k} if not out[k] else set().union(*(reach[y] for y in out[k]))
    return sinks, [sorted(r) for r in reach]


def assign(W: np.ndarray, D: np.ndarray, edges: np.ndarray, bubbles, reach) -> Tuple[np.ndarray, np.ndarray]:
    """D4 and D5: each vertex's group (a converging bubble id) and bubble."""
    n = W.shape[0]
    adjs = [set(a) for a in adjacency(n, edges)]
    homes: List[List[int]] = [[] for _ in range(n)]
    for k, b in enumerate(bubbles):
        for v in b:
            homes[v].append(k)
    group = np.empty(n, dtype=np.int64)
    bubble = np.empty(n, dtype=np.int64)
    for v in range(n):
        cands = sorted(set().union(*(reach[h] for h in homes[v])))
        best_c, best_s = -1, -np.inf
        for c in cands:
            s = 0.0
            for w in bubbles[c]:
                if w != v and w in adjs[v]:
                    s += float(W[v, w])
            if best_c < 0 or s > best_s:
                best_c, best_s = c, s
        group[v] = best_c
        best_b, best_d = -1, np.inf
        for h in sorted(homes[v]):
            if best_c not in reach[h]:
                continue
            d = 0.0
            for w in bubbles[h]:
                d += float(D[v, w])
            if best_b < 0 or d < best_d:
                best_b, best_d = h, d
        bubble[v] = best_b
    return group, bubble


# ---- D6, D7: complete linkage --------------------------------------------------------------
def complete_linkage(Dc: np.ndarray, ids: Sequence[int], next_id: int, sizes: Sequence[int]):
    """D6 over m clusters with ids `ids` and cluster distances Dc (m x m). Returns the merge
    rows, the next free id and the id of the last cluster."""
    m = len(ids)
    Dc = np.array(Dc, dtype=np.float64)
    ids = np.asarray(ids, dtype=np.int64).copy()
    sizes = np.asarray(sizes, dtype=np.int64).copy()
    alive = np.ones(m, dtype=bool)
    rows = []
    iu = np.triu_indices(m, 1)
    for _ in range(m - 1):
        ok = alive[iu[0]] & alive[iu[1]]
        a_all, b_all = iu[0][ok], iu[1][ok]
        d = Dc[a_all, b_all]
        dmin = d.min()
        hit = d == dmin
        a_h, b_h = a_all[hit], b_all[hit]
        lo = np.minimum(ids[a_h], ids[b_h])
        hi = np.maximum(ids[a_h], ids[b_h])
        j = np.lexsort((hi, lo))[0]                 # the lowest (smaller id, larger id)
        a, b = int(a_h[j]), int(b_h[j])
        rows.append((int(lo[j]), int(hi[j]), float(dmin), int(sizes[a] + sizes[b])))
        # the merged cluster takes slot a; complete linkage keeps the larger distance
        Dc[a, :] = np.maximum(Dc[a, :], Dc[b, :])
        Dc[:, a] = Dc[a, :]
        alive[b] = False
        ids[a] = next_id
        sizes[a] += sizes[b]
        next_id += 1
    top = int(ids[np.flatnonzero(alive)[0]]) if m else None
    return rows, next_id, top


def _block_max(D: np.ndarray, blocks: List[List[int]]) -> np.ndarray:
    """Largest distance between every two blocks of vertices (m x m, zero diagonal)."""
    m = len(blocks)
    allv = np.concatenate([np.asarray(b, dtype=np.int64) for b in blocks])
    starts = np.cumsum([0] + [len(b) for b in blocks[:-1]])
    out = np.zeros((m, m))
    for a in range(m):
        R = D[np.ix_(blocks[a], allv)]
        out[a] = np.maximum.reduceat(R.max(axis=0), starts)
    np.fill_diagonal(out, 0.0)
    return out


def dbht_linkage(D: np.ndarray, group: np.ndarray, bubble: np.ndarray) -> np.ndarray:
    """D6: the three-level dendrogram as an (n - 1) x 4 record."""
    n = D.shape[0]
    rows: List[tuple] = []
    next_id = n
    groups = sorted(set(group.tolist()))
    group_ids, group_members = [], []
    for g in groups:
        cells = sorted(set(bubble[group == g].tolist()))
        cell_ids, cell_members = [], []
        for c in cells:
            mem = sorted(np.flatnonzero((group == g) & (bubble == c)).tolist())
            Dc = D[np.ix_(mem, mem)]
            r, next_id, top = complete_linkage(Dc, mem, next_id, [1] * len(mem))
            rows += r
            cell_ids.append(top)
            cell_members.append(mem)
        Dc = _block_max(D, cell_members)
        r, next_id, top = complete_linkage(Dc, cell_ids, next_id, [len(x) for x in cell_members])
        rows += r
        group_ids.append(top)
        group_members.append(sorted(sum(cell_members, [])))
    Dc = _block_max(D, group_members)
    r, next_id, _ = complete_linkage(Dc, group_ids, next_id, [len(x) for x in group_members])
    rows += r
    return np.asarray(rows, dtype=np.float64).reshape(-1, 4)


def cut(Z: np.ndarray, n: int, k: int) -> np.ndarray:
    """D7: labels of the first n - k merges' clusters, numbered by their smallest vertex."""
    parent = list(range(2 * n))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    for m in range(max(n - k, 0)):
        a, b = int(Z[m, 0]), int(Z[m, 1])
        parent[find(a)] = n + m
        parent[find(b)] = n + m
    roots = [find(v) for v in range(n)]
    first = {}
    for v in range(n):
        first.setdefault(roots[v], len(first))
    return np.asarray([first[r] for r in roots], dtype=np.int64)


# ---- D8 -----------------------------------------------------------------------------------
def ari(truth: Sequence[int], pred: Sequence[int]) -> float:
    """D8: the adjusted Rand index as Section 5 writes it."""
    truth = np.asarray(truth)
    pred = np.asarray(pred)
    _, ti = np.unique(truth, return_inverse=True)
    _, pi = np.unique(pred, return_inverse=True)
    nij = np.zeros((ti.max() + 1, pi.max() + 1), dtype=np.int64)
    np.add.at(nij, (ti, pi), 1)
    c2 = lambda x: x * (x - 1) / 2.0
    s_ij = c2(nij).sum()
    s_i = c2(nij.sum(1)).sum()
    s_j = c2(nij.sum(0)).sum()
    n2 = c2(truth.shape[0])
    expected = s_i * s_j / n2
    top = 0.5 * (s_i + s_j) - expected
    return float((s_ij - expected) / top) if top != 0 else 1.0


def dbht(W: np.ndarray, res: Dict[str, np.ndarray], k: int) -> Dict[str, np.ndarray]:
    """The whole procedure on a TMFG result (order, edges, steps) of W."""
    W = np.asarray(W, dtype=np.float32)
    edges = np.asarray(res["edges"]).reshape(-1, 2)
    D = apsp(W, edges)
    bubbles, parent, tri, creator = bubble_tree(res["order"], res["steps"])
    to_child = directions(W, edges, bubbles, parent, tri, creator)
    sinks, reach = converging(bubbles, parent, to_child)
    group, bubble = assign(W, D, edges, bubbles, reach)
    Z = dbht_linkage(D, group, bubble)
    return {"group": group, "bubble": bubble, "linkage": Z, "labels": cut(Z, W.shape[0], k),
            "converging": np.asarray(sinks), "to_child": np.asarray(to_child), "parent": np.asarray(parent)}
