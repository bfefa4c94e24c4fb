"""Exact greedy TMFG construction on the CPU (test infrastructure only).

What is computed (Section 2, "PMFG, TMFG, and DBHT and Sequential Methods"): four
vertices form the starting 4-clique with its 4 triangular faces; then, one vertex at a
time, an uninserted vertex is joined to the three corners of an existing face, the
face/vertex pair being the one whose three new edge weights have the largest sum (the
"gain"). Section 4.1 calls the same per-face rule "picking the vertex that would
maximize the edge sum". The seed is the four vertices with the largest total row sum
(Algorithm 1 and Algorithm 2, first comment). The edge list starts with the six seed
edges and grows by three edges per insertion; a split face is replaced by the three
faces through the new vertex (Algorithm 1 and Algorithm 2, the edge and face updates).

Readings where the paper is silent (each applies to every function in this module):
  R1 seed score: sum of W[v, u] over u != v (diagonal left out), accumulated in float64
     strictly in index order u = 0, 1, ..., n-1; rank by (score desc, id asc); v1..v4 in
     that rank order.
  R2 gain of face (a, b, c), a < b < c, and vertex u: float32((W[a,u] + W[b,u]) + W[c,u])
     with round-to-nearest float32 additions in exactly that order. Signed: no abs.
  R3 selection: the pair of largest gain; ties go to the lowest face id, then to the
     lowest vertex id.
  R4 face ids: the split face f with corners x < y < z and new vertex u keeps its id and
     becomes sorted(u, x, y); sorted(u, y, z) and sorted(u, x, z) get the next two ids.
  R5 n < 4 is an error; n = 4 yields the seed only.
  R6 the input must be finite.
  R7 the result record: order (seed then inserted vertices), edges (seed edges
     (v1,v2),(v1,v3),(v1,v4),(v2,v3),(v2,v4),(v3,v4), then (u,x),(u,y),(u,z) per step),
     steps (f, x, y, z) per step, step_gain per step, faces (final corner triples in
     face-id order).
  R8 signed zero: -0.0 and +0.0 compare equal everywhere (selection, ties), and a gain of
     zero is recorded as +0.0.

Three schedules compute the same result (the cached one and the heap one rest on the
fact that removing vertices from the candidate set never raises a face's best gain):
  tmfg_bruteforce  every step evaluates every (live face, uninserted vertex) pair;
  tmfg_exact       keeps each face's best pair and recomputes, after an insertion, the
                   three new faces and every face whose best vertex was just inserted
                   (the eager update of Algorithm 1 with a prefix of one);
  tmfg_lazy        keeps the best pairs in a max-heap and recomputes a pair only when it
                   is popped with an already inserted vertex (Section 4.2, Algorithm 2's
                   control flow, with the exact per-face rule).

Pinned by: hand-derived golden cases (n = 4, 5, 6), agreement of the three schedules on
hundreds of random and tie-heavy matrices, and the structural invariants in
invariants.py.
"""
from __future__ import annotations

import heapq
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from .pearson import NonFinite


class SizeError(ValueError):
    """Fewer than four vertices."""


def _check(W: np.ndarray) -> np.ndarray:
    W = np.asarray(W)
    if W.dtype != np.float32:
        raise TypeError("W must be float32 (the bytes the GPU consumes)")
    if W.ndim != 2 or W.shape[0] != W.shape[1]:
        raise ValueError("W must be square")
    if W.shape[0] < 4:
        raise SizeError("a TMFG needs at least 4 vertices")
    if not np.isfinite(W).all():
        raise NonFinite("W holds NaN or Inf")
    return W


def seed_scores(W: np.ndarray) -> np.ndarray:
    """R1: score[v] = sum over u != v of W[v, u], float64, added in index order of u.

    numpy's cumulative sum along a row is the running sum out[u] = out[u-1] + x[u], i.e.
    strictly sequential; its last element is the score. The diagonal term is replaced by
    +0.0, which leaves the value of every partial sum unchanged.
    """
    W = np.asarray(W)
    n = W.shape[0]
    out = np.empty(n, dtype=np.float64)
    blk = 256
    for r0 in range(0, n, blk):
        rows = W[r0:r0 + blk].astype(np.float64)
        r = np.arange(rows.shape[0])
        rows[r, r0 + r] = 0.0
        out[r0:r0 + blk] = np.cumsum(rows, axis=1)[:, -1]
    return out


def seed_vertices(W: np.ndarray) -> List[int]:
    """R1: the four vertices of largest score, ties to the lower id, in rank order."""
    s = seed_scores(W)
    order = np.lexsort((np.arange(s.shape[0]), -s))
    return [int(v) for v in order[:4]]


def _gains(W: np.ndarray, face: Sequence[int]) -> np.ndarray:
    """R2 for one face against every vertex: float32 ((W[a] + W[b]) + W[c])."""
    a, b, c = face
    return (W[a] + W[b]) + W[c]


def face_best(W: np.ndarray, face: Sequence[int], inserted: np.ndarray) -> Tuple[int, np.float32]:
    """Exact best vertex of a face: largest gain over uninserted u, lowest u on ties."""
    g = _gains(W, face)
    cand = np.flatnonzero(~inserted)
    if cand.size == 0:
        return -1, np.float32(-np.inf)
    k = int(np.argmax(g[cand]))           # first maximum -> lowest u among ties
    return int(cand[k]), g[cand[k]]


def _seed_record(W: np.ndarray, seed: List[int]):
    v1, v2, v3, v4 = seed
    edges = [(v1, v2), (v1, v3), (v1, v4), (v2, v3), (v2, v4), (v3, v4)]
    faces = [tuple(sorted(t)) for t in ((v1, v2, v3), (v1, v2, v4), (v1, v3, v4), (v2, v3, v4))]
    return edges, faces


def _split(faces: List[tuple], f: int, u: int):
    x, y, z = faces[f]
    faces[f] = tuple(sorted((u, x, y)))
    faces.append(tuple(sorted((u, y, z))))
    faces.append(tuple(sorted((u, x, z))))
    return x, y, z


def _rec_gain(g) -> np.float32:
    """R8: the recorded gain, with -0.0 written as +0.0 (adding +0.0 does exactly that)."""
    return np.float32(g) + np.float32(0.0)


def _result(order, edges, steps, gains, faces) -> Dict[str, np.ndarray]:
    return {
        "order": np.asarray(order, dtype=np.int32),
        "edges": np.asarray(edges, dtype=np.int32).reshape(-1, 2),
        "steps": np.asarray(steps, dtype=np.int32).reshape(-1, 4),
        "step_gain": np.asarray(gains, dtype=np.float32),
        "faces": np.asarray(faces, dtype=np.int32).reshape(-1, 3),
    }


def tmfg_exact(W: np.ndarray) -> Dict[str, np.ndarray]:
    """Cached eager schedule: per-face best pairs, recomputed when they can have changed."""
    W = _check(W)
    n = W.shape[0]
    seed = seed_vertices(W)
    inserted = np.zeros(n, dtype=bool)
    inserted[seed] = True
    edges, faces = _seed_record(W, seed)
    order = list(seed)
    best_u = np.full(2 * n - 4, -1, dtype=np.int64)
    best_g = np.full(2 * n - 4, -np.inf, dtype=np.float32)
    live = 4
    if n > 4:
        for f in range(4):
            best_u[f], best_g[f] = face_best(W, faces[f], inserted)
    steps, gains = [], []
    for _ in range(n - 4):
        g_live = best_g[:live]
        fstar = int(np.flatnonzero(g_live == g_live.max())[0])   # R3: lowest face id
        u = int(best_u[fstar])
        g = best_g[fstar]
        inserted[u] = True
        order.append(u)
        x, y, z = _split(faces, fstar, u)
        edges += [(u, x), (u, y), (u, z)]
        steps.append((fstar, x, y, z))
        gains.append(_rec_gain(g))
        live += 2
        if inserted.all():
            break
        stale = [int(f) for f in np.flatnonzero(best_u[:live - 2] == u) if f != fstar]
        for f in [fstar, live - 2, live - 1] + stale:
            best_u[f], best_g[f] = face_best(W, faces[f], inserted)
    return _result(order, edges, steps, gains, faces)


def tmfg_lazy(W: np.ndarray, max_steps: Optional[int] = None) -> Dict[str, np.ndarray]:
    """Lazy heap schedule (Section 4.2): a stale pair is recomputed only when popped.

    max_steps stops the schedule after that many insertions (to time a prefix of it); the
    result then holds the steps taken and the faces at that point."""
    W = _check(W)
    n = W.shape[0]
    seed = seed_vertices(W)
    inserted = np.zeros(n, dtype=bool)
    inserted[seed] = True
    edges, faces = _seed_record(W, seed)
    order = list(seed)
    heap: List[Tuple[float, int, int]] = []
    if n > 4:
        for f in range(4):
            u, g = face_best(W, faces[f], inserted)
            heap.append((-float(g), f, u))
        heapq.heapify(heap)
    steps, gains = [], []
    while len(order) < n and (max_steps is None or len(steps) < max_steps):
        neg_g, f, u = heapq.heappop(heap)       # largest gain, then lowest face id
        if inserted[u]:
            u2, g2 = face_best(W, faces[f], inserted)
            heapq.heappush(heap, (-float(g2), f, u2))
            continue
        inserted[u] = True
        order.append(u)
        x, y, z = _split(faces, f, u)
        edges += [(u, x), (u, y), (u, z)]
        steps.append((f, x, y, z))
        gains.append(_rec_gain(-neg_g))
        if len(order) < n:
            for nf in (f, len(faces) - 2, len(faces) - 1):
                u2, g2 = face_best(W, faces[nf], inserted)
                heapq.heappush(heap, (-float(g2), nf, u2))
    return _result(order, edges, steps, gains, faces)


def _seed_by_loop(W: np.ndarray) -> List[int]:
    """R1 with plain Python floats (float64), one vertex and one term at a time."""
    n = W.shape[0]
    scores = []
    for v in range(n):
        acc = 0.0
        for u in range(n):
            if u != v:
                acc += float(W[v, u])
        scores.append(acc)
    ranked = sorted(range(n), key=lambda v: (-scores[v], v))
    return ranked[:4]


def tmfg_bruteforce(W: np.ndarray) -> Dict[str, np.ndarray]:
    """Every step evaluates every (live face, uninserted vertex) gain and takes the best.

    For small n only (cubic cost). The seed uses a plain Python loop, so no code is
    shared with the cached schedules beyond the gain formula R2.
    """
    W = _check(W)
    n = W.shape[0]
    seed = _seed_by_loop(W)
    inserted = np.zeros(n, dtype=bool)
    inserted[seed] = True
    edges, faces = _seed_record(W, seed)
    order = list(seed)
    steps, gains = [], []
    for _ in range(n - 4):
        cand = np.flatnonzero(~inserted)
        F = np.asarray(faces, dtype=np.int64)
        G = (W[F[:, 0]][:, cand] + W[F[:, 1]][:, cand]) + W[F[:, 2]][:, cand]
        k = int(np.argmax(G))        # row-major first maximum: lowest face, then lowest u
        f, j = divmod(k, cand.size)
        u = int(cand[j])
        inserted[u] = True
        order.append(u)
        x, y, z = _split(faces, f, u)
        edges += [(u, x), (u, y), (u, z)]
        steps.append((f, x, y, z))
        gains.append(_rec_gain(G[f, j]))
    return _result(order, edges, steps, gains, faces)
