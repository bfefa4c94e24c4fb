"""The paper's candidate-limited TMFG (Algorithm 2, heap-tmfg) on the CPU (test
infrastructure only).

What is computed (Section 4.1 and 4.2, Algorithm 2). Every vertex has its other vertices
sorted by similarity once. MaxCorrs[v] is the uninserted vertex most similar to v (the first
uninserted entry of v's sorted row). The candidates of a face are the MaxCorrs of its
three corners (up to three distinct vertices), and the face's pair is the candidate of
largest gain. Pairs sit in a max-heap; the top pair is popped: if its vertex is still
uninserted it is inserted (the face is split, the three new faces get pairs and are
pushed), otherwise the face's pair is recomputed and pushed back. Because the candidate
set is limited, a recomputed pair can have a larger gain than before, so this lazy
schedule is part of the result (Section 4.2 says the two differ only rarely).

Readings (in addition to R1, R2, R4 and R5-R8 of oracle.tmfg, which apply unchanged):
  P1 MaxCorrs[v] is evaluated whenever it is used, as Algorithm 2 recomputes it right
     before every use: the first entry of sortrows.sorted_row(W, v) not yet inserted.
  P2 the pair of a face {a < b < c}: among the distinct MaxCorrs of a, b and c, the largest
     float32 gain ((W[a,u] + W[b,u]) + W[c,u]), ties to the lowest vertex id.
  P3 the heap order is (gain desc, face id asc), the total order R3 uses for faces; each
     face has exactly one pair in the heap at any time.

Two schedules compute the same result:
  tmfg_paper          the heap, one pop at a time, exactly as Algorithm 2 runs;
  tmfg_paper_batched  between two insertions, all stale pairs that rank above the best fresh
                      pair are recomputed at once and then committed in key order while each
                      one's old key still ranks above every pair made fresh so far; a stale
                      pair that would never have been popped keeps its old key. This is the
                      order in which the heap pops them, so the two agree; the GPU uses this
                      form.

Pinned by: a hand-derived golden case (tests/golden/paper_rule_n7.json) on which the rule
departs from the exact one; the structural invariants of oracle.invariants; the check that
every inserted vertex is the first uninserted entry of one of its face's corners' sorted
rows at the time of insertion (check_paper_steps); and the agreement of the two schedules
on hundreds of random and tie-heavy matrices.
"""
from __future__ import annotations

import heapq
from typing import Dict, List, Sequence, Tuple

import numpy as np

from .sortrows import sorted_row
from .tmfg import _check, _rec_gain, _result, _seed_record, _split, seed_vertices


class _Rows:
    """Sorted rows built on first use, with a cursor per vertex (MaxCorrs, P1)."""

    def __init__(self, W: np.ndarray):
        self.W = W
        self.rows: Dict[int, np.ndarray] = {}
        self.cur: Dict[int, int] = {}

    def maxcorr(self, v: int, inserted: np.ndarray) -> int:
        row = self.rows.get(v)
        if row is None:
            row = self.rows[v] = sorted_row(self.W, v)
            self.cur[v] = 0
        i = self.cur[v]
        while i < row.shape[0] and inserted[row[i]]:
            i += 1
        self.cur[v] = i              # every entry before i is inserted, and stays so
        return int(row[i]) if i < row.shape[0] else -1


def paper_pair(W: np.ndarray, face: Sequence[int], rows: _Rows, inserted: np.ndarray) -> Tuple[int, np.float32]:
    """P2: the best of the face corners' MaxCorrs, (-1, -inf) when none is left."""
    a, b, c = face
    best_u, best_g = -1, np.float32(-np.inf)
    for u in sorted({rows.maxcorr(x, inserted) for x in face} - {-1}):
        g = (W[a, u] + W[b, u]) + W[c, u]
        if best_u < 0 or g > best_g:          # strictly larger: ties keep the lower id
            best_u, best_g = u, g
    return best_u, best_g


def tmfg_paper(W: np.ndarray) -> Dict[str, np.ndarray]:
    """Algorithm 2: the lazy heap with the candidate-limited face rule."""
    W = _check(W)
    n = W.shape[0]
    seed = seed_vertices(W)
    inserted = np.zeros(n, dtype=bool)
    inserted[seed] = True
    edges, faces = _seed_record(W, seed)
    order = list(seed)
    rows = _Rows(W)
    heap: List[Tuple[float, int, int]] = []
    if n > 4:
        for f in range(4):
            u, g = paper_pair(W, faces[f], rows, inserted)
            heap.append((-float(g), f, u))
        heapq.heapify(heap)
    steps, gains = [], []
    while len(order) < n:
        neg_g, f, u = heapq.heappop(heap)
        if inserted[u]:
            u2, g2 = paper_pair(W, faces[f], rows, inserted)
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
                u2, g2 = paper_pair(W, faces[nf], rows, inserted)
                heapq.heappush(heap, (-float(g2), nf, u2))
    return _result(order, edges, steps, gains, faces)


def _key(g, f: int) -> Tuple[float, int]:
    """P3 as a sortable key: larger gain first, then lower face id (-0.0 equals +0.0)."""
    return (float(g) + 0.0, -f)


def tmfg_paper_batched(W: np.ndarray) -> Dict[str, np.ndarray]:
    """The same result by batched recomputation with an ordered commit (see module text).

    Pairs are kept in an array (no heap). Before each insertion: take every stale pair
    (vertex inserted) that ranks above the best fresh pair, recompute them all, then walk
    them in the order of their old keys and commit a recomputed pair only while its old
    key ranks above every fresh pair so far (the best fresh one and the commits before it);
    stop at the first that does not. Repeat until the top pair is fresh, then insert it.
    """
    W = _check(W)
    n = W.shape[0]
    seed = seed_vertices(W)
    inserted = np.zeros(n, dtype=bool)
    inserted[seed] = True
    edges, faces = _seed_record(W, seed)
    order = list(seed)
    rows = _Rows(W)
    pu: List[int] = []
    pg: List[np.float32] = []
    if n > 4:
        for f in range(4):
            u, g = paper_pair(W, faces[f], rows, inserted)
            pu.append(u)
            pg.append(g)
    steps, gains = [], []
    while len(order) < n:
        while True:
            keys = [_key(pg[f], f) for f in range(len(pu))]
            fresh = [f for f in range(len(pu)) if not inserted[pu[f]]]
            floor = max((keys[f] for f in fresh), default=(-np.inf, 0))
            stale = sorted((f for f in range(len(pu)) if inserted[pu[f]] and keys[f] > floor),
                           key=lambda f: keys[f], reverse=True)
            if not stale:
                break
            new = {f: paper_pair(W, faces[f], rows, inserted) for f in stale}
            best = floor
            for f in stale:
                if keys[f] <= best:
                    break
                pu[f], pg[f] = new[f]
                best = max(best, _key(pg[f], f))
        f = max(range(len(pu)), key=lambda q: _key(pg[q], q))
        u, g = pu[f], pg[f]
        inserted[u] = True
        order.append(u)
        x, y, z = _split(faces, f, u)
        edges += [(u, x), (u, y), (u, z)]
        steps.append((f, x, y, z))
        gains.append(_rec_gain(g))
        pu += [0, 0]
        pg += [np.float32(0), np.float32(0)]
        if len(order) < n:
            for nf in (f, len(faces) - 2, len(faces) - 1):
                pu[nf], pg[nf] = paper_pair(W, faces[nf], rows, inserted)
    return _result(order, edges, steps, gains, faces)


def check_paper_steps(W: np.ndarray, res: Dict[str, np.ndarray]) -> None:
    """Each inserted vertex is, when inserted, the first uninserted entry of the sorted row
    of at least one corner of its face (a vertex of the face's candidate set: P1, P2).
    Raise AssertionError otherwise."""
    n = W.shape[0]
    order = [int(v) for v in res["order"]]
    inserted = np.zeros(n, dtype=bool)
    inserted[order[:4]] = True
    for i, (f, x, y, z) in enumerate(np.asarray(res["steps"]).tolist()):
        u = order[4 + i]
        firsts = []
        for c in (x, y, z):
            row = sorted_row(W, c)
            firsts.append(int(row[np.flatnonzero(~inserted[row])[0]]))
        assert u in firsts, f"step {i}: vertex {u} is no corner's most similar uninserted vertex"
        inserted[u] = True
