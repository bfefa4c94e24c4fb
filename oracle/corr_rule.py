"""The paper's correlation-based TMFG with a prefix size (Algorithm 1, corr-tmfg) on the CPU
(test infrastructure only).

What is computed (Section 4.1, Algorithm 1). Every vertex has its other vertices sorted by
similarity once. MaxCorrs[v] is the uninserted vertex most similar to v. Every face holds
one pair in the Gains array: the candidate of largest gain among the MaxCorrs of its three
corners. Each round takes the p pairs of largest gain, keeps for each vertex only its best
pair among them, removes the kept vertices from the uninserted set, and applies every kept
pair (three edges, the face split into three). Then, eagerly, every face whose pair vertex
was just inserted and every new face gets its pair again, from freshly computed MaxCorrs of
its corners. Unlike the heap schedule (oracle.paper_rule), no pair is ever left stale, and
p > 1 inserts several vertices per round.

Readings (in addition to R1, R2 and R4-R8 of oracle.tmfg, and P1 and P2 of
oracle.paper_rule, which apply unchanged):
  C1 the prefix: the p pairs of largest (gain, then lowest face id); fewer if fewer faces.
  C2 conflicts: of the pairs in the prefix that share a vertex, the first in that order is
     kept (the largest gain, ties to the lowest face id).
  C3 the kept pairs are applied in that order: their steps, edges and vertices are recorded
     in that order, and the k-th kept pair's split takes the next two face ids in turn.
  C4 the update set of a round is every face whose pair vertex is one of the round's
     inserted vertices (the conflict losers included) and every face the round created;
     their pairs are computed against the uninserted set after the whole round, as the
     algorithm removes the prefix's vertices before its update loop.
  C5 the prefix size is fixed for the whole build (1 <= p); p = 1 is the eager schedule
     of Algorithm 2's rule, which the paper says differs from the heap only rarely.

Two formulations compute the same result:
  tmfg_corr        Algorithm 1's arrays as written: MaxCorrs is stored for every vertex and
                   recomputed for the corners of the update set (V_update) only;
  tmfg_corr_lazyrows  MaxCorrs evaluated where it is used, from a cursor into each sorted
                   row (P1).

Pinned by: hand-derived golden cases (tests/golden/corr_rule_*.json) for a conflict inside a
prefix and for a round where the eager update departs from the heap schedule; the check that
every inserted vertex is the first uninserted entry of one of its face's corners' sorted rows
(oracle.check_paper_steps); the structural invariants; and the agreement of the two
formulations on random and tie-heavy matrices.
"""
from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np

from .paper_rule import _Rows, paper_pair
from .sortrows import sorted_row
from .tmfg import _check, _rec_gain, _result, _seed_record, _split, seed_vertices


def _key(g, f: int) -> Tuple[float, int]:
    """C1: (gain desc, face id asc) as a sortable key (-0.0 equals +0.0)."""
    return (float(g) + 0.0, -f)


def _first_uninserted(row: np.ndarray, inserted: np.ndarray) -> int:
    """argmax over uninserted u of S[v, u], ties to the lower id: the first such entry of v's
    sorted row (-1 when every vertex is inserted)."""
    free = np.flatnonzero(~inserted[row])
    return int(row[free[0]]) if free.size else -1


def _face_pair(W: np.ndarray, face, maxcorrs: np.ndarray) -> Tuple[int, np.float32]:
    """P2 from the stored MaxCorrs of the face's corners."""
    a, b, c = face
    best_u, best_g = -1, np.float32(-np.inf)
    for u in sorted({int(maxcorrs[x]) for x in face} - {-1}):
        g = (W[a, u] + W[b, u]) + W[c, u]
        if best_u < 0 or g > best_g:
            best_u, best_g = u, g
    return best_u, best_g


def _prefix(pu: List[int], pg: List[np.float32], p: int) -> List[int]:
    """C1 and C2: the kept faces of the round, in key order."""
    live = [f for f in range(len(pu)) if pu[f] >= 0]
    top = sorted(live, key=lambda f: _key(pg[f], f), reverse=True)[:p]
    kept, seen = [], set()
    for f in top:
        if pu[f] not in seen:
            seen.add(pu[f])
            kept.append(f)
    return kept


def _apply(faces, kept, pu, pg, inserted, order, edges, steps, gains) -> List[int]:
    """C3: apply the kept pairs in order; returns the ids of the faces they created."""
    for f in kept:
        inserted[pu[f]] = True                    # the prefix leaves the uninserted set first
    made = []
    for f in kept:
        u = pu[f]
        x, y, z = _split(faces, f, u)
        order.append(u)
        edges += [(u, x), (u, y), (u, z)]
        steps.append((f, x, y, z))
        gains.append(_rec_gain(pg[f]))
        made += [f, len(faces) - 2, len(faces) - 1]
    return made


def tmfg_corr(W: np.ndarray, p: int = 1) -> Dict[str, np.ndarray]:
    """Algorithm 1 with prefix size p, its arrays kept as written."""
    if p < 1:
        raise ValueError("the prefix size is at least 1")
    W = _check(W)
    n = W.shape[0]
    seed = seed_vertices(W)
    inserted = np.zeros(n, dtype=bool)
    inserted[seed] = True
    edges, faces = _seed_record(W, seed)
    order = list(seed)
    rows = [sorted_row(W, v) for v in range(n)]
    maxcorrs = np.array([_first_uninserted(rows[v], inserted) for v in range(n)], dtype=np.int64)
    pu: List[int] = []
    pg: List[np.float32] = []
    if n > 4:
        for f in range(4):
            u, g = _face_pair(W, faces[f], maxcorrs)
            pu.append(u)
            pg.append(g)
    steps, gains = [], []
    while len(order) < n:
        kept = _prefix(pu, pg, p)
        just = {pu[f] for f in kept}
        made = _apply(faces, kept, pu, pg, inserted, order, edges, steps, gains)
        pu += [-1] * (len(faces) - len(pu))
        pg += [np.float32(-np.inf)] * (len(faces) - len(pg))
        if len(order) == n:
            break
        update = sorted(set(made) | {f for f in range(len(faces)) if pu[f] in just})
        v_update = {x for f in update for x in faces[f]}
        for v in v_update:
            maxcorrs[v] = _first_uninserted(rows[v], inserted)
        for f in update:
            pu[f], pg[f] = _face_pair(W, faces[f], maxcorrs)
    return _result(order, edges, steps, gains, faces)


def tmfg_corr_lazyrows(W: np.ndarray, p: int = 1) -> Dict[str, np.ndarray]:
    """The same rounds with MaxCorrs evaluated where it is used (P1)."""
    if p < 1:
        raise ValueError("the prefix size is at least 1")
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
        kept = _prefix(pu, pg, p)
        just = {pu[f] for f in kept}
        made = _apply(faces, kept, pu, pg, inserted, order, edges, steps, gains)
        pu += [-1] * (len(faces) - len(pu))
        pg += [np.float32(-np.inf)] * (len(faces) - len(pg))
        if len(order) == n:
            break
        stale = np.flatnonzero(np.isin(np.asarray(pu), list(just)))
        for f in sorted(set(made) | set(int(q) for q in stale)):
            pu[f], pg[f] = paper_pair(W, faces[f], rows, inserted)
    return _result(order, edges, steps, gains, faces)
