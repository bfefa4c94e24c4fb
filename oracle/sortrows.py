"""Per-vertex similarity order (test infrastructure only).

Algorithm 1 (and Algorithm 2, which shares its set-up) sorts, for every vertex v, the
pairs (S[v, u], u) by similarity, once, before any insertion. The paper does not say
whether v itself is in its list, nor how equal similarities are ordered.

Readings: v is left out (its list holds the other n - 1 vertices); the order is by
similarity descending, then vertex id ascending; -0.0 and +0.0 compare equal.

Pinned by numpy.argsort(-row, kind="stable") (an independent library routine) and by a
hand-sorted tiny row.
"""
from __future__ import annotations

import numpy as np


def sorted_row(W: np.ndarray, v: int) -> np.ndarray:
    """The ids u != v ordered by (W[v, u] descending, u ascending)."""
    row = np.asarray(W[v])
    n = row.shape[0]
    ids = np.concatenate([np.arange(v), np.arange(v + 1, n)]).astype(np.int64)
    # np.lexsort sorts by the last key first: primary key -W[v, u], secondary u.
    vals = row[ids].astype(np.float64)
    order = np.lexsort((ids, -vals))
    return ids[order]


def sorted_rows(W: np.ndarray) -> np.ndarray:
    """All rows: an (n, n - 1) int64 array whose row v is sorted_row(W, v)."""
    n = W.shape[0]
    return np.stack([sorted_row(W, v) for v in range(n)]) if n else np.zeros((0, 0), np.int64)
