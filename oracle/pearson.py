"""Float64 Pearson similarity of n series (test infrastructure only).

The paper builds its similarity matrix S as the Pearson correlation of every pair of
time series (Section 5, Datasets); S[i, j] is the weight of edge (i, j) (Section 2,
Definitions).

Readings where the paper is silent:
  * a series whose L values are all equal has no Pearson correlation (0/0); it is
    rejected as degenerate. "All equal" is decided exactly, on the float32 input;
  * non-finite input is rejected;
  * the diagonal is exactly 1.

Pinned by: numpy.corrcoef (an independent library routine), the textbook formula
evaluated with Python floats on tiny inputs, the closed form r = +-1 for L = 2,
invariance under x -> a*x + b with a > 0, and symmetry.
"""
from __future__ import annotations

import numpy as np


class DegenerateSeries(ValueError):
    """A series with zero variance: its Pearson correlation is undefined."""


class NonFinite(ValueError):
    """The input holds NaN or infinity."""


def pearson64(X: np.ndarray) -> np.ndarray:
    """R[i, j] = sum_t (x_it - m_i)(x_jt - m_j) / (||x_i - m_i|| ||x_j - m_j||), in float64."""
    X = np.asarray(X)
    if X.ndim != 2 or X.shape[1] < 2:
        raise ValueError("X must be (n, L) with L >= 2")
    if not np.isfinite(X).all():
        raise NonFinite("series contain NaN or Inf")
    if (X.max(axis=1) == X.min(axis=1)).any():
        raise DegenerateSeries("a series has all values equal")
    x = X.astype(np.float64)
    c = x - x.mean(axis=1, keepdims=True)
    s = np.sqrt((c * c).sum(axis=1))
    z = c / s[:, None]
    R = z @ z.T
    np.fill_diagonal(R, 1.0)
    return R
