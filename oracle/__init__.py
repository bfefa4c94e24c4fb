"""CPU oracle for TMFG construction (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this
package. The library never calls it, and it shares no code with the GPU path: it is a
plain, slow, obviously correct restatement of what the method computes, written from
the paper (Raphael & Shun, "Faster Parallel Triangular Maximally Filtered Graphs and
Hierarchical Clustering", arXiv 2408.09399).

Modules
  pearson     -- float64 Pearson correlation of n series (Section 5, Datasets).
  sortrows    -- each vertex's other vertices ordered by similarity (Algorithm 1, the
                 per-vertex sort; Algorithm 2 repeats it).
  tmfg        -- the seed tetrahedron and the exact greedy TMFG (Section 2, Massara's
                 serial method: every step joins the face/vertex pair of largest gain),
                 as brute force over every pair, as a cached eager schedule and as a
                 lazy heap schedule (Section 4.2).
  invariants  -- structural checks on a finished TMFG.
  paper_rule  -- the paper's candidate-limited rule with its heap schedule (Algorithm 2), as
                 a heap and as batched recomputation with an ordered commit.
  corr_rule   -- the paper's correlation-based construction with a prefix size and eager
                 updates (Algorithm 1).

Every function states the passage it follows and, where the paper is silent, the reading
taken. Parity status of each function is listed in its docstring.
"""
from .pearson import pearson64, DegenerateSeries, NonFinite
from .sortrows import sorted_row, sorted_rows
from .tmfg import (seed_scores, seed_vertices, tmfg_exact, tmfg_lazy, tmfg_bruteforce,
                   face_best, SizeError)
from .invariants import check_tmfg
from .paper_rule import tmfg_paper, tmfg_paper_batched, check_paper_steps
from .corr_rule import tmfg_corr, tmfg_corr_lazyrows

__all__ = [
    "pearson64", "DegenerateSeries", "NonFinite", "sorted_row", "sorted_rows",
    "seed_scores", "seed_vertices", "tmfg_exact", "tmfg_lazy", "tmfg_bruteforce",
    "tmfg_paper", "tmfg_paper_batched", "check_paper_steps", "tmfg_corr", "tmfg_corr_lazyrows",
    "face_best", "SizeError", "check_tmfg",
]
