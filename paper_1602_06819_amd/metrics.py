"""Evaluation of an online graph against an exact one.

* recall@k: the fraction of exact edges present in the online graph,
  |E_online intersect E_exact| / (n k) -- the paper counts "correct edges"
  against an offline brute-force graph (Section 8.5.2).
* Q (Section 8.5.2): with n initial nodes and n_a added ones, the expected
  number of modified edges is e_m = n_a k + n k n_a / (n_a + n), the
  expected unmodified ones e_u = (n + n_a) k - e_m, and
  Q = (e_c - e_u) / e_m for e_c correct edges.
"""

from __future__ import annotations

import numpy as np


def correct_edges(ids: np.ndarray, exact_ids: np.ndarray) -> int:
    """Number of (u, v) edges of ``ids`` that are also in ``exact_ids``
    (rows are nodes; -1 entries are ignored)."""
    ids = np.asarray(ids, dtype=np.int64)
    ex = np.asarray(exact_ids, dtype=np.int64)
    n = ids.shape[0]
    big = np.int64(1) << 32
    rows = np.arange(n, dtype=np.int64)[:, None]
    a = (rows * big + ids)[ids >= 0]
    b = (rows * big + ex)[ex >= 0]
    return int(np.intersect1d(a, b, assume_unique=False).size)


def recall(ids: np.ndarray, exact_ids: np.ndarray) -> float:
    ex = np.asarray(exact_ids)
    total = int((ex >= 0).sum())
    return correct_edges(ids, ex) / max(total, 1)


def expected_modified_edges(n: int, n_a: int, k: int) -> float:
    return n_a * k + n * k * n_a / (n_a + n)


def expected_unmodified_edges(n: int, n_a: int, k: int) -> float:
    return (n + n_a) * k - expected_modified_edges(n, n_a, k)


def quality(e_c: int, n: int, n_a: int, k: int) -> float:
    e_m = expected_modified_edges(n, n_a, k)
    return (e_c - expected_unmodified_edges(n, n_a, k)) / e_m
