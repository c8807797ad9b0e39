"""Dissimilarities: squared Euclidean distance (the default), and the
negated inner product (the inner-product similarity, a measure that is not
a metric: Section 3 states the method for any similarity).

The paper compares its synthetic Gaussian-mixture points with the Euclidean
distance (Section 8.1.1); squaring preserves every ordering and keeps uint8
data in exact integer arithmetic.

* uint8 points: the exact integer sum of squared coordinate differences
  (Python / int64 arithmetic; at most d * 255^2).
* float32 points: the sum computed in float64 from the float32 inputs,
  accumulated left to right over the coordinates (one fixed order, so every
  oracle path gives bit-identical float64 values; the relative rounding error
  is below d * 2^-53).
"""

from __future__ import annotations

import numpy as np

INF_INT = np.iinfo(np.int64).max


def sqdist(a: np.ndarray, b: np.ndarray):
    """Squared L2 between two single points; int for uint8, float for float."""
    if a.dtype == np.uint8:
        diff = a.astype(np.int64) - b.astype(np.int64)
        return int(np.dot(diff, diff))
    diff = a.astype(np.float64) - b.astype(np.float64)
    return float(np.cumsum(diff * diff)[-1])


def sqdist_many(q: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Squared L2 from one point ``q`` to every row of ``X`` (direct form)."""
    if X.dtype == np.uint8:
        diff = X.astype(np.int64) - q.astype(np.int64)[None, :]
        return np.einsum("ij,ij->i", diff, diff)
    diff = X.astype(np.float64) - q.astype(np.float64)[None, :]
    return np.cumsum(diff * diff, axis=1)[:, -1]


def inf_of(dtype) -> object:
    """The 'absent' distance used to pad short neighbour lists."""
    return INF_INT if dtype == np.uint8 else float("inf")


def inner_product(a: np.ndarray, b: np.ndarray) -> float:
    """a . b in float64 from the inputs, accumulated left to right over the
    coordinates."""
    return float(np.cumsum(a.astype(np.float64) * b.astype(np.float64))[-1])


def dissim(a: np.ndarray, b: np.ndarray, metric: str = "l2"):
    """The dissimilarity the method ranks by (smaller = more similar):
    squared L2, or for metric "ip" the negated inner product -(a . b)."""
    if metric == "ip":
        return -inner_product(a, b)
    return sqdist(a, b)


def dissim_many(q: np.ndarray, X: np.ndarray, metric: str = "l2") -> np.ndarray:
    """dissim from one point to every row of X (same accumulation order)."""
    if metric == "ip":
        return -np.cumsum(X.astype(np.float64) * q.astype(np.float64)[None, :], axis=1)[:, -1]
    return sqdist_many(q, X)
