"""Cosine dissimilarity (an "other similarity" for the float path; the
method applies to any similarity, Section 3).

For unit vectors x^ = x / |x| and y^ = y / |y|,
    |x^ - y^|^2 = 2 - 2 cos(x, y),
so the k nearest neighbours by cosine similarity are the k nearest by
squared Euclidean distance between the normalized points, and every part of
the method runs unchanged on normalized points.  The dissimilarity stored
for a pair is that squared distance, 2 (1 - cos), in [0, 4].  A zero vector
stays zero (its dissimilarity to any unit vector is 1).  Normalization here
is in float64 from the float32 inputs.
"""

from __future__ import annotations

import numpy as np


def normalize(X: np.ndarray) -> np.ndarray:
    """Rows scaled to unit length (float64); zero rows stay zero."""
    Xd = np.asarray(X, dtype=np.float64)
    n = np.sqrt(np.einsum("ij,ij->i", Xd, Xd))
    safe = np.where(n > 0, n, 1.0)
    return Xd / safe[:, None]


def dissimilarity(x: np.ndarray, y: np.ndarray) -> float:
    """2 (1 - cos(x, y)) as the squared distance of the normalized points."""
    a, b = normalize(np.stack([x, y]))
    diff = a - b
    return float(np.cumsum(diff * diff)[-1])
