"""The k-nn graph state and the method's parameters.

A k-nn graph keeps, for every node, an adjacency list of its k most similar
nodes (Section 1; Section 5 calls these adjacency lists).  Here each list is
stored sorted by the key (distance, id) ascending, so the first entry is the
nearest; lists of a graph with n <= k nodes hold n - 1 entries and are padded
with id -1 and an infinite distance.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .distance import inf_of


@dataclass(frozen=True)
class Params:
    """Tunables of the method.

    speedup   -- iGNNS stops after n / speedup similarities (Section 3);
                 1 means exhaustive.
    e_num/e_den -- expansion coefficient e = e_num / e_den > 1 (Section 3).
    depth     -- DEPTH of Algorithm 2; 0 is an exhaustive update used only
                 in tests (every snapshot node is considered).
    seed      -- seed of the restart permutations.
    metric    -- "l2": squared Euclidean distance; "ip": inner-product
                 similarity (float points), dissimilarity its negation.
    """

    k: int
    speedup: int = 10
    e_num: int = 5
    e_den: int = 1
    depth: int = 2
    seed: int = 0x5EED
    metric: str = "l2"

    def __post_init__(self):
        if self.k < 1:
            raise ValueError("k must be >= 1")
        if self.speedup < 1:
            raise ValueError("speedup must be >= 1")
        if not (self.e_den >= 1 and self.e_num > self.e_den):
            raise ValueError("expansion e = e_num/e_den must be > 1")
        if self.depth < 0:
            raise ValueError("depth must be >= 0")
        if self.metric not in ("l2", "ip"):
            raise ValueError("metric must be 'l2' or 'ip'")


def budget(n: int, k: int, speedup: int) -> int:
    """Similarities iGNNS may compute on a graph of n nodes.

    Section 3 gives the cost as n / speedup.  Reading: integer ceiling, at
    least k (so that a full result list can be formed), at most n.
    """
    b = -(-n // speedup)
    return min(n, max(k, b))


@dataclass
class OracleGraph:
    X: np.ndarray       # [n, d] uint8 or float32 points, row = node id
    ids: np.ndarray     # [n, k] int64 neighbour ids, -1 = absent
    dist: np.ndarray    # [n, k] int64 (uint8 data) or float64 distances
    k: int

    @property
    def n(self) -> int:
        return int(self.X.shape[0])

    def neighbours(self, u: int) -> list[int]:
        """Stored list of u, in stored (distance, id) order."""
        row = self.ids[u]
        return [int(v) for v in row if v >= 0]

    def neighbour_pairs(self, u: int) -> list[tuple]:
        out = []
        for v, d in zip(self.ids[u], self.dist[u]):
            if v >= 0:
                out.append((d.item(), int(v)))
        return out

    def copy(self) -> "OracleGraph":
        return OracleGraph(self.X.copy(), self.ids.copy(), self.dist.copy(), self.k)


def empty_lists(n: int, k: int, dtype) -> tuple[np.ndarray, np.ndarray]:
    ids = np.full((n, k), -1, dtype=np.int64)
    if dtype == np.uint8:
        d = np.full((n, k), inf_of(dtype), dtype=np.int64)
    else:
        d = np.full((n, k), np.inf, dtype=np.float64)
    return ids, d


def write_list(ids: np.ndarray, dist: np.ndarray, row: int, pairs: list[tuple]) -> None:
    """Store a (distance, id)-sorted list of at most k pairs into one row."""
    k = ids.shape[1]
    assert len(pairs) <= k
    for j, (d, v) in enumerate(pairs):
        ids[row, j] = v
        dist[row, j] = d
