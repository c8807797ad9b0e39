"""Shared helpers of the test suite: small seeded data sets, conversion of
GPU lists to the oracle's conventions, and an exact graph whose lists are
computed on demand (for sampled checks of large graphs)."""

from __future__ import annotations

import os
import subprocess
import sys

import numpy as np

import oracle as O
from datagen import u8_mixture

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1602_06819_amd", "libknng.so")


def ensure_library() -> None:
    """Build libknng.so if it is not there (tests use what is built)."""
    if not os.path.exists(LIB):
        subprocess.run([sys.executable, "-m", "paper_1602_06819_amd.build"], cwd=ROOT,
                       check=True)


def u8_points(seed: int, n: int, dim: int, clusters: int = 5, sigma: float = 12.0) -> np.ndarray:
    return u8_mixture(seed, clusters, dim, sigma).sample(n, seed + 1000)


def to_oracle_lists(ids: np.ndarray, d: np.ndarray):
    """GPU list arrays (padding id -1, distance INT32_MAX) in the oracle's
    convention (int64, padding distance INT64_MAX)."""
    ids = np.asarray(ids, dtype=np.int64)
    d = np.asarray(d, dtype=np.int64)
    d = np.where(ids < 0, O.INF_INT, d)
    return ids, d


class LazyExactGraph(O.OracleGraph):
    """The exact k-nn graph of X, with each list computed when first read."""

    def __init__(self, X: np.ndarray, k: int):
        super().__init__(X, np.empty((0, k), np.int64), np.empty((0, k), np.int64), k)
        self._rows = O.ExactRows(X, k)
        self._cache: dict[int, list] = {}

    def neighbour_pairs(self, u: int) -> list:
        if u not in self._cache:
            self._cache[u] = self._rows.row(self.X[u], exclude=u)
        return self._cache[u]

    def neighbours(self, u: int) -> list:
        return [v for _, v in self.neighbour_pairs(u)]
