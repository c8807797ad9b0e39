"""Workload descriptions: data recipe, sizes and the method's tunables.

Each workload is an initial point set (whose exact k-nn graph is built by
brute force), followed by a stream of points inserted in fixed-size batches,
and optionally a stream of read-only k-nn queries drawn from the same
mixture.  The tunables are the paper's: the search ``speedup`` (budget
n / speedup similarities, Section 3), the expansion coefficient e > 1 given
as the integer ratio ``expansion_num / expansion_den`` (Section 3), and the
update ``depth`` (Algorithm 2).
"""

from __future__ import annotations

from dataclasses import dataclass, replace

import numpy as np

from .gmm import GaussianMixture, float_mixture, subspace_mixture, u8_mixture


@dataclass(frozen=True)
class Workload:
    name: str
    kind: str                  # "u8" or "f32"
    dim: int
    k: int
    n_initial: int
    n_insert: int
    batch: int
    n_query: int
    n_clusters: int
    # mixture recipe
    sigma: float = 0.0         # u8: common sigma
    lognormal_dim_scale: float | None = None
    subspace_rank: int | None = None   # components of this many dimensions
    subspace_noise: float = 0.05       # isotropic noise, relative to sigma
    # seeds (data)
    mixture_seed: int = 0
    stream_seed: int = 1
    query_seed: int = 2
    # method tunables
    speedup: int = 10
    expansion_num: int = 5
    expansion_den: int = 1
    depth: int = 2
    algo_seed: int = 0x5EED
    score: str = "exact"       # "exact" | "bf16" | "fp8"

    def mixture(self) -> GaussianMixture:
        if self.kind == "u8":
            return u8_mixture(self.mixture_seed, self.n_clusters, self.dim, self.sigma)
        if self.subspace_rank is not None:
            return subspace_mixture(self.mixture_seed, self.n_clusters, self.dim,
                                    self.subspace_rank, noise=self.subspace_noise)
        return float_mixture(self.mixture_seed, self.n_clusters, self.dim,
                             lognormal_dim_scale=self.lognormal_dim_scale)

    def points(self) -> np.ndarray:
        """Initial points followed by the inserted points, one stream."""
        return self.mixture().sample(self.n_initial + self.n_insert, self.stream_seed)

    def queries(self) -> np.ndarray:
        return self.mixture().sample(self.n_query, self.query_seed)

    def batches(self) -> list[tuple[int, int]]:
        """(first index, count) of each insert batch within ``points()``."""
        out = []
        lo = self.n_initial
        end = self.n_initial + self.n_insert
        while lo < end:
            hi = min(end, lo + self.batch)
            out.append((lo, hi - lo))
            lo = hi
        return out

    def scaled(self, **kw) -> "Workload":
        return replace(self, **kw)


WORKLOADS: dict[str, Workload] = {
    # The paper's synthetic data set is a Gaussian mixture in R^3 (Section
    # 8.1.1; its parameters are not given): 10 centres ~ N(0,1)^3, per-cluster
    # sigma ~ U[0.05, 0.3], float32, k = 10.  Used by the experiment harness
    # at the paper's sizes.
    "f32-d3-gmm": Workload(
        name="f32-d3-gmm", kind="f32", dim=3, k=10, n_initial=8000,
        n_insert=16000, batch=1, n_query=1000, n_clusters=10,
        mixture_seed=61, stream_seed=62, query_seed=63,
        speedup=4, expansion_num=5, expansion_den=1, depth=2, score="exact"),
    # 2,000 initial uint8 points, d=16, 10 clusters (centres U[40,215], sigma
    # 12), squared L2, k=10; then 200 inserts one at a time.
    "u8-d16-n2k-b1": Workload(
        name="u8-d16-n2k-b1", kind="u8", dim=16, k=10, n_initial=2000,
        n_insert=200, batch=1, n_query=0, n_clusters=10, sigma=12.0,
        mixture_seed=11, stream_seed=12, query_seed=13,
        speedup=8, expansion_num=5, expansion_den=1, depth=2),
    # 100,000 initial uint8 points, d=64, 100 clusters (sigma 10), k=10;
    # 10,000 inserts in batches of 256; 10,000 read-only queries.
    "u8-d64-n100k-b256": Workload(
        name="u8-d64-n100k-b256", kind="u8", dim=64, k=10, n_initial=100_000,
        n_insert=10_000, batch=256, n_query=10_000, n_clusters=100, sigma=10.0,
        mixture_seed=21, stream_seed=22, query_seed=23,
        speedup=12, expansion_num=5, expansion_den=1, depth=4),
    # 1,000,000 initial float32 points, d=128, 1,000 clusters (centres N(0,1),
    # sigma U[0.05,0.3]), k=20; 50,000 inserts in batches of 1,024; BF16 scoring.
    "f32-d128-n1m-b1024": Workload(
        name="f32-d128-n1m-b1024", kind="f32", dim=128, k=20, n_initial=1_000_000,
        n_insert=50_000, batch=1024, n_query=0, n_clusters=1000,
        mixture_seed=31, stream_seed=32, query_seed=33,
        speedup=5, expansion_num=3, expansion_den=2, depth=2, score="bf16"),
    # Serving: graph grows 1,000,000 -> 2,000,000, d=96 float32, 2,000
    # components, k=10.  Each component is a 3-dimensional Gaussian (the
    # paper's synthetic data is a Gaussian mixture in R^3) along random
    # orthonormal directions of R^96 (sigma ~ U[0.05, 0.3]), plus isotropic
    # noise of 0.05 sigma in all 96 coordinates; centres ~ N(0, 1)^96.
    "serve-f32-d96-1m-2m": Workload(
        name="serve-f32-d96-1m-2m", kind="f32", dim=96, k=10, n_initial=1_000_000,
        n_insert=1_000_000, batch=16384, n_query=0, n_clusters=2000,
        mixture_seed=41, stream_seed=42, query_seed=43, subspace_rank=3,
        speedup=22, expansion_num=5, expansion_den=4, depth=3, score="bf16"),
    # The same sizes with isotropic 96-dimensional components (sigma ~ U[0.05,
    # 0.3] in every coordinate): kept for the measurements that show why the
    # serving workload uses low-dimensional components.
    "serve-f32-d96-1m-2m-iso": Workload(
        name="serve-f32-d96-1m-2m-iso", kind="f32", dim=96, k=10, n_initial=1_000_000,
        n_insert=1_000_000, batch=16384, n_query=0, n_clusters=2000,
        mixture_seed=41, stream_seed=42, query_seed=43,
        speedup=10, expansion_num=3, expansion_den=2, depth=2, score="bf16"),
    # 500,000 initial float32 points, d=960, 500 clusters, heavy-tailed
    # per-dimension scales (log-normal, sigma 1), k=50; 20,000 inserts in
    # batches of 512; FP8 e4m3 scoring with per-vector scales.
    "f32-d960-n500k-b512-fp8": Workload(
        name="f32-d960-n500k-b512-fp8", kind="f32", dim=960, k=50, n_initial=500_000,
        n_insert=20_000, batch=512, n_query=0, n_clusters=500, lognormal_dim_scale=1.0,
        mixture_seed=51, stream_seed=52, query_seed=53,
        speedup=5, expansion_num=3, expansion_den=2, depth=2, score="fp8"),
}


def get_workload(name: str) -> Workload:
    return WORKLOADS[name]


def query_points(w: Workload, count: int | None = None) -> np.ndarray:
    n = w.n_query if count is None else count
    return w.mixture().sample(n, w.query_seed)


__all__ = ["Workload", "WORKLOADS", "get_workload", "query_points", "np"]
