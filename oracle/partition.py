"""Partitioned search on one device: balanced k-medoids partitioning
(Algorithm 4) and the search of every partition merged to the k best
(Algorithm 3), as test infrastructure for the GPU's partitioned search.

Readings, where the paper leaves points open:

* One compute node (c = 1): capacity = n * imbalance / p, imbalance given
  as a fraction num / den >= 1.
* Initial medoids: the first p distinct nodes of the keyed restart
  permutation with key 2^61 (the same generator as the search's restarts).
* Assign: nodes are taken in id order; node u joins the medoid m that
  maximizes similarity(u, m) * w(m) with similarity 1 / (1 + d) and
  w(m) = 1 - |C(m)| / capacity, |C(m)| the cluster's size at that moment.
  In exact arithmetic: m beats m' iff
      (N - |C(m)| P) (1 + d(u, m')) > (N - |C(m')| P) (1 + d(u, m)),
  N = n num, P = p den; ties go to the smaller medoid index.
* Update (Section 6: the distance between two nodes is the length of the
  shortest path in the graph between them, by Dijkstra): the graph is the
  k-nn graph taken as undirected -- u and v are joined if either list holds
  the other, with the stored distance of the pair as the edge's length --
  restricted to the cluster's members (a search within a part moves only
  through the part).  The new medoid of a cluster is the member u that
  minimizes (members it cannot reach, sum of the path lengths from u to
  the members it reaches, u): within a connected cluster, the member with
  the smallest sum of path lengths, ties to the smaller id.  Sums are taken
  over the members in increasing id order (exact integers for uint8
  points).  An empty cluster keeps its medoid.
* Iterations: a fixed number; each is an assign then an update; the
  partition is the last assignment.
* Search of a partition: iGNNS restricted to the partition's nodes (the
  induced subgraph), with the partition's own budget, and the query's key;
  the result is the k best of the p partial results by (distance, id).
"""

from __future__ import annotations

import heapq
from fractions import Fraction

import numpy as np

from .distance import sqdist
from .graph import OracleGraph, Params
from .ignns import SearchResult, ignns
from .restart import RestartOrder

MEDOID_KEY = 1 << 61


def initial_medoids(n: int, p: int, seed: int) -> list[int]:
    order = RestartOrder(n, seed, MEDOID_KEY)
    out: list[int] = []
    while len(out) < p:
        v = order.next_unvisited(set(out))
        if v is None:
            break
        out.append(v)
    return out


def _better(wa: int, da, wb: int, db) -> bool:
    """w_a / (1 + d_a) > w_b / (1 + d_b), exactly."""
    if isinstance(da, int) and isinstance(db, int):
        return wa * (1 + db) > wb * (1 + da)
    return Fraction(wa) * (1 + Fraction(db)) > Fraction(wb) * (1 + Fraction(da))


def assign(X: np.ndarray, medoids: list[int], imb_num: int, imb_den: int) -> np.ndarray:
    n, p = X.shape[0], len(medoids)
    N, P = n * imb_num, p * imb_den
    size = [0] * p
    part = np.empty(n, dtype=np.int64)
    for u in range(n):
        best = None
        for m in range(p):
            d = sqdist(X[u], X[medoids[m]])
            w = N - size[m] * P
            if best is None or _better(w, d, best[1], best[2]):
                best = (m, w, d)
        part[u] = best[0]
        size[best[0]] += 1
    return part


def undirected_edges(ids: np.ndarray, dist: np.ndarray) -> dict:
    """The k-nn graph as an undirected graph: {u: {v: length}}, u and v
    joined if either list holds the other, the length being the stored
    distance of the pair."""
    adj: dict[int, dict] = {}
    n, k = ids.shape
    for u in range(n):
        for j in range(k):
            v = int(ids[u, j])
            if v < 0:
                continue
            w = dist[u, j].item()
            adj.setdefault(u, {})[v] = w
            adj.setdefault(v, {})[u] = w
    return adj


def shortest_paths(adj: dict, source: int, allowed: set) -> dict:
    """Dijkstra from `source` through the nodes of `allowed`: {node: length
    of its shortest path} for every node it reaches."""
    done: dict[int, object] = {}
    heap = [(0, source)]
    while heap:
        d, u = heapq.heappop(heap)
        if u in done:
            continue
        done[u] = d
        for v, w in adj.get(u, {}).items():
            if v in allowed and v not in done:
                heapq.heappush(heap, (d + w, v))
    return done


def member_path_key(adj: dict, u: int, members: list) -> tuple:
    """(members u cannot reach, sum of its path lengths to the others in
    increasing id order, u) within the cluster `members` (sorted ids)."""
    D = shortest_paths(adj, u, set(members))
    tot = 0
    for v in members:
        if v in D:
            tot = tot + D[v]
    return (len(members) - len(D), tot, u)


def update(ids: np.ndarray, dist: np.ndarray, part: np.ndarray, medoids: list[int],
           adj: dict | None = None) -> list[int]:
    """New medoids by graph shortest paths within each cluster (Section 6)."""
    adj = undirected_edges(ids, dist) if adj is None else adj
    out = list(medoids)
    for m in range(len(medoids)):
        members = [int(u) for u in np.nonzero(part == m)[0]]
        if not members:
            continue
        out[m] = min(member_path_key(adj, u, members) for u in members)[2]
    return out


def balanced_kmedoids(X: np.ndarray, ids: np.ndarray, dist: np.ndarray, p: int, iters: int,
                      seed: int, imb_num: int = 1, imb_den: int = 1,
                      medoids: list[int] | None = None):
    """Algorithm 4 on the points X and their k-nn graph (ids, dist): returns
    (part [n], medoids [p])."""
    meds = initial_medoids(X.shape[0], p, seed) if medoids is None else list(medoids)
    adj = undirected_edges(ids, dist)
    part = None
    for _ in range(iters):
        part = assign(X, meds, imb_num, imb_den)
        meds = update(ids, dist, part, meds, adj)
    return part, meds


def partitioned_search(g: OracleGraph, part: np.ndarray, p: int, q, key: int,
                       params: Params) -> tuple[SearchResult, list[int]]:
    """Algorithm 3 on one device: every partition searched with iGNNS on its
    own nodes, the k best of the union kept.  Returns the merged result and
    the evaluations per partition."""
    pairs, evals = [], []
    for t in range(p):
        r = ignns(g, q, key, params, allowed=(part == t))
        pairs.extend(r.pairs)
        evals.append(r.evals)
    pairs.sort()
    return SearchResult(pairs=pairs[:params.k], evals=sum(evals), sequence=None), evals
