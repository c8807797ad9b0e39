"""Exact k-nn graph by brute force.

The paper's naive method computes every pairwise similarity and keeps, for
each node, the k most similar others (Section 2.1); its evaluation builds the
ground-truth graph the same way (Section 8.5.2).  Definition used here: the
list of u is the first min(k, n-1) entries of the pairs (d(u, v), v), v != u,
sorted lexicographically -- ties in distance are broken by the smaller id.

Two implementations:

* :func:`exact_graph_loops` -- nested Python loops; the definition written
  out, for tiny n.
* :func:`exact_graph` -- the same definition, with the distance matrix built
  in row chunks as ||x||^2 + ||y||^2 - 2 X Y^T in float64 (a library matmul).
  For uint8 points every term is an integer below 2^53, so the result is
  exact and is converted to int64.  For float32 points the matmul only
  selects a candidate superset; the candidates' distances are recomputed in
  the direct form sum (x - y)^2 in float64 before sorting, and a row whose
  superset cannot be proved complete falls back to a full direct row.
"""

from __future__ import annotations

import numpy as np
import torch

from .distance import dissim_many, sqdist, sqdist_many
from .graph import empty_lists

_EXTRA = 8   # superset margin beyond k


def exact_row(X: np.ndarray, u: int, k: int, n: int | None = None,
              q: np.ndarray | None = None, exclude: int | None = -2):
    """Exact list of one point against rows [0, n) of X, by the definition.

    By default the point is row u of X and u itself is excluded.  With ``q``
    given, distances are taken from q and ``exclude`` names the id to skip
    (None: skip nothing).
    """
    n = X.shape[0] if n is None else n
    if q is None:
        q = X[u]
        exclude = u if exclude == -2 else exclude
    elif exclude == -2:
        exclude = None
    d = sqdist_many(q, X[:n])
    order = np.lexsort((np.arange(n), d))          # by distance, then id
    out = []
    for v in order:
        if exclude is not None and int(v) == exclude:
            continue
        out.append((d[v].item(), int(v)))
        if len(out) == k:
            break
    return out


def exact_graph_loops(X: np.ndarray, k: int):
    """Brute force with explicit loops over every pair (tiny n only)."""
    n = X.shape[0]
    ids, dist = empty_lists(n, k, X.dtype)
    for u in range(n):
        pairs = []
        for v in range(n):
            if v != u:
                pairs.append((sqdist(X[u], X[v]), v))
        pairs.sort()
        for j, (d, v) in enumerate(pairs[:k]):
            ids[u, j] = v
            dist[u, j] = d
    return ids, dist


def _chunk_distances(Xf: np.ndarray, norms: np.ndarray, lo: int, hi: int) -> np.ndarray:
    D = Xf[lo:hi] @ Xf.T
    D *= -2.0
    D += norms[None, :]
    D += norms[lo:hi, None]
    return D


def exact_graph(X: np.ndarray, k: int, chunk: int = 512, threads: int | None = None):
    """Exact k-nn graph of all rows of X; returns (ids [n,k], dist [n,k])."""
    n = X.shape[0]
    ids, dist = empty_lists(n, k, X.dtype)
    kk = min(k, n - 1)
    if kk <= 0:
        return ids, dist
    if threads is not None:
        torch.set_num_threads(threads)
    Xf = X.astype(np.float64)
    norms = np.einsum("ij,ij->i", Xf, Xf)
    is_int = X.dtype == np.uint8
    max_norm = float(norms.max())
    m = min(n - 1, kk + _EXTRA)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        D = _chunk_distances(Xf, norms, lo, hi)
        rows = np.arange(hi - lo)
        D[rows, lo + rows] = np.inf            # exclude self
        vals, idx = torch.topk(torch.from_numpy(D), m, dim=1, largest=False, sorted=True)
        vals = vals.numpy()
        idx = idx.numpy().astype(np.int64)
        if is_int:
            # uint8 data: D holds exact integers.  Order the m candidates of
            # each row by (distance, id) through one int64 key per entry.
            key = (vals.astype(np.int64) << 31) | idx
            key.sort(axis=1)
            ok = np.full(hi - lo, m == n - 1) | (vals[:, m - 1] > vals[:, kk - 1])
            ids[lo:hi, :kk] = np.where(ok[:, None], key[:, :kk] & ((1 << 31) - 1), -1)
            dist[lo:hi, :kk] = np.where(ok[:, None], key[:, :kk] >> 31, dist[lo:hi, :kk])
            for r in np.nonzero(~ok)[0]:
                # candidate set not provably complete (ties at the k-th): full row
                for j, (d, v) in enumerate(exact_row(X, lo + int(r), kk)):
                    ids[lo + r, j] = v
                    dist[lo + r, j] = d
        else:
            for r in range(hi - lo):
                u = lo + r
                pairs = _float_row(X, u, kk, vals[r], idx[r], m, n, norms[u], max_norm)
                for j, (d, v) in enumerate(pairs):
                    ids[u, j] = v
                    dist[u, j] = d
    return ids, dist


def _float_row(X, u, kk, vals, idx, m, n, norm_u, max_norm):
    """Float rows: recompute the superset's distances directly and accept
    them only if no point outside the superset can be as close as the kk-th.

    A point outside the superset has a Gram-form distance >= vals[m-1]; the
    Gram form differs from the exact value by at most about
    (d + 3) * eps * (||x_u||^2 + ||x_v||^2 + 2 |x_u . x_v|), bounded here by
    4 (d + 3) eps (||x_u||^2 + max ||x||^2).  If vals[m-1] minus that bound
    still exceeds the kk-th direct distance, the superset is complete;
    otherwise the whole row is computed directly."""
    if m == n - 1:
        return exact_row(X, u, kk)
    cv = idx.astype(np.int64)
    cd = sqdist_many(X[u], X[cv])
    o = np.lexsort((cv, cd))[:kk]
    kth = cd[o[-1]]
    err = 4.0 * (X.shape[1] + 3) * np.finfo(np.float64).eps * (norm_u + max_norm)
    if vals[m - 1] - err > kth:
        return [(float(cd[j]), int(cv[j])) for j in o]
    return exact_row(X, u, kk)


class ExactRows:
    """Exact lists of single points against a fixed point set, one at a
    time, by the same definition as :func:`exact_graph` (used to check
    sampled rows of large graphs).  Distances come from the float64 Gram
    form; for uint8 points they are exact integers; float rows are
    recomputed in the direct form."""

    def __init__(self, X: np.ndarray, k: int):
        self.X = X
        self.k = k
        self.Xf = X.astype(np.float64)
        self.norms = np.einsum("ij,ij->i", self.Xf, self.Xf)
        self.is_int = X.dtype == np.uint8

    def row(self, q: np.ndarray, exclude: int | None = None):
        n = self.X.shape[0]
        qf = q.astype(np.float64)
        D = self.norms + float(qf @ qf) - 2.0 * (self.Xf @ qf)
        if exclude is not None:
            D[exclude] = np.inf
        kk = min(self.k, n - (1 if exclude is not None else 0))
        m = min(n - 1, kk + _EXTRA)
        if not self.is_int or m < kk + 1:
            return exact_row(self.X, 0, kk, q=q, exclude=exclude)
        D = np.rint(D)
        cand = np.argpartition(D, m)[: m + 1]      # the m + 1 smallest
        cd = D[cand]
        order = np.lexsort((cand, cd))
        cand, cd = cand[order], cd[order]
        # every point outside the candidate set is at least cd[-1] away; the
        # set is complete for the first kk iff nothing outside can tie them
        if not cd[-1] > cd[kk - 1]:
            return exact_row(self.X, 0, kk, q=q, exclude=exclude)
        return [(int(cd[j]), int(cand[j])) for j in range(kk)]


class GroupedExactRows:
    """Exact lists of single points against a fixed point set by branch and
    bound over a partition of the set, by the definition above (first k of
    (d(q, v), v) sorted lexicographically; d in the direct float64 form, or
    exact integers for uint8 points).

    ``groups`` is any partition of the rows (an int array of group labels);
    it only decides how fast a row is found, never which row: every group
    has a centre c (its float64 mean) and a radius r = max |x - c| over its
    members, so every member is at Euclidean distance at least |q - c| - r
    from q (triangle inequality).  Groups are brute-forced in increasing
    order of that bound, and the search stops only when the next bound,
    squared and shrunk by a rounding margin, is strictly above the current
    k-th distance: no point of the remaining groups can then be closer or
    tie it.
    """

    _MARGIN = 1e-9    # relative slack covering float64 rounding of the bound

    def __init__(self, X: np.ndarray, k: int, groups: np.ndarray):
        self.X = X
        self.k = k
        n = X.shape[0]
        groups = np.asarray(groups)
        if groups.shape != (n,):
            raise ValueError("groups must label every row")
        order = np.argsort(groups, kind="stable")
        labels, starts = np.unique(groups[order], return_index=True)
        ends = np.append(starts[1:], n)
        self.members = [order[s:e] for s, e in zip(starts, ends)]
        Xf = X.astype(np.float64)
        self.centres = np.stack([Xf[m].mean(axis=0) for m in self.members])
        self.radius = np.array([np.sqrt(sqdist_many(c, Xf[m]).max())
                                for c, m in zip(self.centres, self.members)])

    def row(self, q: np.ndarray, exclude: int | None = None):
        n = self.X.shape[0]
        kk = min(self.k, n - (1 if exclude is not None else 0))
        if kk <= 0:
            return []
        dc = np.sqrt(sqdist_many(q.astype(np.float64), self.centres))
        lb = np.maximum(dc - self.radius, 0.0)
        best_d = np.empty(0)
        best_v = np.empty(0, dtype=np.int64)
        for gi in np.argsort(lb, kind="stable"):
            if len(best_d) == kk:
                kth = best_d[-1]
                if lb[gi] * lb[gi] * (1.0 - self._MARGIN) > kth:
                    break
            m = self.members[gi]
            if exclude is not None:
                m = m[m != exclude]
            if len(m) == 0:
                continue
            d = sqdist_many(q, self.X[m])
            cd = np.concatenate([best_d, d])
            cv = np.concatenate([best_v, m.astype(np.int64)])
            o = np.lexsort((cv, cd))[:kk]                 # by distance, then id
            best_d, best_v = cd[o], cv[o]
        return [(best_d[j].item(), int(best_v[j])) for j in range(len(best_d))]


class LazyExactGraph:
    """The exact k-nn graph of a point set (Section 8.5.2's ground truth, the
    initial graph of the online method) whose lists are computed on first
    use and kept: it answers what the online insertion reads from a snapshot
    -- points, node count and the stored lists of the nodes it visits --
    without building every list.  Lists come from :class:`GroupedExactRows`
    (exact for any grouping)."""

    def __init__(self, X: np.ndarray, k: int, groups: np.ndarray):
        self.X = X
        self.k = k
        self._rows = GroupedExactRows(X, k, groups)
        self._cache: dict[int, list] = {}

    @property
    def n(self) -> int:
        return int(self.X.shape[0])

    def neighbour_pairs(self, u: int) -> list[tuple]:
        got = self._cache.get(u)
        if got is None:
            got = self._rows.row(self.X[u], exclude=u)
            self._cache[u] = got
        return list(got)

    def neighbours(self, u: int) -> list[int]:
        return [v for _, v in self.neighbour_pairs(u)]

    def cached(self) -> int:
        return len(self._cache)


def exact_graph_ip(X: np.ndarray, k: int):
    """The exact k-nn graph by inner-product similarity: each node's k
    others of largest inner product, i.e. the first k of (-(x_u . x_v), v),
    v != u, sorted lexicographically (brute force, float64 dissimilarities
    accumulated as in :func:`distance.dissim`)."""
    n = X.shape[0]
    kk = min(k, n - 1)
    ids = np.full((n, k), -1, dtype=np.int64)
    dist = np.full((n, k), np.inf, dtype=np.float64)
    for u in range(n):
        d = dissim_many(X[u], X, "ip")
        d[u] = np.inf
        o = np.lexsort((np.arange(n), d))[:kk]
        ids[u, :kk] = o
        dist[u, :kk] = d[o]
    return ids, dist
