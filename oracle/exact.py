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

from .distance import sqdist, sqdist_many
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
