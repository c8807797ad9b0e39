"""Online insertion (Algorithms 1 and 2) and read-only queries.

Algorithm 1 adds one node in two steps: search its k nearest neighbours with
iGNNS on the existing graph, then Update.  Algorithm 2 (Update) starts from
the found neighbours and explores neighbours of neighbours level by level up
to DEPTH; for every node it reaches it computes the similarity to the new
node and, "if needed", adds the new node to that node's list.

Batch semantics (not in the paper, which adds one node at a time).  A batch
of b points y_0 .. y_{b-1} receives ids n .. n+b-1 and is inserted against
the pre-batch graph G (the snapshot):

  (i)   R_i  = iGNNS(G, y_i, key = n + i), independently for each i.
  (ii)  F_i  = the k best of R_i together with every other batch point
        (d(y_i, y_j), n + j), j != i.  F_i becomes the list of node n + i.
  (iii) Update for each i, on the snapshot lists: level 1 is the ids of R_i;
        level l + 1 is the concatenation of the snapshot lists of the level-l
        nodes.  Each node is processed once (a per-i processed set): its
        distance to y_i is taken from R_i at level 1 and computed otherwise
        (an "update evaluation"); it receives the proposal (u, d, n + i).
        Only levels up to DEPTH are processed.  DEPTH = 0 is read as an
        exhaustive update (every snapshot node), used only in tests.
  (iv)  Merge: for each snapshot node u, its new list is the first k of its
        old list together with all proposals to u, sorted by (distance, id).
        A proposal id is larger than every snapshot id, so a new node loses
        ties against old neighbours.
  (v)   n <- n + b.

With b = 1 there are no peers and the result equals Algorithm 2 applied
immediately, because every node is processed at most once, its list only
changes when it is itself processed, and its neighbours are read before
that change.  :func:`insert_sequential_literal` transcribes Algorithms 1 and
2 in that immediate form so that tests can pin the two against each other.

Counting (Section 4's cost O(n/speedup + k^DEPTH)): the similarities spent
on inserting y_i are the search evaluations, the b - 1 peer distances, and
the update evaluations of levels >= 2 (level-1 distances are reused from the
search; at DEPTH = 2 there are at most k^2 of them).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .distance import dissim
from .graph import OracleGraph, Params, empty_lists, write_list
from .ignns import ignns

QUERY_KEY_BASE = 1 << 62


@dataclass
class BatchResult:
    graph: OracleGraph          # the graph after the batch
    search: list                # SearchResult per batch point
    final_lists: list           # F_i per batch point
    proposals: list             # (u, d, src) in emission order
    update_evals: list          # per batch point
    sims: list                  # search evals + (b - 1) + update evals


def _update_proposals(g: OracleGraph, y, src: int, R_pairs: list, depth: int,
                      metric: str = "l2"):
    """Step (iii) for one batch point: returns (proposals, update evals)."""
    n = g.n
    props = []
    upd = 0
    known = {v: d for d, v in R_pairs}
    processed: set[int] = set()
    if depth == 0:
        for u in range(n):
            if u in known:
                d = known[u]
            else:
                d = dissim(y, g.X[u], metric)
                upd += 1
            props.append((u, d, src))
        return props, upd
    level = [v for _, v in R_pairs]
    for ell in range(1, depth + 1):
        nxt: list[int] = []
        for u in level:
            if u in processed:
                continue
            processed.add(u)
            if ell == 1:
                d = known[u]
            else:
                d = dissim(y, g.X[u], metric)
                upd += 1
            props.append((u, d, src))
            if ell < depth:
                nxt.extend(g.neighbours(u))
        level = nxt
    return props, upd


def point_search_and_proposals(g, Y: np.ndarray, i: int, p: Params, record: bool = False):
    """Steps (i) and (iii) for batch point i of Y on the snapshot g (key
    n + i): (search result, proposals, update evaluations).  The batch's
    points are independent in these steps."""
    r = ignns(g, Y[i], key=g.n + i, p=p, record=record)
    props, upd = _update_proposals(g, Y[i], g.n + i, r.pairs, p.depth, p.metric)
    return r, props, upd


def search_and_propose(g, Y: np.ndarray, p: Params, record: bool = False, run_points=None):
    """Steps (i)-(iii) of a batch on the snapshot g: returns (search results,
    final lists F_i, proposals in emission order, update evaluations, sims).
    Reads from g only its points, node count and stored lists, so g may be
    any snapshot that provides them (e.g. :class:`exact.LazyExactGraph`).
    The batch points are independent in steps (i) and (iii): ``run_points``
    (optional) maps a list of point indices to their
    :func:`point_search_and_proposals` results, in order -- e.g. over worker
    processes; by default they run one after another."""
    n = g.n
    b = Y.shape[0]
    k = p.k
    # (i) search on the snapshot, and (iii) update proposals against the
    # snapshot lists, per batch point
    if run_points is None:
        per_point = [point_search_and_proposals(g, Y, i, p, record) for i in range(b)]
    else:
        per_point = list(run_points(list(range(b))))
    search = [r for r, _, _ in per_point]
    # (ii) batch peers
    final_lists = []
    for i in range(b):
        cand = list(search[i].pairs)
        for j in range(b):
            if j != i:
                cand.append((dissim(Y[i], Y[j], p.metric), n + j))
        cand.sort()
        final_lists.append(cand[:k])
    proposals = []
    update_evals = []
    for _, props, upd in per_point:
        proposals.extend(props)
        update_evals.append(upd)
    sims = [search[i].evals + (b - 1) + update_evals[i] for i in range(b)]
    return search, final_lists, proposals, update_evals, sims


def merge_proposals(g, proposals: list, k: int) -> dict:
    """Step (iv) for the targets that received proposals: {u: the first k of
    u's stored list together with its proposals, by (distance, id)}."""
    by_target: dict[int, list] = {}
    for u, d, src in proposals:
        by_target.setdefault(u, []).append((d, src))
    return {u: sorted(g.neighbour_pairs(u) + props)[:k] for u, props in by_target.items()}


def insert_batch(g: OracleGraph, Y: np.ndarray, p: Params, record: bool = False,
                 run_points=None) -> BatchResult:
    """Insert the points Y (one batch) into g; g itself is not modified.
    ``run_points`` as in :func:`search_and_propose`."""
    n = g.n
    b = Y.shape[0]
    k = p.k
    search, final_lists, proposals, update_evals, sims = search_and_propose(g, Y, p, record,
                                                                            run_points)
    # (iv) merge
    merged = merge_proposals(g, proposals, k)
    ids_new, dist_new = empty_lists(n + b, k, g.X.dtype)
    ids_new[:n] = g.ids
    dist_new[:n] = g.dist
    for u, pairs in merged.items():
        ids_new[u, :] = -1
        dist_new[u, :] = _pad_value(dist_new)
        write_list(ids_new, dist_new, u, pairs)
    for i in range(b):
        write_list(ids_new, dist_new, n + i, final_lists[i])
    # (v)
    X_new = np.concatenate([g.X, Y], axis=0)
    return BatchResult(graph=OracleGraph(X_new, ids_new, dist_new, k), search=search,
                       final_lists=final_lists, proposals=proposals,
                       update_evals=update_evals, sims=sims)


def _pad_value(dist: np.ndarray):
    return np.iinfo(np.int64).max if dist.dtype == np.int64 else np.inf


def insert_stream(g: OracleGraph, Y: np.ndarray, batch: int, p: Params):
    """Insert Y in consecutive batches of ``batch`` points; returns the final
    graph and the per-point similarity counts."""
    sims = []
    for lo in range(0, Y.shape[0], batch):
        res = insert_batch(g, Y[lo:lo + batch], p)
        g = res.graph
        sims.extend(res.sims)
    return g, sims


def query(g: OracleGraph, Q: np.ndarray, p: Params, first_seq: int = 0, record: bool = False):
    """Read-only k-nn search of each row of Q on g (no mutation).  Query j
    uses the restart key 2^62 + first_seq + j."""
    return [ignns(g, Q[j], key=QUERY_KEY_BASE + first_seq + j, p=p, record=record)
            for j in range(Q.shape[0])]


def insert_sequential_literal(g: OracleGraph, y, p: Params) -> OracleGraph:
    """Algorithms 1 and 2 as written: search, then a queue walk that adds the
    new node to a list as soon as its similarity is computed.  Readings:
    a node is processed once (duplicates and the new node itself are never
    re-queued), and "if needed, add" means: insert by (distance, id) and keep
    the first k.  Level-1 distances are recomputed here, as Algorithm 2
    writes them (they equal the search's)."""
    n = g.n
    k = p.k
    res = ignns(g, y, key=n, p=p)
    ids = np.concatenate([g.ids, np.full((1, k), -1, dtype=np.int64)], axis=0)
    pad = _pad_value(g.dist)
    dist = np.concatenate([g.dist, np.full((1, k), pad, dtype=g.dist.dtype)], axis=0)
    X = np.concatenate([g.X, y[None, :]], axis=0)
    out = OracleGraph(X, ids, dist, k)
    processed: set[int] = set()
    if p.depth == 0:
        targets = list(range(n))
        for node in targets:
            _literal_add(out, node, dissim(y, g.X[node], p.metric), n)
    else:
        Q = [v for _, v in res.pairs]
        for _ in range(p.depth):
            Q_next: list[int] = []
            while Q:
                node = Q.pop(0)
                if node in processed or node == n:
                    continue
                processed.add(node)
                Q_next.extend(out.neighbours(node))
                d = dissim(y, g.X[node], p.metric)
                _literal_add(out, node, d, n)
            Q = Q_next
    write_list(out.ids, out.dist, n, res.pairs)
    return out


def _literal_add(g: OracleGraph, node: int, d, new_id: int) -> None:
    pairs = g.neighbour_pairs(node)
    pairs.append((d, new_id))
    pairs.sort()
    pairs = pairs[: g.k]
    g.ids[node, :] = -1
    g.dist[node, :] = _pad_value(g.dist)
    write_list(g.ids, g.dist, node, pairs)
