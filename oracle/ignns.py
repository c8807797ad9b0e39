"""iGNNS: the improved graph-based nearest-neighbour search (Section 3).

Steps, in the paper's order, with the readings used where it is silent:

1. Budget.  The search stops after a given number of similarity
   computations, n / speedup (Section 3, last paragraph); see
   :func:`graph.budget` for the rounding.  Every evaluation counts,
   including evaluations of restart nodes that are then discarded.  The
   search stops immediately after the budget-th evaluation, even in the
   middle of scanning a list.
2. Random restart with expansion test.  A random node r is drawn (order:
   :mod:`restart`); its similarity to the query is computed; r is discarded
   and another one drawn when similarity(q, r) < s_max / e, where s_max is
   the best similarity found so far (Section 3, first improvement).
   Reading of "similarity" for a distance: s = 1 / (1 + d) with d the
   squared Euclidean distance, so r is discarded iff (1 + d_r) > e (1 + d_best),
   evaluated in integers as e_den (1 + d_r) > e_num (1 + d_best).  d_best
   already includes d_r, so the first restart (and any restart that improves
   on the best so far) is always kept.
3. Eager hill climbing.  From the current node c, the neighbours in c's
   list are evaluated one at a time, in stored (distance, id) order, and the
   search moves to the *first* one that is more similar to q than c
   (strictly closer: a tie does not move) (Section 3, second improvement).
   A node already evaluated is never evaluated again, never charged again and
   never moved to.  When a whole list gives no improvement, c is a local
   maximum and the search restarts (step 2).
4. The search keeps the set of the most similar points found (Section 3,
   first paragraph): the result is the k best evaluated nodes by
   (distance, id).

The function returns the result list, the number of similarities computed,
and optionally the ids in evaluation order (for parity checks).
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .distance import dissim
from .graph import OracleGraph, Params, budget
from .restart import RestartOrder


class _Excluding(set):
    """A visited set that also contains every node outside ``allowed``."""

    def __init__(self, base, allowed):
        super().__init__(base)
        self.allowed = allowed

    def __contains__(self, v):
        return (not self.allowed[v]) or set.__contains__(self, v)


@dataclass
class SearchResult:
    pairs: list            # [(distance, id)] sorted, length min(k, evals)
    evals: int             # similarities computed
    sequence: list | None  # ids in evaluation order (if requested)


def expansion_rejects(d_r, d_best, e_num: int, e_den: int, metric: str = "l2") -> bool:
    """True iff similarity(q, r) < s_max / e.  Squared L2: s = 1/(1+d).
    Inner product (unbounded, possibly negative): s = exp(q . r), so the
    ratio test becomes s_max - s_r > ln e on the inner products, i.e.
    d_r - d_best > ln(e_num / e_den) on the negated ones."""
    if metric == "ip":
        return d_r - d_best > math.log(e_num / e_den)
    return e_den * (1 + d_r) > e_num * (1 + d_best)


def ignns(g: OracleGraph, q, key: int, p: Params, n: int | None = None,
          record: bool = False, allowed=None) -> SearchResult:
    """Search the k nearest neighbours of point q among nodes [0, n) of g.

    ``n`` defaults to the whole graph; the adjacency lists used are g's
    lists of those nodes (the snapshot).  ``allowed`` (a boolean array over
    the nodes, or None) restricts the search to a subgraph: nodes outside it
    are never drawn, evaluated or counted, as if they were not in the graph,
    and the budget is that of the subgraph's size (the search of one
    partition in Algorithm 3).
    """
    n = g.n if n is None else n
    size = n if allowed is None else int(np.count_nonzero(allowed[:n]))
    B = budget(size, p.k, p.speedup)
    order = RestartOrder(n, p.seed, key)
    visited: set[int] = set()
    if allowed is not None:
        # nodes outside the subgraph behave as already visited: skipped by
        # the restart draw and by the climb, never evaluated
        visited = _Excluding(visited, allowed)
    evaluated: list[tuple] = []
    seq: list[int] | None = [] if record else None
    state = {"evals": 0, "best": None}

    def evaluate(v: int):
        d = dissim(q, g.X[v], p.metric)
        state["evals"] += 1
        visited.add(v)
        evaluated.append((d, v))
        if seq is not None:
            seq.append(v)
        if state["best"] is None or d < state["best"]:
            state["best"] = d
        return d

    def finish() -> SearchResult:
        evaluated.sort()
        return SearchResult(pairs=evaluated[: p.k], evals=state["evals"], sequence=seq)

    while True:
        # -- restart: draw until a node passes the expansion test ----------
        while True:
            if state["evals"] == B:
                return finish()
            r = order.next_unvisited(visited)
            if r is None:
                return finish()
            d_r = evaluate(r)
            if not expansion_rejects(d_r, state["best"], p.e_num, p.e_den, p.metric):
                break
        # -- eager climb from r ---------------------------------------------
        c, d_c = r, d_r
        while True:
            moved = False
            for v in g.neighbours(c):
                if v in visited:
                    continue
                if state["evals"] == B:
                    return finish()
                d_v = evaluate(v)
                if d_v < d_c:
                    c, d_c = v, d_v
                    moved = True
                    break
            if not moved:
                break
