"""GNNS, the graph nearest-neighbour search iGNNS improves on (Section 2.2
describes it; Section 3 states the differences), as the comparison baseline
of Section 8.2.2.

Steps, with the readings used where the description is silent:

1. Restart.  A random node r is drawn -- from the same keyed permutation as
   iGNNS (without replacement, skipping evaluated nodes) -- and its
   similarity to the query is computed.  There is no expansion test: every
   restart is climbed from.
2. Hill climbing, steepest.  At the current node c, the similarity of q to
   every neighbour of c is computed (neighbours evaluated before are not
   evaluated again, as in iGNNS); the search moves to the most similar of
   the neighbours evaluated at this node -- smallest (distance, id) -- if
   it is strictly closer than c.  Otherwise c is a local maximum.
3. Stop after a fixed number R of restarts (each with its whole climb), or
   when the optional budget of evaluations is spent (immediately after the
   budget-th evaluation), or when the permutation is exhausted.
4. Result: the k best evaluated nodes by (distance, id), and the number of
   similarities computed.
"""

from __future__ import annotations

from .distance import sqdist
from .graph import OracleGraph
from .ignns import SearchResult
from .restart import RestartOrder


def gnns(g: OracleGraph, q, key: int, k: int, restarts: int, seed: int,
         budget: int | None = None, n: int | None = None, record: bool = False) -> SearchResult:
    n = g.n if n is None else n
    B = n if budget is None else min(budget, n)
    order = RestartOrder(n, seed, key)
    visited: set[int] = set()
    evaluated: list[tuple] = []
    seq: list[int] | None = [] if record else None
    evals = 0

    def evaluate(v: int):
        nonlocal evals
        d = sqdist(q, g.X[v])
        evals += 1
        visited.add(v)
        evaluated.append((d, v))
        if seq is not None:
            seq.append(v)
        return d

    def finish() -> SearchResult:
        evaluated.sort()
        return SearchResult(pairs=evaluated[:k], evals=evals, sequence=seq)

    for _ in range(restarts):
        if evals == B:
            return finish()
        r = order.next_unvisited(visited)
        if r is None:
            return finish()
        c, d_c = r, evaluate(r)
        while True:
            step = []
            for v in g.neighbours(c):
                if v in visited:
                    continue
                if evals == B:
                    return finish()
                step.append((evaluate(v), v))
            if not step:
                break
            d_b, b = min(step)
            if d_b < d_c:
                c, d_c = b, d_b
            else:
                break
    return finish()
