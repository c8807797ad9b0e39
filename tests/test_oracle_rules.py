"""Hand-built pins of three rules of the method whose outcome the other
oracle tests cannot see.

* Section 3, first improvement: a random restart r is discarded when its
  similarity to the query is below s_max / e.  A far restart drawn after a
  good one must be evaluated, counted and then *not* climbed from; the
  next draw is tested in turn.
* Section 3, second improvement: the climb moves to the first neighbour that
  *increases* the similarity.  A neighbour exactly as similar as the current
  node does not move the climb; the scan goes on to the next neighbour.
* Section 4: the update costs at most k^DEPTH similarities, because the
  distances of the search result (level 1) are already known.  At DEPTH = 2
  the update evaluates exactly the distinct level-2 nodes that are not in
  level 1.

Each graph is small enough that the expected evaluation sequence (or count)
is worked out by hand in the docstring and written literally in the test,
by node role.  Roles are mapped to ids through the restart permutation,
which has its own pins (tests/test_oracle_basics.py).
"""

import numpy as np

import oracle as O


def _permutation(n: int, seed: int, key: int) -> list[int]:
    order = O.RestartOrder(n, seed, key)
    out: list[int] = []
    while True:
        v = order.next_unvisited(set(out))
        if v is None:
            return out
        out.append(v)


def _graph(points: dict, lists: dict, ids: dict, k: int) -> O.OracleGraph:
    """Graph of the named points with the named lists (stored order as
    given; each list must be sorted by distance to its owner)."""
    n = len(points)
    dim = len(next(iter(points.values())))
    X = np.zeros((n, dim), dtype=np.uint8)
    for role, pt in points.items():
        X[ids[role]] = pt
    nbr = np.full((n, k), -1, dtype=np.int64)
    dist = np.full((n, k), O.INF_INT, dtype=np.int64)
    for role, lst in lists.items():
        u = ids[role]
        ds = [O.sqdist(X[u], X[ids[v]]) for v in lst]
        assert ds == sorted(ds), f"list of {role} is not in distance order"
        for j, v in enumerate(lst):
            nbr[u, j] = ids[v]
            dist[u, j] = ds[j]
    return O.OracleGraph(X, nbr, dist, k)


def test_far_restart_is_discarded_then_near_restart_is_climbed():
    """1-D points, q = 100, k = 1, e = 2, budget = n = 6 (speedup 1).

    role   point  d(q)  list
    A       102     4   [F]      first restart (always kept)
    F       140  1600   [W]
    Rfar    110   100   [W]
    Rnear   101     1   [T]
    T       100     0   [Rnear]
    W       130   900   [Rfar]

    The permutation draws A, Rfar, Rnear first.  By hand:
      A (restart, kept) -> scan [F]: F is farther, local maximum  (best 4)
      Rfar (restart): 1 * (1 + 100) > 2 * (1 + 4) -> discarded
      Rnear (restart): best becomes 1, 1 + 1 <= 2 * (1 + 1) -> kept
      scan [T]: 0 < 1, move to T; scan [Rnear]: visited -> local maximum
      W (restart, the only node left) -> budget of 6 reached.
    Sequence A F Rfar Rnear T W.  Climbing from Rfar instead would
    evaluate W right after Rfar.
    """
    roles = ["A", "Rfar", "Rnear", "F", "T", "W"]
    perm = _permutation(6, seed=7, key=11)
    ids = {r: perm[i] for i, r in enumerate(roles)}
    points = {"A": [102], "F": [140], "Rfar": [110], "Rnear": [101], "T": [100], "W": [130]}
    lists = {"A": ["F"], "F": ["W"], "Rfar": ["W"], "Rnear": ["T"], "T": ["Rnear"],
             "W": ["Rfar"]}
    g = _graph(points, lists, ids, k=1)
    p = O.Params(k=1, speedup=1, e_num=2, e_den=1, seed=7)
    res = O.ignns(g, np.array([100], dtype=np.uint8), key=11, p=p, record=True)
    want = ["A", "F", "Rfar", "Rnear", "T", "W"]
    assert res.sequence == [ids[r] for r in want]
    assert res.evals == 6
    assert res.pairs == [(0, ids["T"])]


def test_discarded_restart_still_counts_and_enters_the_result():
    """Same graph with k = 2 lists padded to one entry and a budget of 3
    (speedup 2): the search stops right after the discarded Rfar, whose
    distance 100 is the second best evaluated and so enters the result."""
    roles = ["A", "Rfar", "Rnear", "F", "T", "W"]
    perm = _permutation(6, seed=7, key=11)
    ids = {r: perm[i] for i, r in enumerate(roles)}
    points = {"A": [102], "F": [140], "Rfar": [110], "Rnear": [101], "T": [100], "W": [130]}
    lists = {"A": ["F"], "F": ["W"], "Rfar": ["W"], "Rnear": ["T"], "T": ["Rnear"],
             "W": ["Rfar"]}
    g = _graph(points, lists, ids, k=2)
    p = O.Params(k=2, speedup=2, e_num=2, e_den=1, seed=7)
    res = O.ignns(g, np.array([100], dtype=np.uint8), key=11, p=p, record=True)
    assert res.sequence == [ids["A"], ids["F"], ids["Rfar"]]
    assert res.pairs == [(4, ids["A"]), (100, ids["Rfar"])]


def test_a_tie_does_not_move_the_climb():
    """2-D points, q = (100, 100), k = 2, e = 5, budget = n = 6.

    role  point      d(q)  list (by distance to the owner)
    c     (105,100)   25   [t (10), v (36)]      first restart
    t     (104,103)   25   [c (10), u (85)]      tie with c
    v     ( 99,100)    1   [w (1), c (36)]
    w     (100,100)    0   [v (1), t (25)]
    u     (110,110)  200   [t (85), c (125)]
    z     (130,100)  900   [u (500), c (625)]

    By hand: c (kept) -> scan c's list: t is as close as c (25), no move;
    v is closer, move to v -> scan: w closer, move to w -> scan: v and t
    visited, local maximum -> the two remaining nodes are drawn in
    permutation order and both discarded (far beyond 5 * (1 + 0)).
    Sequence c t v w, then u and z in permutation order.  Moving on the
    tie would scan t's list next and evaluate u third.
    """
    perm = _permutation(6, seed=3, key=5)
    rest = [v for v in perm[1:]]
    ids = {"c": perm[0], "t": rest[0], "v": rest[1], "w": rest[2], "u": rest[3], "z": rest[4]}
    points = {"c": [105, 100], "t": [104, 103], "v": [99, 100], "w": [100, 100],
              "u": [110, 110], "z": [130, 100]}
    lists = {"c": ["t", "v"], "t": ["c", "u"], "v": ["w", "c"], "w": ["v", "t"],
             "u": ["t", "c"], "z": ["u", "c"]}
    g = _graph(points, lists, ids, k=2)
    p = O.Params(k=2, speedup=1, e_num=5, e_den=1, seed=3)
    res = O.ignns(g, np.array([100, 100], dtype=np.uint8), key=5, p=p, record=True)
    tail = [v for v in perm if v in (ids["u"], ids["z"])]
    assert res.sequence == [ids["c"], ids["t"], ids["v"], ids["w"]] + tail
    assert res.pairs == [(0, ids["w"]), (1, ids["v"])]


def _update_graph(lists_of_ab):
    """1-D snapshot for the update pins: y = 100 is inserted; a (101) and
    b (99) are its two nearest nodes, so an exhaustive search (speedup 1)
    returns R = [b?, a?] by (distance, id) -- both at distance 1.  The other
    nodes c..f sit at 120, 80, 140, 60; g at 200 is reached by nothing."""
    names = ["a", "b", "c", "d", "e", "f", "g"]
    pts = {"a": [101], "b": [99], "c": [120], "d": [80], "e": [140], "f": [60], "g": [200]}
    ids = {r: i for i, r in enumerate(names)}
    lists = {r: [] for r in names}
    lists.update(lists_of_ab)
    # lists of the other nodes: their two nearest by (distance, id)
    X = np.array([pts[r] for r in names], dtype=np.uint8)
    for r in names:
        if r in lists_of_ab:
            continue
        u = ids[r]
        cand = sorted((O.sqdist(X[u], X[v]), v) for v in range(len(names)) if v != u)
        lists[r] = [names[v] for _, v in cand[:2]]
    return _graph(pts, lists, ids, k=2), ids


def test_update_evaluates_exactly_the_new_level_two_nodes():
    """DEPTH = 2, k = 2, lists of a = [c, d] and b = [f, e] (sorted by the
    distance to their owners: a->c 361, a->d 441; b->f 1521, b->e 1681).
    Level 1 = {a, b}: distances known from the search, no evaluation.
    Level 2 = {c, d, e, f}: four evaluations = k^2 exactly.  Every node of
    both levels receives one proposal."""
    g, ids = _update_graph({"a": ["c", "d"], "b": ["f", "e"]})
    p = O.Params(k=2, speedup=1, depth=2, seed=1)
    y = np.array([[100]], dtype=np.uint8)
    res = O.insert_batch(g, y, p)
    assert res.update_evals == [4]
    assert res.sims == [g.n + 4]             # search evaluates all 7, no peers
    targets = sorted(u for u, _, _ in res.proposals)
    assert targets == sorted(ids[r] for r in "abcdef")


def test_update_skips_level_one_and_repeated_nodes():
    """Lists that overlap: a = [b, c], b = [a, c].  Level 2 = a's and b's
    lists = {b, c, a, c}: a and b are level-1 nodes (already processed) and
    c repeats, so exactly one evaluation (c).  Recomputing the level-1
    distances would count 3."""
    g, ids = _update_graph({"a": ["b", "c"], "b": ["a", "c"]})
    p = O.Params(k=2, speedup=1, depth=2, seed=1)
    res = O.insert_batch(g, np.array([[100]], dtype=np.uint8), p)
    assert res.update_evals == [1]
    assert sorted(u for u, _, _ in res.proposals) == sorted([ids["a"], ids["b"], ids["c"]])


def test_update_depth_three_counts_levels_two_and_three():
    """DEPTH = 3 on the disjoint-list graph: level 2 = {c, d, e, f} (4
    evaluations); level 3 = the lists of c, d, e, f, i.e. their two nearest
    nodes: c (120) -> [a, e], d (80) -> [b, f], e (140) -> [c, a],
    f (60) -> [d, b]; every one already processed, so no more evaluations:
    4 in total."""
    g, ids = _update_graph({"a": ["c", "d"], "b": ["f", "e"]})
    assert g.neighbours(ids["c"]) == [ids["a"], ids["e"]]
    assert g.neighbours(ids["f"]) == [ids["d"], ids["b"]]
    p = O.Params(k=2, speedup=1, depth=3, seed=1)
    res = O.insert_batch(g, np.array([[100]], dtype=np.uint8), p)
    assert res.update_evals == [4]
