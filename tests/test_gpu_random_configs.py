"""Bit-exact parity of the integer path with the oracle over seeded random
configurations: dimension 1-256, list length 1-64, update depth 1-4, the
speedup and expansion factor, and a random mix of batch sizes (1 included).
Each configuration builds the exact graph, inserts its batches and answers a
few queries; ids, distances, similarity counts and query evaluation counts
must all equal the oracle's.  The configurations cover every row-size class
of the search kernel (1, 2 and 4 lanes per row, 1-4 chunks per lane) and the
three staged list lengths (16, 32 and 64 ids)."""

import sys

import numpy as np
import pytest

import oracle as O
from tests.helpers import ensure_library, to_oracle_lists, u8_points

pytestmark = pytest.mark.gpu

EXPANSIONS = [(6, 5), (3, 2), (2, 1), (5, 1)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def G():
    ensure_library()
    import torch
    if not torch.cuda.is_available():
        pytest.fail("a GPU test ran without a visible GPU")
    from paper_1602_06819_amd import graph
    return graph


def tensor(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def random_config(seed):
    r = np.random.default_rng(1000 + seed)
    dim = int(r.choice([1, 3, 16, 17, 33, 48, 64, 100, 128, 200, 256]))
    k = int(r.choice([1, 2, 7, 10, 16, 17, 31, 33, 50, 64]))
    n0 = int(r.integers(k + 1, 700))
    nb = int(r.integers(1, 4))
    batches = [int(r.choice([1, int(r.integers(1, 40)), int(r.integers(40, 160))]))
               for _ in range(nb)]
    depth = int(r.integers(1, 5 if k <= 10 else 3))
    speedup = int(r.choice([1, 2, 4, 9, 20]))
    e = EXPANSIONS[int(r.integers(0, len(EXPANSIONS)))]
    clusters = int(r.integers(1, 6))
    sigma = float(r.uniform(4.0, 30.0))
    return dict(dim=dim, k=k, n0=n0, batches=batches, depth=depth, speedup=speedup, e=e,
                clusters=clusters, sigma=sigma)


@pytest.mark.parametrize("seed", range(32))
def test_random_integer_configuration_bit_exact(G, seed):
    c = random_config(seed)
    say(f"random config {seed}: {c}")
    total = c["n0"] + sum(c["batches"])
    X = u8_points(2000 + seed, total, c["dim"], clusters=c["clusters"], sigma=c["sigma"])
    cfg = G.GraphConfig(dim=c["dim"], k=c["k"], capacity=total, max_batch=max(c["batches"]),
                        speedup=c["speedup"], expansion_num=c["e"][0], expansion_den=c["e"][1],
                        depth=c["depth"], seed=0xC0FFEE + seed)
    g = G.KnnGraph.build_exact(cfg, tensor(X[:c["n0"]]))
    og = O.OracleGraph(X[:c["n0"]].copy(), *O.exact_graph(X[:c["n0"]], c["k"]), c["k"])
    p = O.Params(k=c["k"], speedup=c["speedup"], e_num=c["e"][0], e_den=c["e"][1],
                 depth=c["depth"], seed=cfg.seed)
    ids, d = to_oracle_lists(*(t.cpu().numpy() for t in g.lists()))
    assert np.array_equal(ids, og.ids) and np.array_equal(d, og.dist)
    lo = c["n0"]
    for b in c["batches"]:
        first, sims = g.insert(tensor(X[lo:lo + b]))
        res = O.insert_batch(og, X[lo:lo + b], p)
        og = res.graph
        assert first == lo
        assert sims.cpu().numpy().tolist() == res.sims, f"batch at {lo}"
        ids, d = to_oracle_lists(*(t.cpu().numpy() for t in g.lists()))
        assert np.array_equal(ids, og.ids), f"ids after batch at {lo}"
        assert np.array_equal(d, og.dist), f"distances after batch at {lo}"
        lo += b
    Q = u8_points(3000 + seed, 12, c["dim"], clusters=c["clusters"], sigma=c["sigma"])
    qi, qd, qe = (t.cpu().numpy() for t in g.query(tensor(Q)))
    for j, r in enumerate(O.query(og, Q, p, first_seq=0)):
        assert qi[j, :len(r.pairs)].tolist() == [v for _, v in r.pairs], f"query {j}"
        assert qd[j, :len(r.pairs)].tolist() == [dd for dd, _ in r.pairs], f"query {j}"
        assert qe[j] == r.evals, f"query {j}"
