"""Pins of the cosine dissimilarity: closed forms of 2 (1 - cos), scale
invariance of the exact graph, and equality with brute force on angles."""

import numpy as np

import oracle as O
from oracle import cosine as C


def test_closed_forms():
    x = np.array([3.0, 4.0, 0.0], dtype=np.float32)
    assert C.dissimilarity(x, 2.5 * x) == 0.0                        # same direction
    assert abs(C.dissimilarity(x, -x) - 4.0) < 1e-15                   # opposite
    assert abs(C.dissimilarity(x, np.array([0, 0, 7.0], np.float32)) - 2.0) < 1e-15  # orthogonal
    y = np.array([1.0, 0.0, 0.0], dtype=np.float32)
    # cos = 3/5 -> 2 (1 - 0.6) = 0.8
    assert abs(C.dissimilarity(x, y) - 0.8) < 1e-15


def test_matches_angle_formula_on_random_pairs():
    rng = np.random.default_rng(3)
    for _ in range(200):
        x, y = rng.standard_normal((2, 17)).astype(np.float32)
        cos = float(np.dot(x.astype(np.float64), y) / (np.linalg.norm(x.astype(np.float64)) *
                                                      np.linalg.norm(y.astype(np.float64))))
        assert abs(C.dissimilarity(x, y) - 2 * (1 - cos)) < 1e-12


def test_exact_graph_is_invariant_to_positive_row_scaling():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((300, 8)).astype(np.float32)
    scale = rng.uniform(0.1, 10.0, size=(300, 1)).astype(np.float32)
    a_ids, a_d = O.exact_graph(C.normalize(X), 6)
    b_ids, b_d = O.exact_graph(C.normalize(X * scale), 6)
    assert np.mean(a_ids == b_ids) > 0.999
    # the scaled rows are rounded to float32, which moves directions by ~1e-8
    assert np.allclose(a_d, b_d, rtol=1e-6, atol=1e-9)


def test_nearest_by_angle_brute_force():
    rng = np.random.default_rng(5)
    X = rng.standard_normal((120, 5)).astype(np.float32)
    ids, _ = O.exact_graph(C.normalize(X), 3)
    Xd = X.astype(np.float64)
    for u in range(0, 120, 7):
        ang = [(np.arccos(np.clip(np.dot(Xd[u], Xd[v]) / np.linalg.norm(Xd[u]) /
                                  np.linalg.norm(Xd[v]), -1, 1)), v) for v in range(120) if v != u]
        ang.sort()
        assert ids[u].tolist() == [v for _, v in ang[:3]]
