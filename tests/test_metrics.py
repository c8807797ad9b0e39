"""Evaluation helpers: the quality metric Q of Section 8.5.2 against the
values its formula gives for the paper's own parameters, and recall."""

import json
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def M():
    # metrics has no dependency on the compiled library
    import importlib.util
    path = os.path.join(os.path.dirname(GOLDEN), "..", "paper_1602_06819_amd", "metrics.py")
    spec = importlib.util.spec_from_file_location("knng_metrics", os.path.abspath(path))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_quality_worked_values():
    m = M()
    cases = json.load(open(os.path.join(GOLDEN, "quality_metric.json")))["cases"]
    for c in cases:
        assert m.expected_modified_edges(c["n"], c["n_a"], c["k"]) == pytest.approx(c["e_m"])
        assert m.expected_unmodified_edges(c["n"], c["n_a"], c["k"]) == pytest.approx(c["e_u"])
        # a perfect graph has e_c = (n + n_a) k and therefore Q = 1
        assert m.quality((c["n"] + c["n_a"]) * c["k"], c["n"], c["n_a"], c["k"]) == pytest.approx(1)
        # keeping only the unmodified edges gives Q = 0
        assert m.quality(c["e_u"], c["n"], c["n_a"], c["k"]) == pytest.approx(0)


def test_recall_counts_common_edges():
    m = M()
    exact = np.array([[1, 2], [0, 2], [1, 0]])
    online = np.array([[2, 1], [0, -1], [2, 0]])
    # row 0: {1,2} both; row 1: {0}; row 2: {0}
    assert m.correct_edges(online, exact) == 4
    assert m.recall(online, exact) == pytest.approx(4 / 6)
