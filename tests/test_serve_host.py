"""Host logic of the serving loop: request stream, admission, epoch plans."""

import math
from collections import deque

import numpy as np

from paper_1602_06819_amd.serve import (Admission, Request, log_uniform_sizes, make_requests,
                                        plan_epoch, stream_totals)


def test_log_uniform_sizes_range_and_mean():
    rng = np.random.default_rng(1)
    s = log_uniform_sizes(rng, 400_000, 4096)
    assert s.min() == 1 and s.max() <= 4096
    # E floor(exp(U)) with U ~ U[0, ln 4097]: (4097 - 1) / ln 4097 minus the
    # mean fractional part; computed exactly from the distribution of floor
    L = math.log(4097)
    mean = sum(j * (math.log(j + 1) - math.log(j)) / L for j in range(1, 4097))
    assert abs(s.mean() - mean) < 0.01 * mean
    assert abs(mean - 492) < 1.0
    q = log_uniform_sizes(rng, 400_000, 512)
    qmean = sum(j * (math.log(j + 1) - math.log(j)) / math.log(513) for j in range(1, 513))
    assert abs(q.mean() - qmean) < 0.01 * qmean and abs(qmean - 82) < 1.0


def test_requests_poisson_mix_and_offsets():
    reqs = make_requests(7, rate=200.0, count=20000)
    arr = np.array([r.arrival for r in reqs])
    assert np.all(np.diff(arr) >= 0)
    assert abs(np.mean(np.diff(arr)) - 1 / 200.0) < 0.03 / 200.0
    frac = np.mean([r.kind == "insert" for r in reqs])
    assert abs(frac - 0.75) < 0.015
    for kind in ("insert", "query"):
        off = 0
        for r in (r for r in reqs if r.kind == kind):
            assert r.offset == off
            off += r.size
    ins, q = stream_totals(reqs)
    assert ins == sum(r.size for r in reqs if r.kind == "insert") and q > 0


def test_admission_fifo_within_limits():
    reqs = [Request(0, "insert", 3000, 0.0, 0), Request(1, "query", 100, 0.1, 0),
            Request(2, "insert", 2000, 0.2, 3000), Request(3, "query", 50, 0.3, 100),
            Request(4, "insert", 500, 5.0, 5000)]
    adm = Admission(4096, 120)
    pending = deque(reqs)
    e1 = adm.take(pending, now=1.0)
    # request 2 does not fit (3000 + 2000 > 4096): it and everything after wait
    assert [r.rid for r in e1] == [0, 1]
    e2 = adm.take(pending, now=1.0)
    assert [r.rid for r in e2] == [2, 3]
    assert adm.take(pending, now=1.0) == []          # request 4 has not arrived
    assert [r.rid for r in adm.take(pending, now=6.0)] == [4]
    ep = plan_epoch(e2)
    assert (ep.ins_lo, ep.ins_hi, ep.q_lo, ep.q_hi) == (3000, 5000, 100, 150)


def test_admission_query_limit_blocks_head():
    reqs = [Request(0, "query", 100, 0.0, 0), Request(1, "query", 100, 0.0, 100),
            Request(2, "insert", 10, 0.0, 0)]
    adm = Admission(4096, 150)
    pending = deque(reqs)
    assert [r.rid for r in adm.take(pending, 0.0)] == [0]
    assert [r.rid for r in adm.take(pending, 0.0)] == [1, 2]


def test_requests_for_inserts_is_the_shortest_prefix():
    from paper_1602_06819_amd.serve import requests_for_inserts
    for rate in (10.0, 500.0):
        reqs = requests_for_inserts(3, rate, 20_000)
        ins = [r.size for r in reqs if r.kind == "insert"]
        assert sum(ins) >= 20_000 and sum(ins) - ins[-1] < 20_000
        assert reqs[-1].kind == "insert"
    # the stream's kinds and sizes do not depend on the rate
    a = requests_for_inserts(3, 10.0, 20_000)
    b = requests_for_inserts(3, 500.0, 20_000)
    assert [(r.kind, r.size) for r in a] == [(r.kind, r.size) for r in b]
