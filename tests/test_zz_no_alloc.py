"""The entry point that allocates nothing (knng_search_partitioned_noalloc):
called through the C ABI, it returns exactly what knng_search_partitioned
returns with a caller-allocated scratch, on two calls in a row (the second
with fewer queries, over the static scratch the first one left behind), and
rejects a call whose scratch would not fit the static array before any
launch."""

import ctypes
import sys

import numpy as np
import pytest

from tests.helpers import ensure_library, u8_points

pytestmark = pytest.mark.gpu


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


def _call_both(G, g, q, keys, part, p):
    """(ids, d, evals) from knng_search_partitioned with its own scratch and
    from knng_search_partitioned_noalloc, both through the C ABI."""
    import torch
    from paper_1602_06819_amd import _lib
    m = q.shape[0]
    k = g.cfg.k
    ddt = torch.int32 if g.cfg.dtype == "u8" else torch.float32
    out = []
    for noalloc in (False, True):
        ids = torch.full((m, k), -7, dtype=torch.int32, device="cuda")
        d = torch.full((m, k), -7, dtype=ddt, device="cuda")
        ev = torch.full((m,), -7, dtype=torch.int32, device="cuda")
        stream = torch.cuda.current_stream().cuda_stream
        if noalloc:
            st = _lib.lib.knng_search_partitioned_noalloc(
                g._h, q.data_ptr(), m, keys.data_ptr(), part.data_ptr(), p, ids.data_ptr(),
                d.data_ptr(), ev.data_ptr(), stream)
        else:
            nbytes = _lib.lib.knng_search_partitioned_scratch_bytes(g._h, m, p)
            scratch = G._aligned_buffer(nbytes, q.device)
            st = _lib.lib.knng_search_partitioned(
                g._h, q.data_ptr(), m, keys.data_ptr(), part.data_ptr(), p, scratch.data_ptr(),
                nbytes, ids.data_ptr(), d.data_ptr(), ev.data_ptr(), stream)
        assert st == 0, _lib.last_error()
        torch.cuda.synchronize()
        out.append((ids.cpu().numpy(), d.cpu().numpy(), ev.cpu().numpy()))
    return out


@pytest.mark.parametrize("kind", ["u8", "f32"])
def test_noalloc_matches_scratch_entry_point(G, kind):
    import torch
    n, dim, k, p = 6000, 32, 10, 6
    if kind == "u8":
        X = u8_points(131, n + 700, dim, clusters=8, sigma=12.0)
        cfg = G.GraphConfig(dim=dim, k=k, capacity=n, max_batch=64, speedup=6)
    else:
        from datagen import float_mixture
        X = float_mixture(132, 8, dim).sample(n + 700, 1132).astype(np.float32)
        cfg = G.GraphConfig(dim=dim, k=k, capacity=n, max_batch=64, speedup=6, dtype="f32",
                            score="exact")
    g = G.KnnGraph.build_exact(cfg, tensor(X[:n]))
    part, _ = g.partition(p, iters=2, seed=9)
    torch.cuda.synchronize()
    for call, m in enumerate((700, 123)):
        say(f"noalloc partitioned search {kind}: call {call + 1}, m={m}, p={p}")
        q = tensor(X[n:n + m])
        keys = torch.arange(n, n + m, dtype=torch.int64, device="cuda")
        (ia, da, ea), (ib, db, eb) = _call_both(G, g, q, keys, part, p)
        assert (ia >= 0).all() and (ea > 0).all()
        assert np.array_equal(ia, ib)
        assert np.array_equal(da, db)
        assert np.array_equal(ea, eb)


def test_noalloc_rejects_oversized_scratch(G):
    import torch
    from paper_1602_06819_amd import _lib
    n, dim, k, p = 3000, 16, 40, 64
    X = u8_points(133, n, dim, clusters=4)
    cfg = G.GraphConfig(dim=dim, k=k, capacity=n, max_batch=64)
    g = G.KnnGraph.build_exact(cfg, tensor(X))
    part = torch.zeros(n, dtype=torch.int32, device="cuda")
    m = 4096                      # 4096 * 64 parts * 64 ids * 8 B = 128 MiB > 32 MiB
    q = tensor(np.repeat(X[:1], m, axis=0))
    keys = torch.arange(m, dtype=torch.int64, device="cuda")
    ids = torch.full((m, k), -7, dtype=torch.int32, device="cuda")
    d = torch.full((m, k), -7, dtype=torch.int32, device="cuda")
    say("noalloc partitioned search: oversized call")
    st = _lib.lib.knng_search_partitioned_noalloc(
        g._h, q.data_ptr(), m, keys.data_ptr(), part.data_ptr(), p, ids.data_ptr(),
        d.data_ptr(), None, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert st == _lib.KNNG_ECAPACITY
    assert "static scratch" in _lib.last_error()
    assert (ids.cpu().numpy() == -7).all()
