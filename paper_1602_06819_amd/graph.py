"""Python front end of the library: a k-nn graph resident in GPU memory.

PyTorch provides the device memory (storage, workspace, inputs, outputs)
and the stream; every call goes through the C ABI of include/knng.h.
"""

from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import check, knng_params

_DTYPES = {"u8": _lib.KNNG_U8, "f32": _lib.KNNG_F32}
_SCORES = {"exact": _lib.KNNG_SCORE_EXACT, "bf16": _lib.KNNG_SCORE_BF16,
           "fp8": _lib.KNNG_SCORE_FP8, "bf16m": _lib.KNNG_SCORE_BF16_MFMA}
_METRICS = {"l2": _lib.KNNG_METRIC_L2, "cosine": _lib.KNNG_METRIC_COSINE,
            "ip": _lib.KNNG_METRIC_INNER_PRODUCT}


@dataclass(frozen=True)
class GraphConfig:
    dim: int
    k: int
    capacity: int
    max_batch: int
    speedup: int = 10
    expansion_num: int = 5
    expansion_den: int = 1
    depth: int = 2
    seed: int = 0x5EED
    dtype: str = "u8"
    score: str = "exact"
    metric: str = "l2"

    def params(self) -> knng_params:
        return knng_params(dim=self.dim, k=self.k, dtype=_DTYPES[self.dtype],
                           score=_SCORES[self.score], capacity=self.capacity,
                           max_batch=self.max_batch, speedup=self.speedup,
                           expansion_num=self.expansion_num, expansion_den=self.expansion_den,
                           depth=self.depth, seed=self.seed, metric=_METRICS[self.metric])


def storage_bytes(cfg: GraphConfig) -> int:
    p = cfg.params()
    n = _lib.lib.knng_storage_bytes(ctypes.byref(p))
    if n == 0:
        raise _lib.KnngError(_lib.KNNG_EINVAL, _lib.last_error())
    return n


def workspace_bytes(cfg: GraphConfig) -> int:
    p = cfg.params()
    n = _lib.lib.knng_workspace_bytes(ctypes.byref(p))
    if n == 0:
        raise _lib.KnngError(_lib.KNNG_EINVAL, _lib.last_error())
    return n


def _ptr(t: torch.Tensor | None) -> int | None:
    return None if t is None else t.data_ptr()


def _stream(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _aligned_buffer(nbytes: int, device) -> torch.Tensor:
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf[off:off + nbytes]


class KnnGraph:
    """A growing k-nn graph on one GPU.

    Create it with :meth:`build_exact` (brute-force initial graph) or
    :meth:`load` (points and lists supplied), then :meth:`insert` batches
    and :meth:`query` read-only k-nn searches.
    """

    def __init__(self, cfg: GraphConfig, device="cuda"):
        self.cfg = cfg
        self.device = torch.device(device)
        self.storage = _aligned_buffer(storage_bytes(cfg), self.device)
        self.workspace = _aligned_buffer(workspace_bytes(cfg), self.device)
        self._h = ctypes.c_void_p(None)

    # -- construction ---------------------------------------------------------
    @classmethod
    def build_exact(cls, cfg: GraphConfig, x: torch.Tensor, stream=None) -> "KnnGraph":
        g = cls(cfg, x.device)
        x = g._as_points(x)
        p = cfg.params()
        check(_lib.lib.knng_build_exact(ctypes.byref(p), _ptr(x), x.shape[0], _ptr(g.storage),
                                        g.storage.numel(), _ptr(g.workspace),
                                        g.workspace.numel(), _stream(stream),
                                        ctypes.byref(g._h)))
        g._keep = x
        return g

    @classmethod
    def load(cls, cfg: GraphConfig, x: torch.Tensor, ids: torch.Tensor, d: torch.Tensor,
             stream=None) -> "KnnGraph":
        g = cls(cfg, x.device)
        x = g._as_points(x)
        ids = ids.to(device=g.device, dtype=torch.int32).contiguous()
        d = d.to(device=g.device, dtype=torch.int32 if cfg.dtype == "u8" else torch.float32)
        d = d.contiguous()
        if ids.shape != (x.shape[0], cfg.k) or d.shape != ids.shape:
            raise ValueError("ids and d must have shape [n, k]")
        p = cfg.params()
        check(_lib.lib.knng_load(ctypes.byref(p), _ptr(x), x.shape[0], _ptr(ids), _ptr(d),
                                 _ptr(g.storage), g.storage.numel(), _ptr(g.workspace),
                                 g.workspace.numel(), _stream(stream), ctypes.byref(g._h)))
        g._keep = (x, ids, d)
        return g

    def close(self) -> None:
        """Free the handle (the device buffers are released with this object)."""
        h = getattr(self, "_h", None)
        lib = getattr(_lib, "lib", None)
        if h is not None and h.value and lib is not None:
            lib.knng_destroy(h)
        self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers -------------------------------------------------------------
    def _as_points(self, x: torch.Tensor) -> torch.Tensor:
        want = torch.uint8 if self.cfg.dtype == "u8" else torch.float32
        if x.dtype != want:
            raise TypeError(f"points must be {want}, got {x.dtype}")
        if x.dim() != 2 or x.shape[1] != self.cfg.dim:
            raise ValueError(f"points must have shape [m, {self.cfg.dim}]")
        return x.to(self.device).contiguous()

    def _dist_dtype(self):
        return torch.int32 if self.cfg.dtype == "u8" else torch.float32

    @property
    def n(self) -> int:
        return int(_lib.lib.knng_size(self._h))

    @property
    def query_count(self) -> int:
        return int(_lib.lib.knng_query_count(self._h))

    # -- operations ------------------------------------------------------------
    def insert(self, x: torch.Tensor, sims: bool = True, stats: bool = False, stream=None):
        """Insert a batch; returns (first id, per-point similarity counts or
        None) or, with ``stats``, (first id, sims, stats [b, 3] = search
        evaluations, lists read by the search, update evaluations)."""
        x = self._as_points(x)
        out = torch.empty(x.shape[0], dtype=torch.int32, device=self.device) if sims else None
        st = torch.empty((x.shape[0], 3), dtype=torch.int32, device=self.device) if stats else None
        first = ctypes.c_int64(0)
        check(_lib.lib.knng_insert_batch(self._h, _ptr(x), x.shape[0], ctypes.byref(first),
                                         _ptr(out), _ptr(st), _stream(stream)))
        if stats:
            return first.value, out, st
        return first.value, out

    def insert_exact(self, x: torch.Tensor, stream=None) -> int:
        """The naive method: insert a batch by comparing each point with every
        node (the graph stays exact if it was); returns the first new id."""
        x = self._as_points(x)
        first = ctypes.c_int64(0)
        check(_lib.lib.knng_insert_exact(self._h, _ptr(x), x.shape[0], ctypes.byref(first),
                                         _stream(stream)))
        return first.value

    def epoch(self, x: torch.Tensor | None, q: torch.Tensor | None, sims: bool = False,
              stats: bool = False, stream=None):
        """One serving epoch on the current snapshot: queries q and the insert
        batch x searched in one launch, then the batch's update.  Returns
        (first id, sims or None, query ids, query d, query evals); the query
        outputs are None when q is None.  With ``stats`` two more items
        follow: the inserts' [b, 3] stats (as :meth:`insert`) and the
        queries' list reads [m] (None where empty)."""
        b = 0 if x is None else x.shape[0]
        m = 0 if q is None else q.shape[0]
        if b:
            x = self._as_points(x)
        if m:
            q = self._as_points(q)
        qi = torch.empty((m, self.cfg.k), dtype=torch.int32, device=self.device) if m else None
        qd = torch.empty((m, self.cfg.k), dtype=self._dist_dtype(), device=self.device) if m else None
        qe = torch.empty(m, dtype=torch.int32, device=self.device) if m else None
        out = torch.empty(b, dtype=torch.int32, device=self.device) if (sims and b) else None
        st = torch.empty((b, 3), dtype=torch.int32, device=self.device) if (stats and b) else None
        qlr = torch.empty(m, dtype=torch.int32, device=self.device) if (stats and m) else None
        first = ctypes.c_int64(0)
        check(_lib.lib.knng_epoch(self._h, _ptr(x) if b else None, b, _ptr(q) if m else None, m,
                                  _ptr(qi), _ptr(qd), _ptr(qe), _ptr(qlr), ctypes.byref(first),
                                  _ptr(out), _ptr(st), _stream(stream)))
        if stats:
            return first.value, out, qi, qd, qe, st, qlr
        return first.value, out, qi, qd, qe

    def search(self, q: torch.Tensor, keys: torch.Tensor, trace: bool = False,
               list_reads: bool = False, stream=None):
        """Raw iGNNS with explicit restart keys; returns (ids, d, evals, trace)
        or, with ``list_reads``, (ids, d, evals, trace, list_reads)."""
        q = self._as_points(q)
        m = q.shape[0]
        keys = keys.to(device=self.device, dtype=torch.int64).contiguous()
        ids = torch.empty((m, self.cfg.k), dtype=torch.int32, device=self.device)
        d = torch.empty((m, self.cfg.k), dtype=self._dist_dtype(), device=self.device)
        ev = torch.empty(m, dtype=torch.int32, device=self.device)
        lr = torch.empty(m, dtype=torch.int32, device=self.device) if list_reads else None
        tr = None
        stride = 0
        if trace:
            stride = self.budget()
            tr = torch.full((m, stride), -1, dtype=torch.int32, device=self.device)
        check(_lib.lib.knng_search(self._h, _ptr(q), m, _ptr(keys), _ptr(ids), _ptr(d), _ptr(ev),
                                   _ptr(lr), _ptr(tr), stride, _stream(stream)))
        if list_reads:
            return ids, d, ev, tr, lr
        return ids, d, ev, tr

    def search_gnns(self, q: torch.Tensor, keys: torch.Tensor, restarts: int,
                    trace: bool = False, stream=None):
        """GNNS baseline search (fixed restarts, steepest climb); returns
        (ids, d, evals, trace)."""
        q = self._as_points(q)
        m = q.shape[0]
        keys = keys.to(device=self.device, dtype=torch.int64).contiguous()
        ids = torch.empty((m, self.cfg.k), dtype=torch.int32, device=self.device)
        d = torch.empty((m, self.cfg.k), dtype=self._dist_dtype(), device=self.device)
        ev = torch.empty(m, dtype=torch.int32, device=self.device)
        tr = None
        stride = 0
        if trace:
            stride = self.budget()
            tr = torch.full((m, stride), -1, dtype=torch.int32, device=self.device)
        check(_lib.lib.knng_search_gnns(self._h, _ptr(q), m, _ptr(keys), restarts, _ptr(ids),
                                        _ptr(d), _ptr(ev), _ptr(tr), stride, _stream(stream)))
        return ids, d, ev, tr

    def partition(self, p: int, iters: int = 5, imbalance=(1, 1), seed: int = 0x5EED,
                  stream=None):
        """Balanced k-medoids parts of the current nodes; returns (part [n],
        medoids [p]) as int32 device tensors."""
        nbytes = _lib.lib.knng_partition_scratch_bytes(self._h, p)
        if nbytes == 0:
            raise _lib.KnngError(_lib.KNNG_EINVAL, "invalid number of parts")
        scratch = _aligned_buffer(nbytes, self.device)
        part = torch.empty(self.n, dtype=torch.int32, device=self.device)
        med = torch.empty(p, dtype=torch.int32, device=self.device)
        check(_lib.lib.knng_partition(self._h, p, iters, imbalance[0], imbalance[1], seed,
                                      _ptr(scratch), nbytes, _ptr(part), _ptr(med),
                                      _stream(stream)))
        self._scratch = scratch
        return part, med

    def search_partitioned(self, q: torch.Tensor, keys: torch.Tensor, part: torch.Tensor,
                           p: int, stream=None):
        """Search every part separately, keep the k best; returns (ids, d, evals)."""
        q = self._as_points(q)
        m = q.shape[0]
        keys = keys.to(device=self.device, dtype=torch.int64).contiguous()
        part = part.to(device=self.device, dtype=torch.int32).contiguous()
        nbytes = _lib.lib.knng_search_partitioned_scratch_bytes(self._h, m, p)
        scratch = _aligned_buffer(max(nbytes, 256), self.device)
        ids = torch.empty((m, self.cfg.k), dtype=torch.int32, device=self.device)
        d = torch.empty((m, self.cfg.k), dtype=self._dist_dtype(), device=self.device)
        ev = torch.empty(m, dtype=torch.int32, device=self.device)
        check(_lib.lib.knng_search_partitioned(self._h, _ptr(q), m, _ptr(keys), _ptr(part), p,
                                               _ptr(scratch), nbytes, _ptr(ids), _ptr(d),
                                               _ptr(ev), _stream(stream)))
        self._scratch = scratch
        return ids, d, ev

    def query(self, q: torch.Tensor, list_reads: bool = False, stream=None):
        """Read-only k-nn query; returns (ids, d, evals[, list_reads])."""
        q = self._as_points(q)
        m = q.shape[0]
        ids = torch.empty((m, self.cfg.k), dtype=torch.int32, device=self.device)
        d = torch.empty((m, self.cfg.k), dtype=self._dist_dtype(), device=self.device)
        ev = torch.empty(m, dtype=torch.int32, device=self.device)
        lr = torch.empty(m, dtype=torch.int32, device=self.device) if list_reads else None
        check(_lib.lib.knng_query(self._h, _ptr(q), m, _ptr(ids), _ptr(d), _ptr(ev), _ptr(lr),
                                  _stream(stream)))
        if list_reads:
            return ids, d, ev, lr
        return ids, d, ev

    def step_counters(self, reset: bool = False) -> dict:
        """Search step counters since the last reset (the profiling build,
        libknng_counters.so, only; the regular build raises KNNG_EUNSUPPORTED)."""
        buf = (ctypes.c_uint64 * _lib.KNNG_NUM_STEP_COUNTERS)()
        check(_lib.lib.knng_step_counters(self._h, buf, 1 if reset else 0))
        return dict(zip(_lib.STEP_COUNTERS, (int(v) for v in buf)))

    def timing(self, enable: bool) -> None:
        """Start (clearing earlier totals) or stop per-stage event timing."""
        check(_lib.lib.knng_timing_enable(self._h, 1 if enable else 0))

    def timing_read(self) -> dict:
        """{stage: (total GPU ms, launches)} of the stages timed so far."""
        ms = (ctypes.c_double * len(_lib.STAGES))()
        cnt = (ctypes.c_int64 * len(_lib.STAGES))()
        check(_lib.lib.knng_timing_read(self._h, ms, cnt))
        return {name: (ms[i], cnt[i]) for i, name in enumerate(_lib.STAGES)}

    def lists(self, first: int = 0, count: int | None = None, stream=None):
        count = self.n - first if count is None else count
        ids = torch.empty((count, self.cfg.k), dtype=torch.int32, device=self.device)
        d = torch.empty((count, self.cfg.k), dtype=self._dist_dtype(), device=self.device)
        check(_lib.lib.knng_get_lists(self._h, first, count, _ptr(ids), _ptr(d), _stream(stream)))
        return ids, d

    def points(self, first: int = 0, count: int | None = None, stream=None):
        count = self.n - first if count is None else count
        want = torch.uint8 if self.cfg.dtype == "u8" else torch.float32
        x = torch.empty((count, self.cfg.dim), dtype=want, device=self.device)
        check(_lib.lib.knng_get_points(self._h, first, count, _ptr(x), _stream(stream)))
        return x

    def rows(self, first: int = 0, count: int | None = None, stream=None):
        """Stored scoring rows [count, row_bytes] (uint8 view of the bytes) and,
        for FP8 scoring, the row scales [count]; otherwise (rows, None)."""
        count = self.n - first if count is None else count
        rb = int(_lib.lib.knng_row_bytes(self._h))
        rows = torch.empty((count, rb), dtype=torch.uint8, device=self.device)
        scale = (torch.empty(count, dtype=torch.float32, device=self.device)
                 if self.cfg.score == "fp8" else None)
        check(_lib.lib.knng_get_rows(self._h, first, count, _ptr(rows), _ptr(scale),
                                     _stream(stream)))
        return rows, scale

    def budget(self, n: int | None = None) -> int:
        """The search budget B(n) of the library (current size if n is None)."""
        return int(_lib.lib.knng_budget(self._h, -1 if n is None else n))
