"""Oracle: a plain, slow, CPU implementation of the online approximate k-nn
graph builder of "Fast Online k-nn Graph Building" (Debatty, Michiardi &
Mees, arXiv 1602.06819).

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only the tests, the smoke check of the
build entry point and the CPU-baseline leg of the benchmark may import it.
The product path (the HIP library and its Python binding) never imports,
calls or links anything here, and this package imports nothing from the
product.  The only code both sides share is the seeded input generator
package ``datagen``, which holds none of the method's arithmetic.

What is computed, step by step (the readings of points where the paper is
silent are listed in each function's docstring):

* exact k-nn graph by brute force (Section 2.1, "naive method"; Section
  8.5.2 uses it as ground truth)            -> :func:`exact.exact_graph`
* the same lists one row at a time, exact by branch and bound over any
  grouping of the points, and a snapshot graph whose lists are computed on
  first use (large initial graphs)            -> :class:`exact.LazyExactGraph`
* improved graph nearest-neighbour search, iGNNS (Section 3: random restart
  with the expansion test, eager first-improvement step, budget stop after
  n / speedup similarities)                   -> :func:`ignns.ignns`
* online insertion: search then Update (Algorithms 1 and 2), with explicit
  batch semantics; batch size 1 is the paper's sequential insertion
                                              -> :func:`online.insert_batch`
* the literal sequential transcription of Algorithms 1 and 2 (adds happen
  immediately), used to pin the batch form    -> :func:`online.insert_sequential_literal`
* read-only k-nn query on the current graph   -> :func:`online.query`
* GNNS, the baseline iGNNS improves on (fixed number of restarts, steepest
  climb over every neighbour)                 -> :func:`gnns.gnns`
* balanced k-medoids partitioning (Algorithm 4, one compute node) and the
  search of every partition merged to the k best (Algorithm 3)
                                              -> :mod:`partition`
* cosine dissimilarity 2 (1 - cos) as squared distance of normalized
  points                                      -> :mod:`cosine`
* inner-product similarity (not a metric; Params(metric="ip")): the
  dissimilarity -(x . y), the expansion test on exp(x . y)
                                              -> :func:`distance.dissim`,
                                                 :func:`exact.exact_graph_ip`
* the number formats of the float path's scoring rows (bfloat16, FP8 E4M3
  with a row scale), from their definitions  -> :mod:`quantize`

Float data: every distance here is float64 computed from the float32
inputs; the GPU's float path stores float32 distances and may decide near
ties differently, so its parity is checked by distance error, list
invariants and agreement rates rather than bit equality.

Parity status: every function is pinned by tests under ``tests/`` against
brute force, special cases, closed forms or invariants; the approximation
quality of the search (which neighbours a given budget finds) has no printed
value in the paper and is "parity unpinned" beyond those properties.
"""

from .distance import dissim, dissim_many, inner_product, sqdist, sqdist_many, INF_INT  # noqa: F401
from .restart import RestartOrder, restart_params, splitmix64_next  # noqa: F401
from .exact import (ExactRows, GroupedExactRows, LazyExactGraph, exact_graph,  # noqa: F401
                    exact_graph_ip, exact_graph_loops, exact_row)
from .graph import OracleGraph, Params, budget  # noqa: F401
from .ignns import ignns, SearchResult  # noqa: F401
from .gnns import gnns  # noqa: F401
from . import cosine, partition, quantize  # noqa: F401
from .online import (insert_batch, insert_sequential_literal, insert_stream, query,  # noqa: F401
                     merge_proposals, point_search_and_proposals, search_and_propose,
                     BatchResult, QUERY_KEY_BASE)
