"""MI355X-native online approximate k-nn graph builder (Debatty, Michiardi &
Mees, "Fast Online k-nn Graph Building", arXiv 1602.06819).

The compute path is the C-ABI library ``libknng.so`` (include/knng.h) with
hand-written gfx950 HIP kernels; :mod:`.graph` is its Python front end and
:mod:`.metrics` holds evaluation helpers (recall, the paper's quality Q).
Importing :mod:`.graph` loads the library and fails if it is not built.
"""

__all__ = ["graph", "metrics", "build"]
