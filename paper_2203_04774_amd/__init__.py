"""MI355X-native triangle listing under a given vertex ordering.

Implements the listing path of Lecuyer, Jachiet, Magnien, Tabourier,
"Tailored vertex ordering for faster triangle listing in large graphs"
(arXiv 2203.04774): orientation by an ordering (Section 1.3), Algorithms 1
(A++) and 2 (A+-) and the S2 variant (A--), and Definition 1's costs, in HIP
kernels for gfx950 behind the C-ABI of include/tl.h.
"""
from .tl import (ALGOS, JOB_PENDING, Batch, Csr, JobResult, Server, Summary, TLError, batch_from_graphs,
                 batch_orient, cost, get_tuning, order, order_neigh,  # noqa: F401
                 last_list_stats, list_count_noalloc, list_triangles, orient, raw_lib, release_cached_memory,
                 set_chunk_triangles, set_tuning)
from . import tl  # noqa: F401  (status codes: tl.TL_OK, ...)
