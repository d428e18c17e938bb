"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This package only *generates data*: undirected CSR graphs (Chung-Lu and
R-MAT stand-ins for the paper's SNAP networks, Table 3), optional per-slot
edge probabilities, and query traces.  It holds none of the method's
arithmetic (no edge hash, no sampling rule, no labelling, no gains): both the
oracle and the library receive the arrays it returns and apply the method
themselves.
"""

from .graphs import (  # noqa: F401
    Graph,
    splitmix64_stream,
    uniform01,
    chung_lu,
    rmat,
    from_edge_list,
    trivalency_p,
    uniform_p,
    normal_p,
    star_graph,
    path_graph,
    random_small_graph,
    from_arc_list,
    rmat_directed,
    wc_p,
    random_small_digraph,
)
from .configs import CONFIGS, Query, make_config, config_graphs, serving_trace  # noqa: F401
