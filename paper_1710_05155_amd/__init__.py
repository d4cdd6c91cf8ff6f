"""MI355X-native multispin Kob-Andersen Monte Carlo (Boccagna, arXiv 1710.05155).

The product is libka.so (C ABI in include/ka.h: hand-written HIP kernels for gfx950 plus
host C++); `ka` is its thin ctypes binding with the same function names.
"""
from . import ka  # noqa: F401
from .ka import (  # noqa: F401
    KaError, ka_footprint, ka_free, ka_get_state, ka_graph_export, ka_graph_from_adjacency,
    ka_graph_info, ka_graph_lattice, ka_graph_rrg, ka_init, ka_init_k, ka_last_error,
    ka_observe, ka_run, ka_set_option, ka_set_state, ka_sim_path, ka_sweep, ka_timing,
)
