"""Seeded synthetic temporal-graph workloads.

This package only draws random numbers and lays them out as edge lists,
query lists and arrival traces.  It contains none of the traversal
arithmetic: both the CPU oracle and the GPU library consume what it
produces, and neither imports the other.
"""
from .gen import (  # noqa: F401
    INF,
    TMAX,
    Graph,
    uniform_graph,
    rmat_graph,
    bursty_pair_graph,
    tiny_graph,
    sample_sources,
    first_half_windows,
    log_uniform_windows,
    poisson_arrivals,
    query_kinds,
)
from .configs import CONFIGS, make_graph, make_queries  # noqa: F401
