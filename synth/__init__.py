"""Seeded synthetic binary-program generators (inputs only, no solver arithmetic)."""
from .generators import (  # noqa: F401
    Problem, set_cover, independent_set, graph_matching, knapsack, batch_instances,
    random_tiny, workload, WORKLOADS, sigmoid, row_cluster,
)
