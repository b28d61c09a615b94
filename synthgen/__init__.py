"""Seeded synthetic temporal-graph generators.

This module is shared by the CPU oracle's tests, the GPU parity tests and the
benchmark.  It only draws random inputs (edge lists, timestamps, request
streams); it holds none of the betweenness arithmetic.
"""
from .graphs import (  # noqa: F401
    TemporalGraph,
    uniform_graph,
    chung_lu_graph,
    packed_uniform_graphs,
    request_stream,
    workload,
    WORKLOADS,
)
