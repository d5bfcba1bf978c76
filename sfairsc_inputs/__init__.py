"""Seeded synthetic inputs for the s-FairSC solver and its CPU oracle.

This package only *generates* inputs: graphs (CSR adjacency), group labels,
planted clusters, random placeholder constraint matrices and group
memberships.  It contains none of the method's arithmetic (no Laplacian,
no projection, no eigensolver, no k-means), so both the GPU library's tests and
the oracle's tests can draw the same inputs from it without sharing code.
"""

from .msbm import (  # noqa: F401
    MSBMGraph,
    msbm,
    msbm_from_blocks,
    relabel,
    workload,
    WORKLOADS,
    random_sparse_graph,
)
from .general import random_laplacian, overlapping_memberships  # noqa: F401
