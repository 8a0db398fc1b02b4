"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

Geometry, domain tree, block structure (Def. 2.3 under weak admissibility),
kernel entries, factor sets and right-hand sides. Nothing here evaluates the
H-matrix-vector product itself.
"""
from .tree import ClusterTree, BlockList, build_tree, uniform_tree, enumerate_blocks, stored_elements
from .factors import (HMatrixData, make_hmatrix, make_rhs, kernel_matrix, block_kernel,
                      dense_kernel, truncated_svd)
from .configs import WORKLOADS, Workload, build_workload, batch_problems, build_batch_member

__all__ = [
    "ClusterTree", "BlockList", "build_tree", "uniform_tree", "enumerate_blocks",
    "stored_elements", "HMatrixData", "make_hmatrix", "make_rhs", "kernel_matrix",
    "block_kernel", "dense_kernel", "truncated_svd", "WORKLOADS", "Workload",
    "build_workload", "batch_problems", "build_batch_member",
]
