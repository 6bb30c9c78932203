"""Seeded synthetic inputs: trees, model parameters and simulated alignments.

This package only draws and shapes input data.  It computes no transition
probability, likelihood or derivative; both the GPU library and the CPU
oracle consume what it produces.
"""
from .generate import (  # noqa: F401
    TIP_CODE, yule_tree, random_tree, all_topologies, gtr_params,
    simulate, compress, nni_bfs, Alignment, make_alignment, topology_id,
)
