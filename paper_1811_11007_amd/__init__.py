"""MI355X-native batched tree likelihood and branch-length optimisation.

The numerical work (partials, transition matrices, scaling, edge derivatives,
Newton smoothing, gradients) runs in hand-written HIP kernels for gfx950
behind the C ABI of include/pt.h; this package is its ctypes binding plus
the torch autograd wrapper.
"""
from ._lib import (  # noqa: F401
    PT_FP32, PT_FP64, PT_PLAN_GRAD, PT_PLAN_LOGLIK, PT_PLAN_OPTIMIZE, EXPORTS, LIB_PATH,
    PT_LOGLIK_REGISTERS, PT_LOGLIK_STORED,
    Alignment, Context, Plan, PTError, Trees, lib, opt_default, pt_batch_branch_grad,
    pt_batch_loglik, pt_batch_loglik_noalloc, pt_batch_optimize_branches, pt_model_info, pt_nni_neighbors,
    pt_topology_key,
    pt_tree_check, make_model, MLP, PT_NNI_FEATURES, pt_nni_features, pt_topology_keys, pt_radius_masks,
    pt_split_frequencies, pt_majority_consensus,
)
