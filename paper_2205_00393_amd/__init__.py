"""Sliced tensor-network contraction of random quantum circuits on MI355X.

Host planner (network, greedy path, lifetime-based slicing) and HIP
execution, both in libltn (C ABI in include/ltn.h); this package marshals
arguments and lends PyTorch device memory and streams.
"""
from ._lib import LtnError, lib, MODES
from .network import (Network, greedy_path, tree_costs, tree_stem, stem_profile, slice_finder,
                      path_search, slice_refine, slice_greedy_overhead, tree_reconfigure)
from .plan import Plan, Prepared, kernel_name, prepare, permute

__all__ = ["LtnError", "lib", "MODES", "Network", "greedy_path", "tree_costs", "tree_stem",
           "stem_profile", "slice_finder", "path_search", "slice_refine", "slice_greedy_overhead",
           "tree_reconfigure", "Plan", "Prepared", "kernel_name", "prepare", "permute"]
