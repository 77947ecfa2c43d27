"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package only draws and records inputs (gate names, qubit pairs, angles,
bitstrings, slice-id subsets). It holds no gate matrices and no
tensor-network arithmetic, so neither the oracle nor the GPU library can
inherit a mistake from it.
"""
from .circuits import (Gate, Circuit, Workload, make_rqc, grid_sites,
                       coupler_pairs, make_workload, WORKLOADS,
                       bits_of, int_of_bits, sample_bitstrings,
                       sample_slice_ids)

__all__ = ["Gate", "Circuit", "Workload", "make_rqc", "grid_sites",
           "coupler_pairs", "make_workload", "WORKLOADS", "bits_of",
           "int_of_bits", "sample_bitstrings", "sample_slice_ids"]
