"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This package only *draws numbers*: one- and two-electron integrals shaped like
small molecules, the workload descriptions, and the initial parameters of the
amplitude networks.  It contains none of the method's arithmetic (no
Hamiltonian construction, no amplitudes, no sampling), so that the oracle and
the HIP path can both read the same inputs without sharing any computation.
"""
from .integrals import make_integrals
from .params import (mlp_param_spec, transformer_param_spec, make_mlp_params,
                     make_transformer_params, flatten_params, unflatten_params,
                     nade_param_spec, make_nade_params)
from .workloads import (WORKLOADS, BATCHING_MODEL, workload, batching_molecules,
                        batching_params, batching_workload)

__all__ = [
    "make_integrals", "mlp_param_spec", "transformer_param_spec",
    "make_mlp_params", "make_transformer_params", "flatten_params",
    "unflatten_params", "nade_param_spec", "make_nade_params", "WORKLOADS",
    "BATCHING_MODEL", "workload", "batching_molecules", "batching_params", "batching_workload",
]
