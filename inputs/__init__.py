"""Seeded synthetic inputs shared by the oracle and the GPU path (no simulation code)."""
from .circuits import (  # noqa: F401
    PHILOX_SEED, Circuit, Request, batch_circuit, batch_sizes, batch_workload,
    layered_circuit, plain_large, plain_mid, plain_small, plain_xlarge, random_gate_list,
    random_layers, serving_params, serving_request, serving_workload,
    OP_H, OP_S, OP_CNOT, OP_SDG, OP_X, OP_Y, OP_Z, OP_CZ, OP_SWAP, TWO_QUBIT_OPS,
)
from .bm_clifford import (  # noqa: F401,E402
    CliffordCircuit, clifford_from_choices, clifford_workload, random_clifford,
)
from .programs import Program, random_program  # noqa: F401,E402
