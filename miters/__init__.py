"""Seeded synthetic workload generators for exact-simulation (ES) equivalence checking.

This package builds combinational And-Inverter Graphs (AIGs) and miters and
serialises them as AIGER text (``.aag``) or binary (``.aig``) bytes.  It holds
no simulation: nothing here evaluates a circuit.  Both the plain CPU oracle
(``oracle/``) and the GPU path consume what it writes, so it is the one module
they share.

The paper (FastLEC, arXiv 2512.06627) represents circuits as latch-free AIGs
(Section 2.1) and checks two circuits by a miter that XORs paired primary
outputs and ORs the results (Section 2.1).  Its benchmark miters are not
available, so these generators stand in for them: multiplier miters of the
kind measured in Table 1 and Table 5, a multiply-accumulate datapath miter,
and XOR-dense compressor-like layered cones for batching and serving.
"""
from .rng import SplitMix64
from .aig import Aig, import_into
from .arith import (array_mult, wallace_mult, booth_wallace_mult,
                    mac_fused, mac_separate, ripple_add)
from .miter import (miter_of, mult_pair, mult_miter, mac_miter, minterm_miter,
                    inject_fault, layered_cone_miter, cone_batch, serve_pool, WORKLOADS, workload)

__all__ = [
    "SplitMix64", "Aig", "import_into", "array_mult", "wallace_mult",
    "booth_wallace_mult", "mac_fused", "mac_separate", "ripple_add",
    "miter_of", "mult_pair", "mult_miter", "mac_miter", "minterm_miter",
    "inject_fault", "layered_cone_miter", "cone_batch", "serve_pool", "WORKLOADS", "workload",
]
