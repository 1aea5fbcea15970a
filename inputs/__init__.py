"""Seeded synthetic inputs shared by the oracle and the device-path tests.

This package holds no arithmetic of the circuit-cutting method: it only
produces gate lists (the circuits the method is applied to) from a seed.
Both the oracle (``oracle/``) and the HIP path's tests and benchmark take
their circuits from here, so the two sides see identical inputs while
sharing no code of the method itself.
"""

from .brickwork import (  # noqa: F401
    SplitMix64,
    Gate,
    equal_blocks,
    split_cuts,
    boundary_qubits,
    brickwork,
    staircase,
    GATE_KINDS,
)
