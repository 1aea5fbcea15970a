"""Helpers shared by the GPU parity tests (mapping the device arena to oracle keys)."""

import numpy as np


def oracle_key(plan_cuts, oracle_cuts, seg, r):
    """Oracle variant key (segment, bits of adjacent cuts in gate order) of device variant r."""
    from oracle import cutting
    by_gate = {cu["gate_index"]: cu for cu in plan_cuts}
    bits = []
    for j in cutting.adjacent_cuts(oracle_cuts, seg):
        cu = by_gate[oracle_cuts[j].gate_index]
        pos = cu["bit_low"] if cu["boundary"] == seg else cu["bit_high"]
        bits.append((r >> pos) & 1)
    return (seg, tuple(bits))


def to_np(t):
    return t.detach().cpu().numpy().astype(np.complex128)
