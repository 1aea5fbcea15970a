"""Gate-by-gate state-vector simulation in complex128 (test infrastructure only).

This is the uncut baseline T_orig = O(2^q D) of Sec. III.A and the
StateVectorSimulate step that Algorithm 2 calls for every subcircuit.  The
state starts in |0...0>; qubit j is bit j of the amplitude index, as in
Qiskit (Sec. V.A.1).  No gate fusion, no reordering: one gate at a time in
list order, matching the paper's execution model (Sec. III).
"""

from __future__ import annotations

from typing import Iterable

import numpy as np

from .gates import one_qubit_matrix, two_qubit_matrix


def zero_state(q: int) -> np.ndarray:
    psi = np.zeros(1 << q, dtype=np.complex128)
    psi[0] = 1.0
    return psi


def apply_1q(psi: np.ndarray, q: int, t: int, u: np.ndarray) -> np.ndarray:
    """Apply a 2x2 matrix to qubit t: view the index as (high, bit t, low)."""
    v = psi.reshape(1 << (q - t - 1), 2, 1 << t)
    return np.einsum("ab,xbz->xaz", u, v).reshape(-1)


def apply_cz(psi: np.ndarray, q: int, a: int, b: int) -> np.ndarray:
    """CZ: negate every amplitude whose bits a and b are both 1."""
    idx = np.arange(1 << q, dtype=np.int64)
    both = ((idx >> a) & 1) & ((idx >> b) & 1)
    out = psi.copy()
    out[both == 1] *= -1.0
    return out


def apply_cx(psi: np.ndarray, q: int, c: int, t: int) -> np.ndarray:
    """CX: where control bit c is 1, swap the amplitudes that differ in bit t."""
    idx = np.arange(1 << q, dtype=np.int64)
    src = np.where(((idx >> c) & 1) == 1, idx ^ (1 << t), idx)
    return psi[src]


def apply_2q(psi: np.ndarray, q: int, a: int, b: int, u: np.ndarray) -> np.ndarray:
    """Apply a 4x4 matrix to qubits (a, b), its index being bit a + 2 bit b."""
    idx = np.arange(1 << q, dtype=np.int64)
    ba, bb = (idx >> a) & 1, (idx >> b) & 1
    rest = idx & ~((1 << a) | (1 << b))
    out = np.zeros_like(psi)
    for j in range(4):                      # source column: bits (j & 1, j >> 1) on (a, b)
        src = rest | ((j & 1) << a) | ((j >> 1) << b)
        out += u[ba + 2 * bb, j] * psi[src]
    return out


def apply_gate(psi: np.ndarray, q: int, g) -> np.ndarray:
    if g.kind == "CZ":
        return apply_cz(psi, q, g.q0, g.q1)
    if g.kind == "CX":
        return apply_cx(psi, q, g.q0, g.q1)
    if g.q1 >= 0:
        return apply_2q(psi, q, g.q0, g.q1, two_qubit_matrix(g.kind, g.p0))
    return apply_1q(psi, q, g.q0, one_qubit_matrix(g.kind, g.p0, g.p1))


def simulate(q: int, gates: Iterable, psi0: np.ndarray | None = None) -> np.ndarray:
    """Run the gate list on |0...0> (or on psi0) and return the final state."""
    psi = zero_state(q) if psi0 is None else np.array(psi0, dtype=np.complex128)
    for g in gates:
        psi = apply_gate(psi, q, g)
    return psi
