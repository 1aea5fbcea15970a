"""Expectation values of Pauli strings (test infrastructure only).

The paper's closing remark (Sec. VI) names expectation values as the setting
where the O(2^q) merge can be replaced by classical sums over subcircuit
quantities.  This oracle computes the quantity itself, from its definition on
the full 2^q state: <psi| P |psi> with P = P_{q-1} x ... x P_0, the Pauli
factor for qubit j given by character j of the label (I, X, Y, Z; qubit j is
bit j of the amplitude index, as everywhere in this package).
"""

from __future__ import annotations

import numpy as np

from .statevector import apply_1q

PAULI = {
    "I": np.eye(2, dtype=np.complex128),
    "X": np.array([[0, 1], [1, 0]], dtype=np.complex128),
    "Y": np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    "Z": np.array([[1, 0], [0, -1]], dtype=np.complex128),
}


def apply_pauli(psi: np.ndarray, q: int, label: str) -> np.ndarray:
    """P psi, one single-qubit Pauli matrix per qubit."""
    if len(label) != q:
        raise ValueError(f"label has {len(label)} characters for {q} qubits")
    out = np.array(psi, dtype=np.complex128)
    for j, p in enumerate(label):
        if p != "I":
            out = apply_1q(out, q, j, PAULI[p])
    return out


def expval(psi: np.ndarray, q: int, label: str) -> complex:
    """<psi| P |psi> (complex; the imaginary part vanishes for a Pauli string)."""
    return complex(np.vdot(psi, apply_pauli(psi, q, label)))
