"""Single- and two-qubit gate matrices in complex128 (test infrastructure only).

Conventions follow Qiskit, which the paper uses for every measurement
(Sec. V.A.1): Rx(t) = exp(-i t X / 2), Ry(t) = exp(-i t Y / 2),
Rz(t) = exp(-i t Z / 2); S = diag(1, i) as defined next to Eq. (CZ);
T = diag(1, e^{i pi / 4}).  RYRZ(theta, phi) = Ry(theta) Rz(phi), i.e. Rz is
applied first.
"""

from __future__ import annotations

import numpy as np

I2 = np.eye(2, dtype=np.complex128)
H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2.0)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
S = np.array([[1, 0], [0, 1j]], dtype=np.complex128)
SDG = S.conj().T
T = np.array([[1, 0], [0, np.exp(1j * np.pi / 4)]], dtype=np.complex128)
TDG = T.conj().T


def rx(t: float) -> np.ndarray:
    c, s = np.cos(t / 2), np.sin(t / 2)
    return np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)


def ry(t: float) -> np.ndarray:
    c, s = np.cos(t / 2), np.sin(t / 2)
    return np.array([[c, -s], [s, c]], dtype=np.complex128)


def rz(t: float) -> np.ndarray:
    return np.array([[np.exp(-0.5j * t), 0], [0, np.exp(0.5j * t)]], dtype=np.complex128)


def one_qubit_matrix(kind: str, p0: float = 0.0, p1: float = 0.0) -> np.ndarray:
    """2x2 matrix of a single-qubit gate kind."""
    fixed = {"H": H, "X": X, "Y": Y, "Z": Z, "S": S, "SDG": SDG, "T": T, "TDG": TDG}
    if kind in fixed:
        return fixed[kind]
    if kind == "RX":
        return rx(p0)
    if kind == "RY":
        return ry(p0)
    if kind == "RZ":
        return rz(p0)
    if kind == "RYRZ":
        return ry(p0) @ rz(p1)
    raise ValueError(f"not a single-qubit gate kind: {kind}")


TWO_QUBIT_KINDS = ("CZ", "CX", "SWAP", "ISWAP", "RXX", "RYY", "RZZ")

# Two-qubit matrices act on (q0, q1) with row/column index i = bit(q0) + 2 bit(q1).
SWAP = np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], dtype=np.complex128)
# iSWAP: |01> -> i|10>, |10> -> i|01>, |00> and |11> unchanged
ISWAP = np.array([[1, 0, 0, 0], [0, 0, 1j, 0], [0, 1j, 0, 0], [0, 0, 0, 1]], dtype=np.complex128)
CZ4 = np.diag([1, 1, 1, -1]).astype(np.complex128)
# CX with control q0 (bit 0) and target q1 (bit 1): flips bit 1 where bit 0 is set
CX4 = np.array([[1, 0, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0], [0, 1, 0, 0]], dtype=np.complex128)


def pauli_rotation(p: np.ndarray, t: float) -> np.ndarray:
    """exp(-i t P(x)P / 2) = cos(t/2) I - i sin(t/2) P(x)P, since (P(x)P)^2 = I."""
    pp = np.kron(p, p)
    return np.cos(t / 2) * np.eye(4, dtype=np.complex128) - 1j * np.sin(t / 2) * pp


def two_qubit_matrix(kind: str, p0: float = 0.0) -> np.ndarray:
    """4x4 matrix of a two-qubit gate kind (index bit(q0) + 2 bit(q1))."""
    if kind == "CZ":
        return CZ4
    if kind == "CX":
        return CX4
    if kind == "SWAP":
        return SWAP
    if kind == "ISWAP":
        return ISWAP
    if kind == "RXX":
        return pauli_rotation(X, p0)
    if kind == "RYY":
        return pauli_rotation(Y, p0)
    if kind == "RZZ":
        return pauli_rotation(Z, p0)
    raise ValueError(f"not a two-qubit gate kind: {kind}")
