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


TWO_QUBIT_KINDS = ("CZ", "CX")
