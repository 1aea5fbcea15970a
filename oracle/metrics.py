"""Float64 diagnostics of a reconstructed state (test infrastructure only).

The paper states that cutting recovers the uncut state exactly up to machine
precision (Sec. III); these functions measure how close a state is to a
reference: squared norm, overlap <ref|psi>, fidelity
F = |<ref|psi>|^2 / (|ref|^2 |psi|^2), and the largest amplitude error with no
phase alignment (cutting fixes the global phase exactly).

1 - F is computed from the distance of the normalised, phase-aligned states,
d^2 = | psi/|psi| - e^{i arg<ref|psi>} ref/|ref| |^2, using 1 - F = d^2 - d^4/4,
which keeps full relative accuracy when F is close to 1.
"""

from __future__ import annotations

import numpy as np


def norm2(psi: np.ndarray) -> float:
    return float(np.vdot(psi, psi).real)


def overlap(ref: np.ndarray, psi: np.ndarray) -> complex:
    return complex(np.vdot(ref, psi))


def fidelity(ref: np.ndarray, psi: np.ndarray) -> float:
    ov = overlap(ref, psi)
    return abs(ov) ** 2 / (norm2(ref) * norm2(psi))


def one_minus_fidelity(ref: np.ndarray, psi: np.ndarray) -> float:
    ref = np.asarray(ref, dtype=np.complex128)
    psi = np.asarray(psi, dtype=np.complex128)
    ov = overlap(ref, psi)
    phase = ov / abs(ov) if abs(ov) > 0 else 1.0
    a = psi / np.sqrt(norm2(psi))
    b = phase * ref / np.sqrt(norm2(ref))
    d2 = norm2(a - b)
    return float(d2 - 0.25 * d2 * d2)


def max_abs_error(ref: np.ndarray, psi: np.ndarray) -> float:
    return float(np.max(np.abs(np.asarray(psi, dtype=np.complex128) - ref)))
