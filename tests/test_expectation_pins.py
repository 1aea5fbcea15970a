"""Pins of the expectation-value oracle against closed forms (no GPU)."""

import numpy as np
import pytest

from inputs import Gate, brickwork, equal_blocks
from oracle import cutting, statevector
from oracle.expectation import apply_pauli, expval


def test_product_state_closed_forms():
    """Ry(t)|0> has <Z> = cos t, <X> = sin t, <Y> = 0; Rx(t)|0> has <Y> = -sin t."""
    rng = np.random.default_rng(3)
    q = 5
    th = rng.uniform(0, 2 * np.pi, q)
    psi = statevector.simulate(q, [Gate("RY", j, -1, th[j]) for j in range(q)])
    for j in range(q):
        lab = ["I"] * q
        for p, want in (("Z", np.cos(th[j])), ("X", np.sin(th[j])), ("Y", 0.0)):
            lab[j] = p
            assert abs(expval(psi, q, "".join(lab)) - want) < 1e-12
    lab = ["I"] * q
    lab[1], lab[3] = "Z", "X"
    assert abs(expval(psi, q, "".join(lab)) - np.cos(th[1]) * np.sin(th[3])) < 1e-12
    psi = statevector.simulate(q, [Gate("RX", j, -1, th[j]) for j in range(q)])
    for j in range(q):
        lab = ["I"] * q
        lab[j] = "Y"
        assert abs(expval(psi, q, "".join(lab)) + np.sin(th[j])) < 1e-12


def test_ghz_and_graph_state_stabilisers():
    q = 6
    ghz = statevector.simulate(q, [Gate("H", 0)] + [Gate("CX", j, j + 1) for j in range(q - 1)])
    assert abs(expval(ghz, q, "X" * q) - 1) < 1e-12
    assert abs(expval(ghz, q, "ZZIIII") - 1) < 1e-12
    assert abs(expval(ghz, q, "ZIIIII")) < 1e-12
    assert abs(expval(ghz, q, "YYXXXX") + 1) < 1e-12    # Y.Y on a GHZ pair gives -1
    # ring graph state: K_j = X_j Z_{j-1} Z_{j+1} has expectation 1
    g = [Gate("H", j) for j in range(q)] + [Gate("CZ", j, (j + 1) % q) for j in range(q)]
    gs = statevector.simulate(q, g)
    for j in range(q):
        lab = ["I"] * q
        lab[j] = "X"
        lab[(j - 1) % q] = "Z"
        lab[(j + 1) % q] = "Z"
        assert abs(expval(gs, q, "".join(lab)) - 1) < 1e-12


def test_norm_hermiticity_and_label_checks():
    q = 8
    psi = statevector.simulate(q, brickwork(q, 4, 2, 2, seed=1))
    assert abs(expval(psi, q, "I" * q) - 1) < 1e-12
    rng = np.random.default_rng(0)
    for _ in range(5):
        lab = "".join(rng.choice(list("IXYZ"), q))
        v = expval(psi, q, lab)
        assert abs(v.imag) < 1e-12 and abs(v.real) <= 1 + 1e-12
        # P^2 = I: applying the string twice returns the state
        assert np.max(np.abs(apply_pauli(apply_pauli(psi, q, lab), q, lab) - psi)) < 1e-12
    with pytest.raises(ValueError):
        expval(psi, q, "XX")


def test_cut_state_expectations_equal_uncut():
    """Cutting is exact (Sec. III), so every Pauli expectation of the merged state equals the uncut one."""
    q, n = 10, 2
    g = brickwork(q, 6, n, 3, seed=2)
    sizes = equal_blocks(q, n)
    cut = cutting.cut_simulate(q, g, sizes)
    ref = statevector.simulate(q, g)
    rng = np.random.default_rng(1)
    for _ in range(6):
        lab = "".join(rng.choice(list("IXYZ"), q))
        assert abs(expval(cut, q, lab) - expval(ref, q, lab)) < 1e-12
