"""Pins of the oracle's two-qubit gates and their operator-Schmidt cuts (no GPU).

Eq. (schmidt): U = sum_l s_l A_l (x) B_l with Schmidt rank k = 2 for controlled
gates (CZ, CX) and k = 4 for the other non-local gates such as SWAP (Sec. II.A.2).
The oracle takes the decomposition from a singular value decomposition; these
tests pin it to the ranks the paper states, to closed forms of the Schmidt
values, to the gates' defining actions on basis states, and to the exactness of
cutting (Sec. III).
"""

import numpy as np
import pytest

from inputs import Gate, brickwork, equal_blocks
from oracle import cutting, statevector
from oracle.gates import CX4, CZ4, ISWAP, SWAP, H, T, X, Y, Z, pauli_rotation, two_qubit_matrix


def basis(q, x):
    v = np.zeros(1 << q, dtype=np.complex128)
    v[x] = 1.0
    return v


def test_two_qubit_gates_on_basis_states():
    """Defining actions, with qubit 0 = bit 0: SWAP exchanges the bits, iSWAP does so
    with a factor i on |01> and |10>, RZZ(t) multiplies by e^{-i t z0 z1 / 2}."""
    q = 3
    for x in range(8):
        b0, b1 = x & 1, (x >> 1) & 1
        swapped = (x & 4) | (b0 << 1) | b1
        got = statevector.simulate(q, [Gate("SWAP", 0, 1)], basis(q, x))
        assert np.allclose(got, basis(q, swapped))
        got = statevector.simulate(q, [Gate("ISWAP", 1, 0)], basis(q, x))
        assert np.allclose(got, (1j if b0 != b1 else 1.0) * basis(q, swapped))
        t = 0.83
        got = statevector.simulate(q, [Gate("RZZ", 0, 2, t)], basis(q, x))
        z = (1 - 2 * b0) * (1 - 2 * ((x >> 2) & 1))
        assert np.allclose(got, np.exp(-0.5j * t * z) * basis(q, x))
    # RXX(pi) = -i X (x) X and RYY(pi) = -i Y (x) Y
    assert np.allclose(pauli_rotation(X, np.pi), -1j * np.kron(X, X))
    assert np.allclose(two_qubit_matrix("RYY", np.pi), -1j * np.kron(Y, Y))
    # CX4: control on the first qubit (bit 0)
    psi = statevector.simulate(2, [Gate("X", 0)])
    assert np.allclose(statevector.apply_2q(psi, 2, 0, 1, CX4), basis(2, 3))


def test_schmidt_ranks_are_the_papers():
    """k = 2 for CZ and CX, k = 4 for SWAP, iSWAP and a generic interaction; a
    product of single-qubit gates has rank 1; RZZ(t) has rank 2 unless t is a
    multiple of pi (then it is a product, up to phase)."""
    rank = lambda u: len(cutting.schmidt_terms(u))
    assert rank(CZ4) == 2 and rank(CX4) == 2
    assert rank(SWAP) == 4 and rank(ISWAP) == 4
    gen = pauli_rotation(X, 0.4) @ pauli_rotation(Y, 1.1) @ pauli_rotation(Z, 2.3)
    assert rank(gen) == 4
    assert rank(np.kron(T, H)) == 1
    assert rank(pauli_rotation(Z, 0.7)) == 2
    assert rank(pauli_rotation(Z, np.pi)) == 1


def test_schmidt_values_closed_forms():
    """Realigned SWAP is a permutation matrix: values (1, 1, 1, 1).  CZ =
    |0><0| (x) I + |1><1| (x) Z: (sqrt 2, sqrt 2).  RZZ(t) = cos(t/2) II - i sin(t/2) ZZ
    with orthogonal I, Z of norm sqrt 2: (2 |cos t/2|, 2 |sin t/2|).  Any 4 x 4
    unitary has sum of s_l^2 = ||U||_F^2 = 4."""
    sv = lambda u: sorted(abs(t[0]) for t in cutting.schmidt_terms(u))
    assert np.allclose(sv(SWAP), [1, 1, 1, 1])
    assert np.allclose(sv(CZ4), [np.sqrt(2)] * 2)
    t = 0.7
    assert np.allclose(sv(pauli_rotation(Z, t)), sorted([2 * np.cos(t / 2), 2 * np.sin(t / 2)]))
    rng = np.random.default_rng(0)
    a = rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4))
    u, _ = np.linalg.qr(a)
    assert abs(sum(s ** 2 for s in sv(u)) - 4) < 1e-12


def test_schmidt_terms_rebuild_the_gate():
    """The terms, placed with A on q0 (bit 0) and B on q1 (bit 1), give back U; a
    transposed placement (B on q0) fails for a non-symmetric gate, so the
    realignment is pinned to the index convention."""
    rng = np.random.default_rng(1)
    u, _ = np.linalg.qr(rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4)))
    terms = cutting.schmidt_terms(u)
    assert np.allclose(sum(s * np.kron(b, a) for s, a, b in terms), u)
    assert not np.allclose(sum(s * np.kron(a, b) for s, a, b in terms), u)


@pytest.mark.parametrize("kind", ["SWAP", "ISWAP", "RXX", "RYY", "RZZ", "CAN"])
@pytest.mark.parametrize("n,q,c", [(2, 8, 3), (3, 9, 4)])
def test_cut_equals_uncut(kind, n, q, c):
    """Sec. III: cutting is exact, for rank-4 and rank-2 Schmidt cuts too."""
    g = brickwork(q, 5, n, c, seed=q + n, boundary_gate=kind, bulk_gate="SWAP" if kind == "CAN" else "CZ")
    sizes = equal_blocks(q, n)
    ref = statevector.simulate(q, g)
    got = cutting.cut_simulate(q, g, sizes)
    assert np.max(np.abs(ref - got)) < 1e-12


def test_swap_carries_a_qubit_across_the_boundary():
    """X on the last qubit of segment 0, then SWAP across the boundary: the cut
    pipeline returns the basis state with the bit on the first qubit of segment 1."""
    q, sizes = 6, [3, 3]
    got = cutting.cut_simulate(q, [Gate("X", 2), Gate("SWAP", 2, 3)], sizes)
    assert np.allclose(got, basis(q, 1 << 3))
    cuts = cutting.find_cuts(q, [Gate("X", 2), Gate("SWAP", 2, 3)], sizes)
    assert cutting.n_subcircuits(cuts, 2) == 4 + 4


def test_planted_mistakes_break_exactness():
    """Each plausible mistake in the Schmidt cut breaks cut == uncut: a conjugated
    factor, a transposed factor, or a dropped term (rank 4 truncated to 3).  (The
    SVD's Schmidt values are real and positive, so the phases sit in the factors.)"""
    q, sizes = 8, [4, 4]
    g = brickwork(q, 4, 2, 2, seed=5, boundary_gate="ISWAP")
    ref = statevector.simulate(q, g)
    real_terms = cutting.cut_terms
    planted = {
        "conjugated factor": lambda c: [(s, a.conj(), b) for s, a, b in real_terms(c)],
        "transposed factor": lambda c: [(s, a.T, b) for s, a, b in real_terms(c)],
        "dropped term": lambda c: real_terms(c)[:3],
    }
    try:
        for name, fake in planted.items():
            cutting.cut_terms = fake
            got = cutting.cut_simulate(q, g, sizes)
            assert np.max(np.abs(ref - got)) > 1e-3, name
    finally:
        cutting.cut_terms = real_terms
    assert np.max(np.abs(ref - cutting.cut_simulate(q, g, sizes))) < 1e-12


def dense_two_qubit(q, a, b, u):
    """2^q x 2^q matrix of a 4x4 gate on (a, b), entry by entry."""
    out = np.zeros((1 << q, 1 << q), dtype=np.complex128)
    mask = (1 << a) | (1 << b)
    for x in range(1 << q):
        for y in range(1 << q):
            if (x & ~mask) == (y & ~mask):
                out[y, x] = u[((y >> a) & 1) + 2 * ((y >> b) & 1), ((x >> a) & 1) + 2 * ((x >> b) & 1)]
    return out


@pytest.mark.parametrize("q", [2, 3, 4])
def test_two_qubit_apply_matches_dense_matrices(q):
    """Gate-by-gate simulation with the new kinds (both qubit orders) against the
    product of dense matrices built entry by entry."""
    rng = np.random.default_rng(q)
    circ = [Gate("H", j) for j in range(q)] + [Gate("T", 0)]
    for _ in range(12):
        a, b = rng.choice(q, 2, replace=False)
        circ.append(Gate(str(rng.choice(["SWAP", "ISWAP", "RXX", "RYY", "RZZ"])), int(a), int(b),
                         float(rng.uniform(0, 2 * np.pi))))
        circ.append(Gate("RYRZ", int(rng.integers(q)), -1, float(rng.uniform(0, 6)), float(rng.uniform(0, 6))))
    u = np.eye(1 << q, dtype=np.complex128)
    for g in circ:
        if g.q1 >= 0:
            u = dense_two_qubit(q, g.q0, g.q1, two_qubit_matrix(g.kind, g.p0)) @ u
        else:
            u = _dense_1q(q, g) @ u
    assert np.max(np.abs(statevector.simulate(q, circ) - u[:, 0])) < 1e-13


def _dense_1q(q, g):
    from oracle.gates import one_qubit_matrix
    m = one_qubit_matrix(g.kind, g.p0, g.p1)
    out = np.ones((1, 1), dtype=np.complex128)
    for j in reversed(range(q)):                      # qubit 0 rightmost
        out = np.kron(out, m if j == g.q0 else np.eye(2))
    return out
