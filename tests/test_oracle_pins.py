"""Pins of the complex128 oracle against facts the paper and the mathematics fix.

None of these re-type the oracle's own formulas: they check it against exact
matrix identities (Eq. CZ, the CX/CZ relation), brute-force Kronecker-product
unitaries on tiny registers, textbook closed forms (uniform superposition,
product states, graph states, GHZ), and the paper's claim that cutting
recovers the uncut state exactly (Sec. III).
"""

import itertools
import math
import os

import numpy as np
import pytest

from inputs import Gate, SplitMix64, brickwork, equal_blocks, split_cuts, staircase
from oracle import cutting, gates as og, metrics, statevector

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- inputs

def test_splitmix64_reference_outputs():
    want = [int(l, 16) for l in open(os.path.join(GOLDEN, "splitmix64_seed0.txt"))
            if l.strip() and not l.startswith("#")]
    rng = SplitMix64(0)
    assert [rng.next_u64() for _ in range(3)] == want


def test_brickwork_structure():
    q, d, n, c = 12, 10, 2, 2
    g = brickwork(q, d, n, c, seed=0)
    assert sum(1 for x in g if x.kind == "RYRZ") == q * d
    cross = [k for k, x in enumerate(g) if x.kind == "CZ" and (x.q0 < 6) != (x.q1 < 6)]
    assert len(cross) == c
    # cut CZs close layers floor(j d / c) = 0 and 5
    layer_of = []
    layer = -1
    for x in g:
        if x.kind == "RYRZ" and x.q0 == 0:
            layer += 1
        layer_of.append(layer)
    assert [layer_of[k] for k in cross] == [0, 5]
    assert brickwork(q, d, n, c, seed=0) == g
    assert brickwork(q, d, n, c, seed=1) != g


def test_block_and_cut_splits():
    assert equal_blocks(32, 3) == [10, 11, 11]
    assert equal_blocks(12, 2) == [6, 6]
    assert split_cuts(6, 3) == [3, 3]
    assert split_cuts(8, 4) == [3, 3, 2]


# ---------------------------------------------------------------- gate identities

def kron_list(mats):
    out = np.ones((1, 1), dtype=np.complex128)
    for m in mats:
        out = np.kron(out, m)
    return out


def test_cz_decomposition_is_exact():
    """Eq. (CZ): CZ = (S x S + i S^dag x S^dag) / (1 + i), exactly in float64."""
    cz = np.diag([1, 1, 1, -1]).astype(np.complex128)
    rhs = cutting.S0 * np.kron(og.S, og.S) + cutting.S1 * np.kron(og.SDG, og.SDG)
    assert np.max(np.abs(rhs - cz)) == 0.0


def test_cx_from_cz_with_hadamards():
    """CX = (I x H) CZ (I x H) with H on the target (Sec. II.A.2); target side gets H S H."""
    # two qubits, little-endian: control = qubit 0 (bit 0), target = qubit 1 (bit 1)
    cx = np.zeros((4, 4), dtype=np.complex128)
    for x in range(4):
        y = x ^ 2 if x & 1 else x
        cx[y, x] = 1
    cz = np.diag([1, 1, 1, -1]).astype(np.complex128)
    h_t = np.kron(og.H, og.I2)          # kron(qubit1, qubit0)
    assert np.max(np.abs(h_t @ cz @ h_t - cx)) < 1e-15
    rhs = (cutting.S0 * np.kron(og.H @ og.S @ og.H, og.S)
           + cutting.S1 * np.kron(og.H @ og.SDG @ og.H, og.SDG))
    assert np.max(np.abs(rhs - cx)) < 1e-15


def random_small_circuit(q, ngates, seed):
    rng = SplitMix64(seed)
    kinds1 = ["H", "X", "Y", "Z", "S", "SDG", "T", "TDG", "RX", "RY", "RZ", "RYRZ"]
    out = []
    for _ in range(ngates):
        r = rng.next_u64()
        if r % 4 == 0 and q > 1:
            a = rng.next_u64() % q
            b = (a + 1 + rng.next_u64() % (q - 1)) % q
            out.append(Gate("CZ" if r % 8 == 0 else "CX", int(a), int(b)))
        else:
            k = kinds1[rng.next_u64() % len(kinds1)]
            out.append(Gate(k, int(rng.next_u64() % q), -1,
                            2 * math.pi * rng.uniform(), 2 * math.pi * rng.uniform()))
    return out


def dense_unitary(q, g):
    """Full 2^q x 2^q matrix of one gate, built from Kronecker products (qubit 0 rightmost)."""
    if g.kind in ("CZ", "CX"):
        u = np.zeros((1 << q, 1 << q), dtype=np.complex128)
        for x in range(1 << q):
            a, b = (x >> g.q0) & 1, (x >> g.q1) & 1
            if g.kind == "CZ":
                u[x, x] = -1 if (a and b) else 1
            else:
                u[x ^ (1 << g.q1) if a else x, x] = 1
        return u
    m = og.one_qubit_matrix(g.kind, g.p0, g.p1)
    return kron_list([m if j == g.q0 else og.I2 for j in reversed(range(q))])


@pytest.mark.parametrize("q,seed", [(1, 0), (2, 1), (3, 2), (4, 3), (5, 4)])
def test_statevector_matches_dense_unitary(q, seed):
    circ = random_small_circuit(q, 25, seed)
    psi = statevector.zero_state(q)
    u = np.eye(1 << q, dtype=np.complex128)
    for g in circ:
        u = dense_unitary(q, g) @ u
    assert np.max(np.abs(statevector.simulate(q, circ) - u @ psi)) < 1e-13


def test_textbook_states():
    q = 7
    psi = statevector.simulate(q, [Gate("H", j) for j in range(q)])
    assert np.allclose(psi, 2 ** (-q / 2), atol=1e-15, rtol=0)
    thetas = [0.3 * (j + 1) for j in range(q)]
    psi = statevector.simulate(q, [Gate("RY", j, -1, t) for j, t in enumerate(thetas)])
    want = np.ones(1, dtype=np.complex128)
    for t in thetas:                                   # qubit 0 rightmost
        want = np.kron(np.array([math.cos(t / 2), math.sin(t / 2)]), want)
    assert np.max(np.abs(psi - want)) < 1e-15
    phis = [0.7 * (j + 1) for j in range(q)]
    circ = [Gate("H", j) for j in range(q)] + [Gate("RZ", j, -1, p) for j, p in enumerate(phis)]
    psi = statevector.simulate(q, circ)
    x = np.arange(1 << q)
    phase = sum(np.where((x >> j) & 1, p / 2, -p / 2) for j, p in enumerate(phis))
    assert np.max(np.abs(psi - 2 ** (-q / 2) * np.exp(1j * phase))) < 1e-14


def test_ryrz_order_rz_acts_first():
    """The workload's single-qubit gate is Ry(theta) Rz(phi): Rz acts first.

    On |0>, Rz(phi) contributes only the global phase e^{-i phi/2}, so
    Ry(theta) Rz(phi)|0> = e^{-i phi/2} (cos theta/2, sin theta/2): both amplitudes
    share one phase.  The reversed order Rz(phi) Ry(theta)|0> would give them the
    phases e^{-i phi/2} and e^{+i phi/2}.  The matrix is checked entry by entry
    against its hand expansion with Qiskit's Ry(t) = [[c, -s], [s, c]] and
    Rz(t) = diag(e^{-it/2}, e^{it/2}).
    """
    th, ph = 1.1, 2.3
    c, s = math.cos(th / 2), math.sin(th / 2)
    em, ep = complex(math.cos(ph / 2), -math.sin(ph / 2)), complex(math.cos(ph / 2), math.sin(ph / 2))
    want = np.array([[c * em, -s * ep], [s * em, c * ep]])
    assert np.max(np.abs(og.one_qubit_matrix("RYRZ", th, ph) - want)) < 1e-15
    # through the simulator: single gates on |0> and on |1> (X first) of a 3-qubit register
    q = 3
    for pre, col in ((False, (c * em, s * em)), (True, (-s * ep, c * ep))):
        circ = ([Gate("X", 1)] if pre else []) + [Gate("RYRZ", 1, -1, th, ph)]
        psi = statevector.simulate(q, circ)
        assert abs(psi[0] - col[0]) < 1e-15 and abs(psi[2] - col[1]) < 1e-15
        assert np.max(np.abs(np.delete(psi, [0, 2]))) == 0.0


def test_brickwork_layer_product_state_closed_form():
    """One brickwork layer from |0^q>: RYRZ on every qubit, then CZ on the even pairs.

    The RYRZ layer gives the product state prod_j e^{-i phi_j/2} (cos theta_j/2,
    sin theta_j/2); the CZs multiply amplitude x by (-1)^{sum x_i x_{i+1}} over the
    even pairs (i, i+1).  Angles are read from the generated gate list itself.
    """
    q = 6
    g = brickwork(q, 1, 1, 0, seed=3)
    ang = {x.q0: (x.p0, x.p1) for x in g if x.kind == "RYRZ"}
    pairs = [(x.q0, x.q1) for x in g if x.kind == "CZ"]
    assert sorted(pairs) == [(0, 1), (2, 3), (4, 5)]
    x = np.arange(1 << q)
    want = np.ones(1 << q, dtype=np.complex128)
    for j, (th, ph) in ang.items():
        b = (x >> j) & 1
        want *= np.exp(-0.5j * ph) * np.where(b == 1, math.sin(th / 2), math.cos(th / 2))
    for a, b in pairs:
        want *= (-1.0) ** (((x >> a) & 1) * ((x >> b) & 1))
    assert np.max(np.abs(statevector.simulate(q, g) - want)) < 1e-14


def test_graph_state_closed_form():
    q = 8
    edges = [(0, 1), (1, 2), (2, 5), (3, 7), (4, 6), (0, 7), (5, 6)]
    circ = [Gate("H", j) for j in range(q)] + [Gate("CZ", a, b) for a, b in edges]
    psi = statevector.simulate(q, circ)
    x = np.arange(1 << q)
    par = sum(((x >> a) & 1) * ((x >> b) & 1) for a, b in edges)
    assert np.max(np.abs(psi - 2 ** (-q / 2) * (-1.0) ** par)) < 1e-15


# ---------------------------------------------------------------- cutting

def test_alpha_closed_form():
    """alpha over c cuts with p ones = 2^{-c/2} exp(i pi (2p - c)/4); each value exact dyadic."""
    for c in range(0, 7):
        for bits in itertools.product((0, 1), repeat=c):
            p = sum(bits)
            want = 2 ** (-c / 2) * np.exp(1j * math.pi * (2 * p - c) / 4)
            assert abs(cutting.alpha(bits) - want) < 1e-15


def test_nsub_counts():
    """N_sub = sum 2^{c_i}; n = 2 gives 2 * 2^c (Appendix B, Algorithm 1 complexity)."""
    for c in range(0, 5):
        g = brickwork(12, 10, 2, c, seed=0)
        cuts = cutting.find_cuts(12, g, [6, 6])
        assert len(cuts) == c
        assert cutting.n_subcircuits(cuts, 2) == 2 * 2 ** c
    g = brickwork(12, 10, 3, 4, seed=0)
    cuts = cutting.find_cuts(12, g, [4, 4, 4])
    assert [len(cutting.adjacent_cuts(cuts, i)) for i in range(3)] == [2, 4, 2]
    assert cutting.n_subcircuits(cuts, 3) == 4 + 16 + 4


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_cut_equals_uncut_small_config(seed):
    """Sec. III: cutting recovers the uncut state up to machine precision (q=12, 6+6, d=10, c=2)."""
    q = 12
    g = brickwork(q, 10, 2, 2, seed)
    ref = statevector.simulate(q, g)
    psi = cutting.cut_simulate(q, g, [6, 6])
    assert metrics.max_abs_error(ref, psi) < 1e-12
    assert abs(metrics.norm2(psi) - 1.0) < 1e-12


@pytest.mark.parametrize("q,n,c,sizes", [
    (12, 3, 4, [4, 4, 4]),
    (12, 4, 4, [3, 3, 3, 3]),       # 1+2+1 cuts: c_total exceeds c_max, all 2^{c_total} terms needed
    (13, 3, 3, [4, 4, 5]),
    (11, 2, 5, [3, 8]),
    (10, 2, 0, [5, 5]),
])
def test_cut_equals_uncut_more_partitions(q, n, c, sizes):
    g = brickwork(q, 8, n, c, seed=7, seg_sizes=sizes,
                  cuts_per_boundary=[1, 2, 1] if n == 4 else None)
    ref = statevector.simulate(q, g)
    assert metrics.max_abs_error(ref, cutting.cut_simulate(q, g, sizes)) < 1e-12


@pytest.mark.parametrize("q,n,copies", [(6, 2, 1), (6, 2, 3), (6, 3, 2), (9, 3, 1)])
def test_cut_cx_staircase(q, n, copies):
    """The paper's Fig. 1 family: CX cuts via H S H on the target side."""
    g = staircase(q, copies)
    sizes = equal_blocks(q, n)
    ref = statevector.simulate(q, g)
    cuts = cutting.find_cuts(q, g, sizes)
    assert len(cuts) == copies * (n - 1)
    assert metrics.max_abs_error(ref, cutting.cut_simulate(q, g, sizes)) < 1e-12


def test_ghz_via_one_cx_cut():
    q = 6
    g = [Gate("H", 0)] + [Gate("CX", i, i + 1) for i in range(q - 1)]
    psi = cutting.cut_simulate(q, g, [3, 3])
    want = np.zeros(1 << q, dtype=np.complex128)
    want[0] = want[-1] = 2 ** -0.5
    assert metrics.max_abs_error(want, psi) < 1e-15


def test_sampled_amplitudes_match_full_merge():
    q, sizes = 10, [5, 5]
    g = brickwork(q, 6, 2, 3, seed=3)
    cuts = cutting.find_cuts(q, g, sizes)
    states = cutting.variant_states(q, g, sizes, cuts)
    full = cutting.merge(sizes, cuts, states)
    xs = [0, 1, 31, 32, 513, 1023]
    assert np.max(np.abs(cutting.amplitudes(xs, sizes, cuts, states) - full[xs])) < 1e-15


def test_uncuttable_gate_rejected():
    g = [Gate("H", 0), Gate("CZ", 1, 2)]
    with pytest.raises(ValueError):
        # a two-qubit gate joining segments 0 and 2 has no boundary to be cut at
        cutting.find_cuts(6, [Gate("SWAP", 1, 4)], [2, 2, 2])
    assert len(cutting.find_cuts(4, g, [2, 2])) == 1
    assert len(cutting.find_cuts(4, [Gate("SWAP", 1, 2)], [2, 2])) == 1


def test_fidelity_metrics():
    rng = np.random.default_rng(0)
    a = rng.normal(size=64) + 1j * rng.normal(size=64)
    a /= np.linalg.norm(a)
    b = a * np.exp(0.3j)
    assert metrics.one_minus_fidelity(a, b) < 1e-15
    c = a.copy()
    c[0] += 1e-4
    f = metrics.fidelity(a, c)
    assert abs((1 - f) - metrics.one_minus_fidelity(a, c)) < 1e-12
