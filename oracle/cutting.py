"""Gate cutting, subcircuit simulation and merging in complex128 (test infrastructure only).

Follows the paper's three stages (Sec. III.A, Appendix B):

* Algorithm 1 (preprocessing): scan the circuit for two-qubit gates whose
  qubits lie in different segments, split each segment's gate list at those
  gates, and form one subcircuit per assignment b in {0,1}^{c_i} of the cuts
  adjacent to the segment: S where b_j = 0 and S^dagger where b_j = 1 on the
  cut qubit (H S H / H S^dagger H on the target of a cut CX, because
  CX = (I x H) CZ (I x H), Sec. II.A.2 and Appendix B).
* Algorithm 2 (subcircuit simulation): simulate every subcircuit on its own
  2^{q_i} register.
* Algorithm 3 (merging): Psi = sum over global combinations m of
  alpha_m (psi_n^{(r_n)} x ... x psi_1^{(r_1)}).

The weights come from Eq. (CZ): CZ = (1/(1+i)) (S x S + i S^dagger x S^dagger),
so each cut contributes s_0 = 1/(1+i) for the S term and s_1 = i/(1+i) for
the S^dagger term, and alpha_m is the product over all cuts.

Reading taken where the paper is loose: Algorithm 3 and Table I count
2^{c_max} merge terms, but the number of distinct global combinations is
2^{c_total} (they coincide for n <= 3).  This oracle sums all 2^{c_total}
combinations, which is what the exact identity requires.

Other two-qubit gates (SWAP, iSWAP, RXX, RYY, RZZ) are cut through the
operator-Schmidt decomposition of Eq. (schmidt): U = sum_l s_l A_l (x) B_l.
This oracle obtains it from the singular value decomposition of the 4x4
matrix realigned so that rows index qubit q0's (row, column) pair and columns
qubit q1's; the rank k (1, 2 or 4) is the number of nonzero singular values
and every cut contributes k terms.  A variant key then lists, per adjacent
cut, the index of its term (0/1 = S / S^dagger for CZ and CX).

Segment 0 holds the lowest-index qubits; the Kronecker product places
segment 0 in the least significant position (little-endian, Qiskit order).
"""

from __future__ import annotations

import itertools
from typing import Dict, List, NamedTuple, Sequence, Tuple

import numpy as np

from .gates import H, S, SDG, two_qubit_matrix
from .statevector import apply_1q, apply_2q, simulate

S0 = 1.0 / (1.0 + 1.0j)      # weight of the S (x) S term, Eq. (CZ)
S1 = 1.0j / (1.0 + 1.0j)     # weight of the S^dagger (x) S^dagger term, Eq. (CZ)


class Cut(NamedTuple):
    gate_index: int
    kind: str          # gate kind ("CZ", "CX", "SWAP", ...)
    qubits: Tuple[int, int]   # (q0, q1) as in the gate (CX: control, target)
    segs: Tuple[int, int]     # segment of q0, segment of q1
    p0: float = 0.0           # angle of RXX / RYY / RZZ


def schmidt_terms(u: np.ndarray, tol: float = 1e-12) -> List[Tuple[complex, np.ndarray, np.ndarray]]:
    """Operator-Schmidt decomposition (Eq. schmidt) of a 4x4 matrix acting on (q0, q1)
    with index bit(q0) + 2 bit(q1): terms (s_l, A_l on q0, B_l on q1), nonzero s_l only.

    u[(a0 + 2 a1), (b0 + 2 b1)] = sum_l s_l A_l[a0, b0] B_l[a1, b1]; realigning to
    R[(a0, b0), (a1, b1)] turns this into the singular value decomposition of R."""
    u4 = np.asarray(u, dtype=np.complex128).reshape(2, 2, 2, 2)      # [a1, a0, b1, b0]
    r = u4.transpose(1, 3, 0, 2).reshape(4, 4)                         # [(a0, b0), (a1, b1)]
    left, sv, right = np.linalg.svd(r)
    return [(complex(sv[l]), left[:, l].reshape(2, 2), right[l, :].reshape(2, 2))
            for l in range(4) if sv[l] > tol * sv[0]]


def cut_terms(c: Cut) -> List[Tuple[complex, np.ndarray, np.ndarray]]:
    """The terms (weight, matrix on q0, matrix on q1) a cut contributes.

    CZ and CX: Eq. (CZ), S (x) S with s_0 and S^dagger (x) S^dagger with s_1 (H S H
    on the target of a CX).  Other kinds: the Schmidt terms of their matrix."""
    if c.kind == "CZ":
        return [(S0, S, S), (S1, SDG, SDG)]
    if c.kind == "CX":
        return [(S0, S, H @ S @ H), (S1, SDG, H @ SDG @ H)]
    return schmidt_terms(two_qubit_matrix(c.kind, c.p0))


class LocalGate(NamedTuple):
    kind: str
    q0: int
    q1: int = -1
    p0: float = 0.0
    p1: float = 0.0
    matrix: np.ndarray | None = None   # set for cut insertions


def segment_offsets(sizes: Sequence[int]) -> List[int]:
    out, acc = [], 0
    for s in sizes:
        out.append(acc)
        acc += s
    return out


def segment_of_qubit(sizes: Sequence[int]) -> List[int]:
    seg = []
    for i, s in enumerate(sizes):
        seg += [i] * s
    return seg


def find_cuts(q: int, gates: Sequence, sizes: Sequence[int]) -> List[Cut]:
    """Algorithm 1, first step: the two-qubit gates that straddle segments, in gate order."""
    if sum(sizes) != q:
        raise ValueError("segment sizes must add up to q")
    seg = segment_of_qubit(sizes)
    cuts = []
    for k, g in enumerate(gates):
        if g.q1 < 0:
            continue
        sa, sb = seg[g.q0], seg[g.q1]
        if sa == sb:
            continue
        if abs(sa - sb) != 1:
            raise ValueError(f"gate {k} ({g.kind}) joins non-adjacent segments")
        cuts.append(Cut(k, g.kind, (g.q0, g.q1), (sa, sb), g.p0))
    return cuts


def adjacent_cuts(cuts: Sequence[Cut], i: int) -> List[int]:
    """Indices of the cuts touching segment i, in gate order (c_i = their count)."""
    return [j for j, c in enumerate(cuts) if i in c.segs]


def n_subcircuits(cuts: Sequence[Cut], n: int) -> int:
    """N_sub = sum_i prod over the cuts adjacent to segment i of their rank k_j
    (Sec. III.A: sum_i k^{c_i} when every cut has rank k)."""
    total = 0
    for i in range(n):
        v = 1
        for j in adjacent_cuts(cuts, i):
            v *= len(cut_terms(cuts[j]))
        total += v
    return total


def subcircuit(gates: Sequence, sizes: Sequence[int], i: int, cuts: Sequence[Cut],
               bits: Dict[int, int]) -> List[LocalGate]:
    """Algorithm 1: the gate list of segment i for one assignment of its cut terms.

    ``bits`` maps a cut index (into ``cuts``) to the index of its term (for CZ and
    CX: 0 = S term, 1 = S^dagger term).  Qubits are renumbered to the segment's
    local register.
    """
    off = segment_offsets(sizes)[i]
    seg = segment_of_qubit(sizes)
    cut_at = {c.gate_index: j for j, c in enumerate(cuts)}
    out: List[LocalGate] = []
    for k, g in enumerate(gates):
        if k in cut_at:
            j = cut_at[k]
            c = cuts[j]
            if i not in c.segs:
                continue
            side = 0 if c.segs[0] == i else 1
            local = c.qubits[side] - off
            _, a, b = cut_terms(c)[bits[j]]
            out.append(LocalGate("U", local, matrix=a if side == 0 else b))
            continue
        if seg[g.q0] != i:
            continue
        if g.q1 >= 0:
            out.append(LocalGate(g.kind, g.q0 - off, g.q1 - off, g.p0))
        else:
            out.append(LocalGate(g.kind, g.q0 - off, -1, g.p0, g.p1))
    return out


def simulate_local(nq: int, local: Sequence[LocalGate]) -> np.ndarray:
    """StateVectorSimulate (Algorithm 2) on a segment register."""
    from .statevector import apply_cx, apply_cz
    from .gates import one_qubit_matrix
    psi = np.zeros(1 << nq, dtype=np.complex128)
    psi[0] = 1.0
    for g in local:
        if g.kind == "U":
            psi = apply_1q(psi, nq, g.q0, g.matrix)
        elif g.kind == "CZ":
            psi = apply_cz(psi, nq, g.q0, g.q1)
        elif g.kind == "CX":
            psi = apply_cx(psi, nq, g.q0, g.q1)
        elif g.q1 >= 0:
            psi = apply_2q(psi, nq, g.q0, g.q1, two_qubit_matrix(g.kind, g.p0))
        else:
            psi = apply_1q(psi, nq, g.q0, one_qubit_matrix(g.kind, g.p0, g.p1))
    return psi


def variant_states(q: int, gates: Sequence, sizes: Sequence[int],
                   cuts: Sequence[Cut] | None = None) -> Dict[Tuple[int, Tuple[int, ...]], np.ndarray]:
    """Algorithm 2: every subcircuit state, keyed by (segment, term indices of its adjacent cuts in gate order)."""
    if cuts is None:
        cuts = find_cuts(q, gates, sizes)
    out = {}
    for i, nq in enumerate(sizes):
        adj = adjacent_cuts(cuts, i)
        for b in itertools.product(*[range(len(cut_terms(cuts[j]))) for j in adj]):
            bits = dict(zip(adj, b))
            out[(i, tuple(b))] = simulate_local(nq, subcircuit(gates, sizes, i, cuts, bits))
    return out


def alpha(bits: Sequence[int], cuts: Sequence[Cut] | None = None) -> complex:
    """alpha_m = product over cuts of the weight of the chosen term: s_{b_j} from
    Eq. (CZ) for CZ / CX (the default when ``cuts`` is omitted), the Schmidt
    coefficient for the other kinds."""
    a = 1.0 + 0.0j
    for j, b in enumerate(bits):
        if cuts is None:
            a *= S0 if b == 0 else S1
        else:
            a *= cut_terms(cuts[j])[b][0]
    return a


def combinations(cuts: Sequence[Cut]):
    """Every global combination m: one term index per cut."""
    return itertools.product(*[range(len(cut_terms(c))) for c in cuts])


def merge(sizes: Sequence[int], cuts: Sequence[Cut], states) -> np.ndarray:
    """Algorithm 3: plain sum over all global combinations (2^{c_total} for rank-2 cuts)."""
    n = len(sizes)
    adj = [adjacent_cuts(cuts, i) for i in range(n)]
    psi = None
    for m in combinations(cuts):
        phi = np.ones(1, dtype=np.complex128)
        for i in range(n):                      # segment 0 ends up least significant
            r = tuple(m[j] for j in adj[i])
            phi = np.kron(states[(i, r)], phi)
        term = alpha(m, cuts) * phi
        psi = term if psi is None else psi + term
    return psi


def cut_simulate(q: int, gates: Sequence, sizes: Sequence[int]) -> np.ndarray:
    """The whole cut pipeline (Algorithms 1-3): returns the reconstructed 2^q state."""
    cuts = find_cuts(q, gates, sizes)
    states = variant_states(q, gates, sizes, cuts)
    return merge(sizes, cuts, states)


def amplitudes(xs: Sequence[int], sizes: Sequence[int], cuts: Sequence[Cut], states) -> np.ndarray:
    """Selected amplitudes Psi[x] of the merged state, each summed over all combinations."""
    n = len(sizes)
    off = segment_offsets(sizes)
    adj = [adjacent_cuts(cuts, i) for i in range(n)]
    out = np.zeros(len(xs), dtype=np.complex128)
    combos = list(combinations(cuts))
    weights = [alpha(m, cuts) for m in combos]
    for t, x in enumerate(xs):
        local = [(int(x) >> off[i]) & ((1 << sizes[i]) - 1) for i in range(n)]
        acc = 0.0 + 0.0j
        for m, w in zip(combos, weights):
            term = w
            for i in range(n):
                term *= states[(i, tuple(m[j] for j in adj[i]))][local[i]]
            acc += term
        out[t] = acc
    return out


def uncut_simulate(q: int, gates: Sequence) -> np.ndarray:
    """T_orig: the same circuit simulated without cutting."""
    return simulate(q, gates)
