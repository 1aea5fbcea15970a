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

Segment 0 holds the lowest-index qubits; the Kronecker product places
segment 0 in the least significant position (little-endian, Qiskit order).
"""

from __future__ import annotations

import itertools
from typing import Dict, List, NamedTuple, Sequence, Tuple

import numpy as np

from .gates import H, S, SDG
from .statevector import apply_1q, simulate

S0 = 1.0 / (1.0 + 1.0j)      # weight of the S (x) S term, Eq. (CZ)
S1 = 1.0j / (1.0 + 1.0j)     # weight of the S^dagger (x) S^dagger term, Eq. (CZ)


class Cut(NamedTuple):
    gate_index: int
    kind: str          # "CZ" or "CX"
    qubits: Tuple[int, int]   # (q0, q1) as in the gate (CX: control, target)
    segs: Tuple[int, int]     # segment of q0, segment of q1


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
        if g.kind not in ("CZ", "CX"):
            raise ValueError(f"gate {k} ({g.kind}) crosses a boundary and is not CZ/CX")
        cuts.append(Cut(k, g.kind, (g.q0, g.q1), (sa, sb)))
    return cuts


def adjacent_cuts(cuts: Sequence[Cut], i: int) -> List[int]:
    """Indices of the cuts touching segment i, in gate order (c_i = their count)."""
    return [j for j, c in enumerate(cuts) if i in c.segs]


def n_subcircuits(cuts: Sequence[Cut], n: int) -> int:
    """N_sub = sum_i 2^{c_i} (Sec. III.A with Schmidt rank k = 2)."""
    return sum(2 ** len(adjacent_cuts(cuts, i)) for i in range(n))


def subcircuit(gates: Sequence, sizes: Sequence[int], i: int, cuts: Sequence[Cut],
               bits: Dict[int, int]) -> List[LocalGate]:
    """Algorithm 1: the gate list of segment i for one assignment of its cut bits.

    ``bits`` maps a cut index (into ``cuts``) to 0 (S term) or 1 (S^dagger term).
    Qubits are renumbered to the segment's local register.
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
            phase = S if bits[j] == 0 else SDG
            if c.kind == "CX" and side == 1:          # target of a cut CX: H S H
                out.append(LocalGate("U", local, matrix=H @ phase @ H))
            else:
                out.append(LocalGate("U", local, matrix=phase))
            continue
        if seg[g.q0] != i:
            continue
        if g.q1 >= 0:
            out.append(LocalGate(g.kind, g.q0 - off, g.q1 - off))
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
        else:
            psi = apply_1q(psi, nq, g.q0, one_qubit_matrix(g.kind, g.p0, g.p1))
    return psi


def variant_states(q: int, gates: Sequence, sizes: Sequence[int],
                   cuts: Sequence[Cut] | None = None) -> Dict[Tuple[int, Tuple[int, ...]], np.ndarray]:
    """Algorithm 2: every subcircuit state, keyed by (segment, bits of its adjacent cuts in gate order)."""
    if cuts is None:
        cuts = find_cuts(q, gates, sizes)
    out = {}
    for i, nq in enumerate(sizes):
        adj = adjacent_cuts(cuts, i)
        for b in itertools.product((0, 1), repeat=len(adj)):
            bits = dict(zip(adj, b))
            out[(i, tuple(b))] = simulate_local(nq, subcircuit(gates, sizes, i, cuts, bits))
    return out


def alpha(bits: Sequence[int]) -> complex:
    """alpha_m = product over cuts of s_{b_j}, from Eq. (CZ)."""
    a = 1.0 + 0.0j
    for b in bits:
        a *= S0 if b == 0 else S1
    return a


def merge(sizes: Sequence[int], cuts: Sequence[Cut], states) -> np.ndarray:
    """Algorithm 3: plain sum over all 2^{c_total} global combinations."""
    n = len(sizes)
    adj = [adjacent_cuts(cuts, i) for i in range(n)]
    psi = None
    for m in itertools.product((0, 1), repeat=len(cuts)):
        phi = np.ones(1, dtype=np.complex128)
        for i in range(n):                      # segment 0 ends up least significant
            r = tuple(m[j] for j in adj[i])
            phi = np.kron(states[(i, r)], phi)
        term = alpha(m) * phi
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
    combos = list(itertools.product((0, 1), repeat=len(cuts)))
    for t, x in enumerate(xs):
        local = [(int(x) >> off[i]) & ((1 << sizes[i]) - 1) for i in range(n)]
        acc = 0.0 + 0.0j
        for m in combos:
            term = alpha(m)
            for i in range(n):
                term *= states[(i, tuple(m[j] for j in adj[i]))][local[i]]
            acc += term
        out[t] = acc
    return out


def uncut_simulate(q: int, gates: Sequence) -> np.ndarray:
    """T_orig: the same circuit simulated without cutting."""
    return simulate(q, gates)
