"""Seeded circuit generators (input data only; no arithmetic of the method).

Two families are produced here.

* ``brickwork``: the random brickwork used for every measured workload.
  Layer l (0-based) applies U = Ry(theta) Rz(phi) to every qubit (Rz acts
  first), then CZ on nearest-neighbour pairs (i, i+1) with i = l mod 2.
  A pair that straddles a segment boundary is removed from that pattern;
  instead boundary b receives exactly ``c_b`` CZ gates, appended at the end of
  layers floor(j * d / c_b), j = 0..c_b-1.  Exactly ``c_b`` two-qubit gates
  therefore cross boundary b, which is what makes the segments separable
  after those gates are cut (the cut count of the paper's problem statement,
  Sec. IV: c cuts per boundary, c_total = c (n - 1)).

* ``staircase``: the paper's own synthetic family (Fig. 1, Sec. V.A.2):
  H on every qubit, then a staircase of CX(i, i+1) with T gates around each
  CX; for two or more cuts the staircase (without the initial H layer) is
  repeated once per cut.  The optional ``tx_layers`` argument appends the
  depth-sweep padding of Fig. 8 (alternating T and X on the top qubit before
  the first staircase and on the bottom qubit after the last).

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014): the 64-bit state advances by
the golden-gamma constant and the output is the two-round xor-shift-multiply
finaliser.  A double in [0, 1) takes the top 53 bits.  Draw order: layer,
then qubit, then theta before phi.

Qubit convention: qubit j is bit j of the amplitude index (little-endian);
segment 0 holds the lowest-index qubits.
"""

from __future__ import annotations

import math
from typing import List, NamedTuple, Optional, Sequence

MASK64 = (1 << 64) - 1
GOLDEN_GAMMA = 0x9E3779B97F4A7C15
TWO_PI = 2.0 * math.pi

# Gate kinds understood by both the oracle and the C-ABI.  Parameters:
#   RX/RY/RZ: p0 = angle.  RYRZ: U = Ry(p0) . Rz(p1)  (Rz applied first).
#   CZ: (q0, q1) symmetric.  CX: q0 = control, q1 = target.
GATE_KINDS = {
    "H": 0, "X": 1, "Y": 2, "Z": 3, "S": 4, "SDG": 5, "T": 6, "TDG": 7,
    "RX": 8, "RY": 9, "RZ": 10, "RYRZ": 11,
    "CZ": 16, "CX": 17,
    "SWAP": 18, "ISWAP": 19, "RXX": 20, "RYY": 21, "RZZ": 22,
}
# Two-qubit kinds; all but CX are symmetric in (q0, q1).
#   SWAP, ISWAP (|01> -> i|10>, |10> -> i|01>), RXX/RYY/RZZ: exp(-i p0 PP / 2).
TWO_QUBIT = ("CZ", "CX", "SWAP", "ISWAP", "RXX", "RYY", "RZZ")


class Gate(NamedTuple):
    kind: str
    q0: int
    q1: int = -1
    p0: float = 0.0
    p1: float = 0.0


class SplitMix64:
    """SplitMix64 counter-based generator (Steele, Lea, Flood 2014)."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next_u64(self) -> int:
        self.state = (self.state + GOLDEN_GAMMA) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform(self) -> float:
        """Double in [0, 1) from the top 53 bits."""
        return (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)


def equal_blocks(q: int, n: int) -> List[int]:
    """Contiguous block sizes floor(q/n), remainder spread over the last blocks."""
    if n < 1 or q < n:
        raise ValueError(f"cannot split {q} qubits into {n} segments")
    base, rem = divmod(q, n)
    return [base + (1 if i >= n - rem else 0) for i in range(n)]


def split_cuts(c_total: int, n: int) -> List[int]:
    """Cuts per boundary: as even as possible, extras on the lower boundaries."""
    nb = n - 1
    if nb == 0:
        if c_total != 0:
            raise ValueError("a single segment has no boundary to cut")
        return []
    base, rem = divmod(c_total, nb)
    return [base + (1 if b < rem else 0) for b in range(nb)]


def boundary_qubits(seg_sizes: Sequence[int]) -> List[int]:
    """First qubit of each segment after the first (boundary b sits below it)."""
    out, acc = [], 0
    for s in seg_sizes[:-1]:
        acc += s
        out.append(acc)
    return out


def _pair_gates(kind: str, a: int, b: int, rng: "SplitMix64") -> List[Gate]:
    """The gates placed on pair (a, b): one gate of ``kind``, or for "CAN" the run
    RXX, RYY, RZZ with three drawn angles (a general two-qubit interaction)."""
    if kind in ("CZ", "CX", "SWAP", "ISWAP"):
        return [Gate(kind, a, b)]
    if kind in ("RXX", "RYY", "RZZ"):
        return [Gate(kind, a, b, TWO_PI * rng.uniform())]
    if kind == "CAN":
        return [Gate(k, a, b, TWO_PI * rng.uniform()) for k in ("RXX", "RYY", "RZZ")]
    raise ValueError(f"unknown pair gate {kind}")


def brickwork(q: int, d: int, n: int, c_total: int, seed: int,
              seg_sizes: Optional[Sequence[int]] = None,
              cuts_per_boundary: Optional[Sequence[int]] = None,
              boundary_gate: str = "CZ", bulk_gate: str = "CZ") -> List[Gate]:
    """Random Ry.Rz + CZ brickwork with exactly c_b two-qubit gates across boundary b.

    ``boundary_gate`` / ``bulk_gate`` replace the CZ on the boundary pairs / on the
    other pairs by another two-qubit kind ("CAN": an RXX, RYY, RZZ run).  Angles of
    those gates are drawn right after the layer's single-qubit angles, pair by pair;
    with the CZ defaults nothing extra is drawn."""
    sizes = list(seg_sizes) if seg_sizes is not None else equal_blocks(q, n)
    if len(sizes) != n or sum(sizes) != q or min(sizes) < 1:
        raise ValueError(f"bad segment sizes {sizes} for q={q}, n={n}")
    cb = list(cuts_per_boundary) if cuts_per_boundary is not None else split_cuts(c_total, n)
    if len(cb) != n - 1 or sum(cb) != c_total:
        raise ValueError(f"bad cuts per boundary {cb} for c_total={c_total}")
    if any(c > d for c in cb):
        raise ValueError("each boundary can take at most one cut per layer (c_b <= d)")
    betas = boundary_qubits(sizes)
    boundary_pairs = {(b - 1, b) for b in betas}
    cut_layers = [sorted({(j * d) // c for j in range(c)}) if c else [] for c in cb]
    rng = SplitMix64(seed)
    gates: List[Gate] = []
    for layer in range(d):
        for j in range(q):
            theta = TWO_PI * rng.uniform()
            phi = TWO_PI * rng.uniform()
            gates.append(Gate("RYRZ", j, -1, theta, phi))
        for i in range(layer % 2, q - 1, 2):
            if (i, i + 1) not in boundary_pairs:
                gates += _pair_gates(bulk_gate, i, i + 1, rng)
        for b, beta in enumerate(betas):
            if layer in cut_layers[b]:
                gates += _pair_gates(boundary_gate, beta - 1, beta, rng)
    return gates


def staircase(q: int, copies: int, tx_layers: int = 0) -> List[Gate]:
    """The paper's Fig. 1 family: H layer, then ``copies`` CX staircases with T gates.

    Each staircase step i applies T on the target qubit i+1, CX(i, i+1), then T
    on both qubits (the very first step also puts a T on qubit 0 before its CX).
    ``tx_layers`` > 0 adds the Fig. 8 depth padding: alternating T, X on qubit 0
    before the first staircase and on qubit q-1 after the last one.
    """
    if q < 2 or copies < 1:
        raise ValueError("staircase needs q >= 2 and at least one copy")
    gates: List[Gate] = [Gate("H", j) for j in range(q)]
    for _ in range(tx_layers):
        gates += [Gate("T", 0), Gate("X", 0)]
    for _ in range(copies):
        for i in range(q - 1):
            if i == 0:
                gates.append(Gate("T", 0))
            gates.append(Gate("T", i + 1))
            gates.append(Gate("CX", i, i + 1))
            gates.append(Gate("T", i))
            gates.append(Gate("T", i + 1))
    for _ in range(tx_layers):
        gates += [Gate("T", q - 1), Gate("X", q - 1)]
    return gates
