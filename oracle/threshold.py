"""Closed-form cut thresholds of Sec. IV (test infrastructure only).

Equal partitioning into n segments of q/n qubits, c cuts per boundary,
c_total = c (n - 1), Schmidt rank k = 2.

* Eq. (speedup_depth_free): cutting beats the uncut simulation in the
  subcircuit stage when N_sub / n < 2^{q (1 - 1/n)}  (depth cancels).
* Eq. (threshold_n2): n = 2 gives c_total < q / 2.
* Eq. (threshold_nge3): n >= 3 gives
  c_total < q (n-1)^2 / (2n) + (n-1) log2(n / (n-2)) / 2, the second term being
  delta of Table II.
* Eq. (threshold_with_D): with a non-uniform gate distribution
  (N_sub / 2^{q(1-1/n)}) (D_seg / D) < 1; in the worst case D_seg = D the
  threshold drops by 1 cut for n = 2 and by (n-1) log2(n) / 2 for n >= 3.
"""

from __future__ import annotations

import math
from typing import Sequence


def n_sub_from_cuts(cuts_per_boundary: Sequence[int]) -> int:
    """N_sub = sum_i 2^{c_i}; c_i counts the cuts on both boundaries next to segment i."""
    n = len(cuts_per_boundary) + 1
    total = 0
    for i in range(n):
        ci = (cuts_per_boundary[i - 1] if i > 0 else 0) + (cuts_per_boundary[i] if i < n - 1 else 0)
        total += 2 ** ci
    return total


def n_sub_equal(c: int, n: int) -> int:
    """Equal cuts per boundary: edge segments have c_i = c, interior ones 2c (Appendix B)."""
    return n_sub_from_cuts([c] * (n - 1))


def speedup_margin(q: int, n: int, n_sub: int) -> float:
    """log2 of 2^{q(1-1/n)} / (N_sub / n); positive means Eq. (speedup_depth_free) holds."""
    return q * (1.0 - 1.0 / n) - math.log2(n_sub / n)


def speedup_condition(q: int, n: int, n_sub: int) -> bool:
    return n_sub / n < 2.0 ** (q * (1.0 - 1.0 / n))


def speedup_condition_nonuniform(q: int, n: int, n_sub: int, dseg_over_d: float) -> bool:
    """Eq. (threshold_with_D)."""
    return (n_sub / 2.0 ** (q * (1.0 - 1.0 / n))) * dseg_over_d < 1.0


def slope_delta(n: int):
    """Table II: threshold c_total < slope * q + delta."""
    if n == 2:
        return 0.5, 0.0
    if n < 2:
        raise ValueError("n must be at least 2")
    return (n - 1) ** 2 / (2.0 * n), (n - 1) * math.log2(n / (n - 2)) / 2.0


def threshold_ctotal(q: float, n: int) -> float:
    """Eqs. (threshold_n2) and (threshold_nge3): the largest admissible c_total (strict bound)."""
    slope, delta = slope_delta(n)
    return slope * q + delta


def nonuniform_reduction(n: int) -> float:
    """Drop of the c_total threshold in the worst case D_seg = D (Sec. IV.B.2)."""
    if n == 2:
        return 1.0
    return (n - 1) * math.log2(n) / 2.0


def closed_form_choice(q: int, c_total: int, candidates: Sequence[int] = (2, 3, 4)) -> int:
    """Fallback decision: the segment count whose Eq. (speedup_depth_free) margin is largest.

    c_total is split over the n - 1 boundaries as evenly as possible (extra cuts on
    the lower boundaries) and N_sub is counted exactly.  Returns 0 (do not cut)
    when no candidate satisfies the condition.
    """
    best, best_margin = 0, 0.0
    for n in candidates:
        if n > q:
            continue
        base, rem = divmod(c_total, n - 1)
        split = [base + (1 if b < rem else 0) for b in range(n - 1)]
        m = speedup_margin(q, n, n_sub_from_cuts(split))
        if m > best_margin:
            best, best_margin = n, m
    return best
