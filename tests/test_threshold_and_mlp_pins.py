"""Pins of the closed-form thresholds (Table II) and of the float64 MLP reference."""

import math
import os

import numpy as np
import pytest

from inputs.mlp_init import glorot_params
from oracle import mlp, threshold

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def table2():
    rows = []
    for line in open(os.path.join(GOLDEN, "table2_thresholds.txt")):
        if line.strip() and not line.startswith("#"):
            n, sn, sd, delta, red = line.split()
            rows.append((int(n), int(sn) / int(sd), float(delta), float(red)))
    return rows


def test_table2_slopes_and_deltas():
    for n, slope, delta, red in table2():
        s, dl = threshold.slope_delta(n)
        assert abs(s - slope) < 1e-12
        assert abs(dl - delta) < 0.005                 # the table prints 1.58 for log2 3
        assert round(threshold.nonuniform_reduction(n), 1) == red


def test_delta_close_to_one_and_a_half():
    """Sec. IV.B.1: delta stays near 1.5 for n up to about 10, tending to 1/ln 2."""
    for n in range(3, 11):
        assert 1.44 <= threshold.slope_delta(n)[1] <= math.log2(3) + 1e-12
    assert abs(threshold.slope_delta(10 ** 6)[1] - 1 / math.log(2)) < 1e-3


def test_n2_threshold_is_the_exact_condition():
    """For n = 2, N_sub = 2 * 2^c and Eq. (speedup_depth_free) is exactly c_total < q/2."""
    for q in range(2, 40):
        for c in range(0, 30):
            exact = threshold.speedup_condition(q, 2, threshold.n_sub_equal(c, 2))
            assert exact == (c < q / 2)


def test_nge3_threshold_tracks_exact_condition():
    """Eq. (threshold_nge3) drops the edge-segment terms; its bound stays within one cut."""
    for n in (3, 4, 5):
        for q in range(3 * n, 40, n):
            bound = threshold.threshold_ctotal(q, n)
            ok = [c * (n - 1) for c in range(0, 30)
                  if threshold.speedup_condition(q, n, threshold.n_sub_equal(c, n))]
            largest = max(ok) if ok else -1
            assert largest < bound + 1e-9
            assert largest >= bound - (n - 1) - 1


def test_nsub_interior_edges():
    assert threshold.n_sub_equal(3, 2) == 16
    assert threshold.n_sub_equal(3, 3) == 8 + 64 + 8
    assert threshold.n_sub_from_cuts([3, 3, 2]) == 8 + 64 + 32 + 4


def test_closed_form_choice():
    assert threshold.closed_form_choice(24, 30) == 0       # far past every threshold
    assert threshold.closed_form_choice(24, 2) in (2, 3, 4)
    assert threshold.closed_form_choice(24, 11, candidates=(2,)) == 2
    assert threshold.closed_form_choice(24, 12, candidates=(2,)) == 0


# ---------------------------------------------------------------- MLP reference

def test_features_hand_worked():
    """q = 24, d = 20, n = 3, c_total = 4: cuts (2, 2), c_i = (2, 4, 2), N_sub = 4 + 16 + 4 = 24,
    q_max = 8, merge work 2^4 2^24.  Uncut q = 20, d = 10: N_sub = 1, q_max = 20."""
    l24, l20, l10 = math.log2(24), math.log2(20), math.log2(10)
    want = [0.0, 0.0, 0.0, 0.0, (l24 - 6) / 4, (8 - 12) / 4, (l24 + 8 + l20 - 24) / 6, (4 + 24 - 30) / 6]
    assert np.allclose(mlp.features(24, 20, 3, 4), want, atol=1e-12)
    want = [-0.5, l10 - l20, -2.0, -1.0, -1.5, 2.0, (20 + l10 - 24) / 6, -10 / 6]
    assert np.allclose(mlp.features(20, 10, 1, 0), want, atol=1e-12)
    # n = 2, c_total = 5: both segments see all 5 cuts; q = 17 gives blocks 8 + 9, q_max = 9
    assert np.isclose(mlp.features(17, 20, 2, 5)[4], (6 - 6) / 4)
    assert np.isclose(mlp.features(17, 20, 2, 5)[5], (9 - 12) / 4)


def test_mlp_gradient_matches_finite_differences():
    flat = glorot_params(5)
    rng = np.random.default_rng(1)
    x = rng.normal(size=(17, mlp.N_IN))
    t = rng.normal(size=(17, 3))
    y, cache = mlp.forward(flat, x)
    g = mlp.backward(flat, cache, y, t)
    idx = list(range(0, mlp.N_PARAMS, 97)) + [mlp.N_PARAMS - 1, mlp.N_PARAMS - 3, 256, 320]
    h = 1e-6
    for i in idx:
        e = np.zeros_like(flat)
        e[i] = h
        num = (mlp.loss(mlp.forward(flat + e, x)[0], t) - mlp.loss(mlp.forward(flat - e, x)[0], t)) / (2 * h)
        assert abs(num - g[i]) < 1e-8 * max(1.0, abs(num)), i


def test_mlp_layout_and_adam_first_step():
    assert mlp.N_PARAMS == 4931
    flat = glorot_params(0)
    assert flat.shape == (4931,)
    g = np.linspace(-1, 1, 4931)
    g[g == 0] = 0.5
    new, m, v = mlp.adam_step(flat, g, np.zeros(4931), np.zeros(4931), 1, 1e-3)
    # bias-corrected first step moves every weight by lr * sign(g) (up to eps)
    assert np.max(np.abs((flat - new) - 1e-3 * np.sign(g))) < 1e-3 * 1e-4


def test_mlp_training_reduces_loss():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(64, mlp.N_IN))
    t = np.stack([x[:, 0] + 0.5 * x[:, 1], np.sin(x[:, 2]), x[:, 3] ** 2], axis=1)
    _, hist = mlp.train(glorot_params(3), x, t, epochs=300, lr=1e-2)
    assert hist[-1] < 0.2 * hist[0]


def test_closed_form_choice_takes_the_largest_margin():
    """Fallback rule: among admissible n, the largest Eq. (speedup_depth_free) margin.

    Worked by hand at q = 24, c_total = 4 (cuts split evenly, extras low):
      n = 2: cuts [4], N_sub = 2^4 + 2^4 = 32, margin 24/2 - log2(32/2) = 8;
      n = 3: cuts [2, 2], N_sub = 4 + 16 + 4 = 24, margin 16 - log2(24/3) = 13;
      n = 4: cuts [2, 1, 1], N_sub = 4 + 8 + 4 + 2 = 18, margin 18 - log2(18/4) = 15.83.
    All three are admissible and distinct, so the order in which candidates are
    listed must not matter: the answer is the n with margin 15.83, or 13 when n = 4
    is not offered.
    """
    assert threshold.speedup_margin(24, 2, 32) == 8.0
    assert threshold.speedup_margin(24, 3, 24) == 13.0
    assert abs(threshold.speedup_margin(24, 4, 18) - (18 - math.log2(4.5))) < 1e-12
    assert threshold.n_sub_from_cuts([2, 1, 1]) == 18
    assert threshold.closed_form_choice(24, 4, (2, 3, 4)) == 4
    assert threshold.closed_form_choice(24, 4, (4, 3, 2)) == 4
    assert threshold.closed_form_choice(24, 4, (2, 3)) == 3
    assert threshold.closed_form_choice(24, 4, (3, 2)) == 3
    assert threshold.closed_form_choice(24, 4, (2,)) == 2


def test_closed_form_choice_strict_condition():
    """Eq. (speedup_depth_free) is strict: a zero margin is not a speedup.

    q = 8, n = 2, c_total = 4: N_sub/2 = 16 = 2^{8/2}, margin exactly 0, so no cut;
    c_total = 3 gives margin 1 and cuts.  A c_total far above every threshold
    (q = 10, c_total = 40) leaves no admissible n at all.
    """
    assert threshold.speedup_margin(8, 2, threshold.n_sub_equal(4, 2)) == 0.0
    assert threshold.closed_form_choice(8, 4, (2,)) == 0
    assert threshold.closed_form_choice(8, 3, (2,)) == 2
    assert threshold.closed_form_choice(10, 40) == 0
