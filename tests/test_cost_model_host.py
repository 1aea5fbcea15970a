"""Host-side cost-model entry points against the oracle's closed forms (Sec. IV)."""

import math

import numpy as np
import pytest

from oracle import mlp as omlp, threshold

# the library must be built (build() in __graft_entry__) before these run: a missing
# libccut.so is a failure here, not a skip
from paper_2603_01443_amd import ccut  # noqa: E402


@pytest.mark.parametrize("n", [2, 3, 4, 5, 8])
def test_threshold_matches_oracle(n):
    for q in range(n, 40):
        assert abs(ccut.threshold_ctotal(q, n) - threshold.threshold_ctotal(q, n)) < 1e-12


def test_speedup_margin_matches_oracle():
    for n in (2, 3, 4):
        for q in range(n, 33):
            for c in range(0, 10):
                cb = [c] * (n - 1)
                want = threshold.speedup_margin(q, n, threshold.n_sub_from_cuts(cb))
                assert abs(ccut.speedup_margin(q, n, cb) - want) < 1e-12


def test_features_match_oracle():
    for q, d, n, c in [(16, 10, 2, 0), (24, 20, 3, 4), (32, 40, 4, 8), (20, 20, 1, 0)]:
        assert np.allclose(ccut.cost_features(q, d, n, c), omlp.features(q, d, n, c), atol=1e-6)


def test_closed_form_decision_matches_oracle():
    for q in range(4, 34, 2):
        for c in range(0, 16):
            choice, pred = ccut.decide(q, 20, c)
            assert choice == threshold.closed_form_choice(q, c), (q, c)
            assert math.isnan(pred)


def test_mlp_work_bytes_grows_with_rows():
    assert ccut.mlp_work_bytes(1000, 10) > ccut.mlp_work_bytes(10, 10) > 4 * 4931
