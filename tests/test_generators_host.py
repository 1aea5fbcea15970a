"""The library's seeded generators (ccut_brickwork, ccut_staircase) against the
Python generators of `inputs/`: two independent implementations of one recipe
(SplitMix64 angles, the brickwork layout of the problem statement of Sec. IV,
the staircase of Fig. 1) must give the same ccut_gate_t bytes.  Host-only."""
import ctypes

import numpy as np
import pytest

from inputs import brickwork, staircase

# the library must be built (build() in __graft_entry__) before these run: a missing
# libccut.so is a failure here, not a skip
from paper_2603_01443_amd import ccut  # noqa: E402


@pytest.mark.parametrize("q,d,n,c,seed,sizes,cuts", [
    (12, 10, 2, 2, 0, None, None),           # the small parity configuration
    (28, 20, 2, 6, 0, None, None),           # the bench workload
    (28, 20, 2, 6, 1, None, None),
    (32, 30, 3, 6, 2, [10, 11, 11], None),   # three segments, uneven sizes
    (17, 9, 4, 8, 7, None, [3, 3, 2]),       # extras on the lower boundaries
    (16, 4, 2, 0, 3, None, None),            # no cuts
    (9, 0, 3, 0, 5, None, None),             # no layers
    (24, 12, 2, 12, 2**63 + 5, None, None),  # c_b = d, seed above 2^63
])
def test_brickwork_matches_python_generator(q, d, n, c, seed, sizes, cuts):
    want = ccut.gate_array(brickwork(q, d, n, c, seed, seg_sizes=sizes, cuts_per_boundary=cuts))
    got = ccut.brickwork_gates(q, d, n, c, seed, seg_sizes=sizes, cuts_per_boundary=cuts)
    assert got.dtype == want.dtype and len(got) == len(want)
    assert got.tobytes() == want.tobytes()


def test_brickwork_cut_count_and_angles():
    """Exactly c_b CZs cross each boundary; every angle lies in [0, 2 pi)."""
    q, d, sizes, cuts = 20, 12, [6, 7, 7], [5, 4]
    g = ccut.brickwork_gates(q, d, 3, 9, 11, seg_sizes=sizes, cuts_per_boundary=cuts)
    cz = g[g["kind"] == 16]
    for b, beta in enumerate((6, 13)):
        assert int(np.sum((cz["q0"] == beta - 1) & (cz["q1"] == beta))) == cuts[b]
    rot = g[g["kind"] == 11]
    assert len(rot) == q * d
    assert np.all((rot["p0"] >= 0) & (rot["p0"] < 2 * np.pi) & (rot["p1"] >= 0) & (rot["p1"] < 2 * np.pi))


@pytest.mark.parametrize("q,copies,tx", [(2, 1, 0), (5, 2, 3), (12, 4, 0), (8, 1, 10)])
def test_staircase_matches_python_generator(q, copies, tx):
    want = ccut.gate_array(staircase(q, copies, tx))
    got = ccut.staircase_gates(q, copies, tx)
    assert got.tobytes() == want.tobytes()


def test_generator_errors():
    n = ctypes.c_int64(0)
    with pytest.raises(ccut.CcutError) as e:
        ccut.brickwork_gates(12, 3, 2, 4, 0)                 # c_b = 4 > d = 3
    assert e.value.code == ccut.EINVAL
    with pytest.raises(ccut.CcutError) as e:
        ccut.brickwork_gates(12, 3, 2, 2, 0, seg_sizes=[5, 6])
    assert e.value.code == ccut.EINVAL
    with pytest.raises(ccut.CcutError) as e:
        ccut.brickwork_gates(12, 3, 3, 2, 0, cuts_per_boundary=[2, 1])
    assert e.value.code == ccut.EINVAL
    with pytest.raises(ccut.CcutError) as e:
        ccut.staircase_gates(1, 1)
    assert e.value.code == ccut.EINVAL
    # an exact fit, then a buffer too small: ENOSPC, and the count needed comes back
    buf = np.zeros(3, dtype=ccut.GATE_DTYPE)
    rc = ccut._lib.ccut_brickwork(2, 1, 1, 0, None, None, 0, buf.ctypes.data, len(buf), ctypes.byref(n))
    assert rc == 0 and n.value == 3                       # 2 rotations and CZ(0, 1) on layer 0
    rc = ccut._lib.ccut_brickwork(4, 2, 1, 0, None, None, 0, buf.ctypes.data, len(buf), ctypes.byref(n))
    assert rc == ccut.ENOSPC and n.value == len(ccut.brickwork_gates(4, 2, 1, 0, 0))


def test_gate_array_keeps_packed_input():
    """A ccut_gate_t array passes through gate_array unchanged (no field shift)."""
    g = ccut.brickwork_gates(10, 4, 2, 2, 3)
    again = ccut.gate_array(g)
    assert again.tobytes() == g.tobytes() and again is not g
