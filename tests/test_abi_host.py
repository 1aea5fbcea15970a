"""Host-side checks of the C-ABI library: it loads, exports what include/ccut.h
declares, and its preprocessing (cut_plan, Algorithm 1) agrees with the
oracle's independent plan.  No GPU call is made here."""

import os
import re

import numpy as np

import pytest

from inputs import Gate, brickwork, equal_blocks, staircase
from oracle import cutting

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# the library must be built (build() in __graft_entry__) before these run: a missing
# libccut.so is a failure here, not a skip
from paper_2603_01443_amd import ccut  # noqa: E402


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"\b(ccut_[a-z0-9_]+)\s*\(", text))
    return names


def test_library_exports_every_declared_symbol():
    import ctypes
    lib = ctypes.CDLL(ccut.library_path())
    names = declared_symbols()
    assert len(names) >= 10
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_version_string():
    assert "gfx950" in ccut.version()


def test_cut_weights_are_eq_cz():
    """Eq. (CZ): s_0 = 1/(1+i), s_1 = i/(1+i)."""
    assert ccut.cut_weight(0) == 1 / (1 + 1j)
    assert ccut.cut_weight(1) == 1j / (1 + 1j)
    with pytest.raises(ccut.CcutError):
        ccut.cut_weight(2)


@pytest.mark.parametrize("q,d,n,c,sizes", [
    (12, 10, 2, 2, None), (24, 20, 2, 6, None), (32, 30, 3, 6, None), (16, 10, 4, 8, None),
    (15, 6, 2, 3, [7, 8]), (10, 4, 2, 0, None), (2, 3, 2, 1, None),
])
def test_plan_matches_oracle_plan(q, d, n, c, sizes):
    g = brickwork(q, d, n, c, seed=1, seg_sizes=sizes)
    sizes = sizes or equal_blocks(q, n)
    plan = ccut.cut_plan(q, g, n, sizes)
    info = plan.info()
    ocuts = cutting.find_cuts(q, g, sizes)
    assert info["seg_size"] == sizes
    assert info["c_total"] == len(ocuts)
    assert info["n_sub"] == cutting.n_subcircuits(ocuts, n)
    assert info["n_terms"] == 2 ** len(ocuts)
    assert info["c_seg"] == [len(cutting.adjacent_cuts(ocuts, i)) for i in range(n)]
    assert sorted(cu["gate_index"] for cu in plan.cuts()) == [oc.gate_index for oc in ocuts]
    assert info["psi_bytes"] == 8 << q
    # arena: segment-major, variant-minor, every state 8 * 2^{q_i} bytes
    for i in range(n):
        assert info["seg_state_offset"][i] % 256 == 0
        if i + 1 < n:
            assert info["seg_state_offset"][i + 1] >= info["seg_state_offset"][i] + (8 << sizes[i]) * 2 ** info["c_seg"][i]
    assert info["arena_bytes"] >= info["state_bytes"]


def test_default_blocks_put_remainder_last():
    g = brickwork(32, 4, 3, 6, seed=0)
    assert ccut.cut_plan(32, g, 3).info()["seg_size"] == [10, 11, 11]


def test_cx_cut_info():
    g = staircase(6, 2)
    plan = ccut.cut_plan(6, g, 2)
    cuts = plan.cuts()
    assert len(cuts) == 2 and all(cu["kind"] == 17 and cu["target_high"] == 1 for cu in cuts)
    assert [cu["bit_low"] for cu in cuts] == [0, 1] and [cu["bit_high"] for cu in cuts] == [0, 1]


def test_variant_bits_boundary_major():
    g = brickwork(12, 10, 3, 4, seed=0)
    cuts = ccut.cut_plan(12, g, 3).cuts()
    lo = [cu for cu in cuts if cu["boundary"] == 0]
    hi = [cu for cu in cuts if cu["boundary"] == 1]
    assert [cu["bit_high"] for cu in lo] == [0, 1]        # segment 1: lower boundary bits first
    assert [cu["bit_low"] for cu in hi] == [2, 3]
    assert [cu["bit_low"] for cu in lo] == [0, 1]         # segment 0 sees only boundary 0


def test_error_codes():
    with pytest.raises(ccut.CcutError) as e:
        ccut.cut_plan(0, [], 1)
    assert e.value.code == ccut.EINVAL
    with pytest.raises(ccut.CcutError) as e:
        ccut.cut_plan(6, [Gate("CZ", 0, 5)], 3)           # joins segments 0 and 2
    assert e.value.code == ccut.EUNCUTTABLE
    with pytest.raises(ccut.CcutError) as e:
        ccut.cut_plan(6, [Gate("H", 6)], 2)
    assert e.value.code == ccut.EINVAL
    with pytest.raises(ccut.CcutError) as e:
        ccut.cut_plan(6, [Gate("H", 0)], 2, [2, 3])
    assert e.value.code == ccut.EINVAL
    with pytest.raises(ccut.CcutError) as e:
        ccut.cut_plan(8, [Gate("CZ", 3, 4)] * 17, 2)     # c_i above the per-segment limit
    assert e.value.code == ccut.EUNSUPPORTED
    assert "limit" in str(e.value) or "max" in str(e.value)


def test_merge_variant_range():
    """Merge GEMM variants 0..6 are accepted and read back; 7 and negative grids are not."""
    plan = ccut.cut_plan(16, brickwork(16, 4, 2, 3, seed=1), 2)
    for v in range(7):
        ccut.plan_set_merge(plan, v, 256)
        assert ccut.plan_get_merge(plan) == {"variant": v, "grid_cap": 256}
    for v, cap in ((7, 0), (-1, 0), (3, -1)):
        with pytest.raises(ccut.CcutError) as e:
            ccut.plan_set_merge(plan, v, cap)
        assert e.value.code == ccut.EINVAL


def test_auto_precision_is_fully_split_by_default():
    """AUTO merges in a fully split arithmetic (fp16x3) unless told otherwise; fp16x2 is
    an explicit opt-in, and only MFMA split arithmetics are accepted."""
    plan = ccut.cut_plan(16, brickwork(16, 4, 2, 3, seed=1), 2)
    assert ccut.plan_get_auto_precision(plan) == "fp16x3"
    assert ccut.resolved_precision(plan, "auto", 8) == "fp16x3"
    assert ccut.resolved_precision(plan, "auto", 4) == "fp32"
    for p in ("bf16x3", "fp16x2", "fp16x3"):
        ccut.plan_set_auto_precision(plan, p)
        assert ccut.plan_get_auto_precision(plan) == p
    for p in ("fp32", "bf16", "auto"):
        with pytest.raises(ccut.CcutError) as e:
            ccut.plan_set_auto_precision(plan, p)
        assert e.value.code == ccut.EINVAL


def test_block_bits_reschedule():
    """The LDS block size reschedules the segment programs: smaller blocks mean
    more passes and launches but the same fused program; the automatic choice
    gives the first launch a workgroup per compute unit (256) when it can."""
    q, n = 28, 2
    g = brickwork(q, 20, n, 6, seed=0)
    plan = ccut.cut_plan(q, g, n)
    assert ccut.plan_get_block_bits(plan) == 13          # 128 variants x 2 blocks = 256 workgroups
    arena0 = plan.info()["arena_bytes"]
    stats = {}
    for bits in (14, 13, 12, 9, 0):
        ccut.plan_set_block_bits(plan, bits)
        stats[bits] = ccut.plan_stats(plan)
        assert plan.info()["arena_bytes"] >= arena0
    assert ccut.plan_get_block_bits(plan) == 13
    assert stats[14]["passes"] == 2 and stats[14]["launches"] == 1 and stats[14]["jobs"] == 128
    assert stats[13]["passes"] > 2 and stats[12]["passes"] >= stats[13]["passes"]
    assert stats[9]["passes"] > stats[12]["passes"]
    for b in (13, 12, 9):
        assert stats[b]["fused_ops"] == stats[14]["fused_ops"]
        assert stats[b]["dense_ops"] == stats[14]["dense_ops"]
        assert stats[b]["jobs"] == 128 * stats[b]["launches"]
    # small segments fit one block at any size: one pass each
    small = ccut.cut_plan(20, brickwork(20, 8, 2, 4, seed=1), 2)
    for bits in (14, 12, 10):
        ccut.plan_set_block_bits(small, bits)
        assert ccut.plan_stats(small)["passes"] == 2
    for bad in (-1, 1, 4, 15):
        with pytest.raises(ccut.CcutError):
            ccut.plan_set_block_bits(plan, bad)
    assert ccut.plan_get_block_bits(plan) == 13


def test_prefix_sharing_tree_shape():
    """Prefix sharing: one launch per tree level (single-pass segments), 2^l jobs per
    segment at level l, final level at the variants; automatic mode by total size."""
    q, n = 20, 2
    g = brickwork(q, 10, n, 4, seed=3)
    plan = ccut.cut_plan(q, g, n)
    assert not ccut.plan_get_prefix_sharing(plan)        # 2 x 16 x 2^10 amplitudes: below the automatic bar
    flat = ccut.plan_stats(plan)
    arena = plan.info()["arena_bytes"]
    ccut.plan_set_prefix_sharing(plan, 1)
    assert ccut.plan_get_prefix_sharing(plan)
    tree = ccut.plan_stats(plan)
    assert plan.info()["arena_bytes"] == arena             # scratch is reserved in both modes
    assert tree["launches"] == 4 + 1 and flat["launches"] == 1
    assert tree["jobs"] == 2 * sum(2 ** l for l in range(5)) and flat["jobs"] == 2 * 16
    assert tree["fused_ops"] == flat["fused_ops"] and tree["dense_ops"] == flat["dense_ops"]
    ccut.plan_set_prefix_sharing(plan, 0)
    assert ccut.plan_stats(plan) == flat
    # tree from level 2: the 4 level-2 states run the program up to slot 2 from |0>
    ccut.plan_set_prefix_sharing(plan, 1)
    ccut.plan_set_prefix_start(plan, 2)
    st2 = ccut.plan_stats(plan)
    assert st2["launches"] == 3 and st2["jobs"] == 2 * (4 + 8 + 16)
    assert st2["fused_ops"] == flat["fused_ops"]
    ccut.plan_set_prefix_start(plan, 4)                   # = c_i: the flat schedule
    assert ccut.plan_stats(plan)["jobs"] == flat["jobs"] and ccut.plan_stats(plan)["launches"] == 1
    ccut.plan_set_prefix_start(plan, 0)
    assert ccut.plan_stats(plan) == tree
    with pytest.raises(ccut.CcutError):
        ccut.plan_set_prefix_start(plan, -1)
    ccut.plan_set_prefix_sharing(plan, 0)
    big = ccut.cut_plan(24, brickwork(24, 20, 2, 12, seed=0), 2)   # 2 x 4096 x 2^12 = 2^25 amplitudes
    assert ccut.plan_get_prefix_sharing(big)
    for bad in (-2, 2):
        with pytest.raises(ccut.CcutError):
            ccut.plan_set_prefix_sharing(plan, bad)


def test_gate_fusion_option():
    """Fusion reschedules the stages but not the work: the same gate applications and
    passes; off by default; only 0 and 1 accepted; the graph layout changes with it."""
    q, n = 20, 2
    plan = ccut.cut_plan(q, brickwork(q, 10, n, 4, seed=3), n)
    ccut.plan_set_block_bits(plan, 12)
    assert not ccut.plan_get_fusion(plan)
    flat_work, flat_stats = ccut.plan_work(plan), ccut.plan_stats(plan)
    ccut.plan_set_fusion(plan, True)
    assert ccut.plan_get_fusion(plan)
    fused_work, fused_stats = ccut.plan_work(plan), ccut.plan_stats(plan)
    for k in ("dense_amp_ops", "diag_amp_ops", "amps_moved", "flat_dense_amp_ops"):
        assert fused_work[k] == flat_work[k], k
    assert fused_stats["passes"] == flat_stats["passes"] and fused_stats["stages"] == flat_stats["stages"]
    assert fused_stats["device_ops"] > flat_stats["device_ops"]   # run headers, split CZ records
    ccut.plan_set_fusion(plan, False)
    assert ccut.plan_stats(plan) == flat_stats
    for bad in (-1, 2):
        with pytest.raises(ccut.CcutError):
            ccut.plan_set_fusion(plan, bad)


def test_expectation_argument_checks():
    """Label and workspace errors come back before anything touches the GPU."""
    plan = ccut.cut_plan(12, brickwork(12, 4, 2, 2, seed=0), 2)
    need = ccut.expectation_work_bytes(plan)
    assert need >= 2 * 4 * 4 * 16        # two segments, 4 x 4 complex128 entries at least
    fake = 1 << 20                         # never dereferenced: every call below fails its checks first
    for label in ("Z" * 11, "Z" * 13, "ZZZZZZZZZZZQ", "zzzzzzzzzzzz"):
        with pytest.raises(ccut.CcutError):
            ccut.expectation_pauli(plan, fake, label, fake, arena_bytes=1 << 30, work_bytes=need)
    with pytest.raises(ccut.CcutError, match="work buffer"):
        ccut.expectation_pauli(plan, fake, "IXYZ" * 3, fake, arena_bytes=1 << 30, work_bytes=need - 1)
    # 13 cuts on the one boundary: a 8192 x 8192 matrix per segment is refused
    big = ccut.cut_plan(16, brickwork(16, 14, 2, 13, seed=0), 2)
    assert big.info()["c_total"] == 13
    with pytest.raises(ccut.CcutError, match="at most 12 cuts"):
        ccut.expectation_pauli(big, fake, "Z" * 16, fake, arena_bytes=1 << 40, work_bytes=1 << 40)


@pytest.mark.parametrize("kind", ["SWAP", "ISWAP", "RXX", "RYY", "RZZ", "CZ", "CX"])
def test_schmidt_cuts_match_oracle_ranks(kind):
    """Each cut takes log2(k) variant bits, k its Schmidt rank from the oracle's SVD
    (Eq. schmidt); N_sub = sum_i prod_j k_j and the term count follow; the term
    weights carry the norm of the decomposition: with Pauli or S factors (Frobenius
    norm sqrt 2) sum 4 |w|^2 equals sum |s|^2 |A|^2 |B|^2 of the oracle's terms
    (4 = |U|_F^2 for the SVD's unit factors)."""
    q, n = 12, 3
    g = brickwork(q, 6, n, 4, seed=2, boundary_gate=kind) if kind != "CX" else staircase(q, 2)
    sizes = equal_blocks(q, n)
    plan = ccut.cut_plan(q, g, n)
    info = plan.info()
    cuts = plan.cuts()
    ocuts = cutting.find_cuts(q, g, sizes)
    by_gate = {oc.gate_index: oc for oc in ocuts}         # plan cuts are boundary-major
    assert sorted(cu["gate_index"] for cu in cuts) == sorted(by_gate)
    ranks = []
    for j, cu in enumerate(cuts):
        terms = cutting.cut_terms(by_gate[cu["gate_index"]])
        ranks.append(len(terms))
        assert 2 ** cu["n_bits"] == len(terms) and cu["n_gates"] == 1
        w = plan.cut_terms(j)
        onorm = sum(abs(s) ** 2 * np.linalg.norm(a) ** 2 * np.linalg.norm(b) ** 2 for s, a, b in terms)
        assert abs(sum(abs(x) ** 2 for x in w) * 4 - onorm) < 1e-12
    assert info["n_sub"] == cutting.n_subcircuits(ocuts, n)
    assert info["n_terms"] == int(np.prod(ranks))
    assert sum(info["c_boundary"][: n - 1]) == sum(cu["n_bits"] for cu in cuts)


def test_pauli_rotation_runs_fuse_into_one_cut():
    """RXX, RYY, RZZ on the same cross-boundary pair with nothing in between on
    either qubit commute: one rank-4 cut (two bits), not three rank-2 cuts; a gate
    on one of the qubits between them keeps the runs apart."""
    q = 8
    run = [Gate("RXX", 3, 4, 0.3), Gate("RYY", 4, 3, 1.2), Gate("RZZ", 3, 4, 2.1)]
    plan = ccut.cut_plan(q, run, 2)
    cuts = plan.cuts()
    assert len(cuts) == 1 and cuts[0]["n_bits"] == 2 and cuts[0]["n_gates"] == 3
    assert plan.info()["n_terms"] == 4
    split = run[:1] + [Gate("H", 3)] + run[1:]
    cuts = ccut.cut_plan(q, split, 2).cuts()
    assert [cu["n_gates"] for cu in cuts] == [1, 2] and [cu["n_bits"] for cu in cuts] == [1, 2]
    # a single rotation alone is rank 2 (one bit), SWAP rank 4 (two bits)
    assert ccut.cut_plan(q, [Gate("RZZ", 3, 4, 0.5)], 2).cuts()[0]["n_bits"] == 1
    assert ccut.cut_plan(q, [Gate("SWAP", 3, 4)], 2).cuts()[0]["n_bits"] == 2


def test_term_count_saturates():
    """Eight segments with 16 cut bits on every other boundary (each segment within its
    16-bit limit) have 2^64 global terms: reported as INT64_MAX, not an overflow."""
    q, sizes = 16, [2] * 8
    g = []
    for b in (0, 2, 4, 6):                 # boundaries between segments b and b + 1
        lo, hi = 2 * b + 1, 2 * b + 2
        g += [Gate("CZ", lo, hi)] * 16
    info = ccut.cut_plan(q, g, 8, sizes).info()
    assert info["c_boundary"][:7] == [16, 0, 16, 0, 16, 0, 16]
    assert info["n_terms"] == 2 ** 63 - 1
