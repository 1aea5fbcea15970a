"""GPU parity of the HIP path against the complex128 oracle, through the C-ABI.

Tolerances for the float32 path (complex64 states, float32 arithmetic): every
fused gate adds a relative rounding error of a few units of 2^-24 to each
amplitude, so after the ~10^2-10^3 gates of these circuits the relative error
of an amplitude is ~1e-6; the merge adds K float32 products of such values.
We require 1 - F <= 1e-9 against the oracle and max-abs <= 1e-4 * 2^{-q/2}
(2^{-q/2} is the size of a typical amplitude).
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from inputs import Gate, brickwork, equal_blocks, staircase  # noqa: E402
from oracle import cutting, metrics, statevector  # noqa: E402

from .gpu_util import oracle_key, to_np  # noqa: E402


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_01443_amd import ccut, pipeline
    return ccut, pipeline


def fp32_tol(q):
    return 1e-4 * 2 ** (-q / 2)


def check_state(ref, got, q, label):
    err = metrics.max_abs_error(ref, got)
    inf = metrics.one_minus_fidelity(ref, got)
    print(f"{label}: max-abs {err:.3e} (tol {fp32_tol(q):.1e}), 1-F {inf:.3e}", flush=True)
    assert err <= fp32_tol(q), label
    assert inf <= 1e-9, label


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_small_config_variants_merge_uncut(lib, seed):
    ccut, pipeline = lib
    q, d, n, c = 12, 10, 2, 2
    g = brickwork(q, d, n, c, seed)
    run = pipeline.CutRun(q, g, n)
    run.simulate_subcircuits()
    torch.cuda.synchronize()
    sizes = [6, 6]
    ocuts = cutting.find_cuts(q, g, sizes)
    ostates = cutting.variant_states(q, g, sizes, ocuts)
    pcuts = run.plan.cuts()
    for i in range(n):
        for r in range(2 ** run.info["c_seg"][i]):
            ref = ostates[oracle_key(pcuts, ocuts, i, r)]
            got = to_np(run.variant_state(i, r))
            assert metrics.max_abs_error(ref, got) < 1e-5 * 2 ** (-6 / 2), (i, r)
    psi = to_np(run.merge("fp32"))
    check_state(cutting.merge(sizes, ocuts, ostates), psi, q, f"C1 seed {seed} cut")
    uncut = to_np(pipeline.uncut(q, g))
    check_state(statevector.simulate(q, g), uncut, q, f"C1 seed {seed} uncut")


@pytest.mark.parametrize("c", [2, 4, 6, 8])
def test_q20_fp32_merge(lib, c):
    ccut, pipeline = lib
    q, d, n = 20, 20, 2
    g = brickwork(q, d, n, c, seed=c)
    run = pipeline.CutRun(q, g, n)
    psi = to_np(run.run("fp32"))
    ref = cutting.cut_simulate(q, g, [10, 10])
    check_state(ref, psi, q, f"q20 c{c} fp32")


def test_q20_uncut_multipass(lib):
    ccut, pipeline = lib
    q = 20
    g = brickwork(q, 12, 2, 3, seed=11)
    got = to_np(pipeline.uncut(q, g))
    check_state(statevector.simulate(q, g), got, q, "q20 uncut")


@pytest.mark.parametrize("q,n,cuts,sizes,d", [
    (12, 3, [2, 2], [4, 4, 4], 8),
    (16, 4, [1, 2, 1], [4, 4, 4, 4], 6),
    (15, 2, [3], [7, 8], 6),
    (13, 3, [1, 2], [4, 4, 5], 5),
    (10, 2, [0], [5, 5], 6),
    (2, 2, [1], [1, 1], 3),
    (9, 1, [], [9], 4),
])
def test_partitions(lib, q, n, cuts, sizes, d):
    ccut, pipeline = lib
    g = brickwork(q, d, n, sum(cuts), seed=q + n, seg_sizes=sizes, cuts_per_boundary=cuts)
    run = pipeline.CutRun(q, g, n, sizes)
    psi = to_np(run.run("fp32"))
    ref = statevector.simulate(q, g)
    check_state(ref, psi, q, f"q{q} n{n} cuts{cuts}")


def _degenerate_cases():
    H, T = "H", "T"
    yield "empty circuit, two segments", 6, [], [3, 3]
    yield "one qubit, one segment", 1, [Gate(H, 0), Gate(T, 0)], [1]
    yield "gates on the first segment only", 9, [Gate(H, 0), Gate("CX", 0, 1), Gate("RY", 2, -1, 0.7)], [3, 3, 3]
    g = [Gate("CZ", 3, 4)] + [Gate(H, j) for j in range(8)] + [Gate("RX", 4, -1, 1.1), Gate("CX", 4, 3)]
    yield "cut gates first and last", 8, g, [4, 4]
    g = [Gate(H, j) for j in range(16)]
    g += [Gate("CZ", 2 * b + 1, 2 * b + 2) for b in range(7)]
    g += [Gate("RYRZ", j, -1, 0.3 * j, 0.2 * j) for j in range(16)]
    g += [Gate("CX", 2 * b + 2, 2 * b + 1) for b in range(7)]
    yield "eight segments of two, two cuts per boundary", 16, g, [2] * 8


@pytest.mark.parametrize("case", list(_degenerate_cases()), ids=lambda c: c[0])
def test_degenerate_circuits(lib, case):
    """Empty and one-qubit circuits, segments without gates, cuts at the ends of the gate
    list and the largest segment count (a seven-stage chain)."""
    ccut, pipeline = lib
    _, q, g, sizes = case
    n = len(sizes)
    ref = statevector.simulate(q, g)
    run = pipeline.CutRun(q, g, n, sizes)
    for prec in ("fp32", "auto"):
        psi = to_np(run.run(prec))
        assert metrics.max_abs_error(ref, psi) < 1e-3 * 2 ** (-q / 2) + 1e-7, prec
        assert metrics.one_minus_fidelity(ref, psi) < 1e-6, prec
    assert metrics.max_abs_error(ref, to_np(pipeline.uncut(q, g))) < 1e-6


@pytest.mark.parametrize("q,n,copies", [(6, 2, 1), (8, 2, 3), (9, 3, 2)])
def test_cx_staircase(lib, q, n, copies):
    ccut, pipeline = lib
    g = staircase(q, copies)
    run = pipeline.CutRun(q, g, n)
    psi = to_np(run.run("fp32"))
    check_state(statevector.simulate(q, g), psi, q, f"staircase q{q} n{n}")
    check_state(statevector.simulate(q, g), to_np(pipeline.uncut(q, g)), q, "staircase uncut")


def test_multipass_subcircuits_q30(lib):
    """15-qubit segments exceed one LDS block: variants run as multi-pass HBM states."""
    ccut, pipeline = lib
    q, d, n, c = 30, 6, 2, 2
    g = brickwork(q, d, n, c, seed=5)
    run = pipeline.CutRun(q, g, n)
    run.simulate_subcircuits()
    torch.cuda.synchronize()
    sizes = [15, 15]
    ocuts = cutting.find_cuts(q, g, sizes)
    ostates = cutting.variant_states(q, g, sizes, ocuts)
    pcuts = run.plan.cuts()
    for i in range(n):
        for r in range(4):
            ref = ostates[oracle_key(pcuts, ocuts, i, r)]
            assert metrics.max_abs_error(ref, to_np(run.variant_state(i, r))) < fp32_tol(15), (i, r)
    psi = run.merge("fp32")
    rng = np.random.default_rng(0)
    xs = sorted(set(int(x) for x in rng.integers(0, 2 ** q, size=300)) | {0, 2 ** q - 1, 2 ** 15, 2 ** 15 - 1})
    want = cutting.amplitudes(xs, sizes, ocuts, ostates)
    got = to_np(psi[torch.tensor(xs, device=psi.device)])
    assert np.max(np.abs(got - want)) < fp32_tol(q)


_Q26 = {}


def _q26_oracle():
    """13 + 13 qubits, c_total = 4, d = 8: 16 variants per segment, oracle states cached."""
    if not _Q26:
        q, d, n, c = 26, 8, 2, 4
        g = brickwork(q, d, n, c, seed=8)
        sizes = [13, 13]
        ocuts = cutting.find_cuts(q, g, sizes)
        _Q26.update(g=g, sizes=sizes, ocuts=ocuts, ostates=cutting.variant_states(q, g, sizes, ocuts))
    return _Q26


@pytest.mark.parametrize("bits", [13, 12, 11, 9, 5])
def test_block_bits_variants_match_oracle(lib, bits):
    """Every LDS block size (one block per state, down to 2^5-amplitude blocks and
    37 HBM passes per variant) gives the oracle's subcircuit states, and
    the merged state agrees with the oracle on sampled amplitudes."""
    ccut, pipeline = lib
    o = _q26_oracle()
    q = 26
    run = pipeline.CutRun(q, o["g"], 2)
    ccut.plan_set_block_bits(run.plan, bits)
    assert ccut.plan_get_block_bits(run.plan) == bits
    assert run.info["arena_bytes"] <= run.plan.info()["arena_bytes"] <= run.arena.numel()
    st = ccut.plan_stats(run.plan)
    print(f"bits {bits}: {st}", flush=True)
    run.simulate_subcircuits()
    torch.cuda.synchronize()
    pcuts = run.plan.cuts()
    for i in range(2):
        for r in range(16):
            ref = o["ostates"][oracle_key(pcuts, o["ocuts"], i, r)]
            assert metrics.max_abs_error(ref, to_np(run.variant_state(i, r))) < fp32_tol(13), (bits, i, r)
    psi = run.merge("fp32")
    rng = np.random.default_rng(bits)
    xs = sorted(set(int(x) for x in rng.integers(0, 2 ** q, size=300)) | {0, 2 ** q - 1, 2 ** 13, 2 ** 13 - 1})
    want = cutting.amplitudes(xs, o["sizes"], o["ocuts"], o["ostates"])
    got = to_np(psi[torch.tensor(xs, device=psi.device)])
    assert np.max(np.abs(got - want)) < fp32_tol(q)


@pytest.mark.parametrize("prec,bits", [("fp32", 13), ("fp16x3", 13), ("fp32", 11), ("fp16x3", 11),
                                       ("fp16x3", 9)])
def test_sim_precisions_match_oracle(lib, prec, bits):
    """Both gate arithmetics of the simulation (float32 vector ALUs, split-float16
    MFMA groups) give the oracle's subcircuit states to the float32 tolerance."""
    ccut, pipeline = lib
    o = _q26_oracle()
    run = pipeline.CutRun(26, o["g"], 2)
    ccut.plan_set_sim_precision(run.plan, prec)
    assert ccut.plan_get_sim_precision(run.plan) == prec
    ccut.plan_set_block_bits(run.plan, bits)
    run.simulate_subcircuits()
    torch.cuda.synchronize()
    pcuts = run.plan.cuts()
    worst = 0.0
    for i in range(2):
        for r in range(16):
            ref = o["ostates"][oracle_key(pcuts, o["ocuts"], i, r)]
            got = to_np(run.variant_state(i, r))
            worst = max(worst, metrics.max_abs_error(ref, got))
            assert metrics.one_minus_fidelity(ref, got) < 1e-9, (prec, bits, i, r)
    print(f"{prec} bits {bits}: worst max-abs {worst:.3e} (tol {fp32_tol(13):.1e})", flush=True)
    assert worst < fp32_tol(13)


@pytest.mark.parametrize("prec,bits,start", [("fp16x3", 13, 0), ("fp32", 13, 0), ("fp16x3", 11, 0), ("fp32", 9, 0),
                                             ("fp16x3", 13, 2), ("fp32", 11, 3), ("fp16x3", 12, 4)])
def test_prefix_sharing_matches_oracle(lib, prec, bits, start):
    """Prefix sharing (a tree over the slots: each chunk of the segment program run once
    per prefix of slot choices, from tree level `start` on) gives the oracle's subcircuit
    states, multi-pass too."""
    ccut, pipeline = lib
    o = _q26_oracle()
    run = pipeline.CutRun(26, o["g"], 2)
    ccut.plan_set_sim_precision(run.plan, prec)
    ccut.plan_set_block_bits(run.plan, bits)
    ccut.plan_set_prefix_sharing(run.plan, 1)
    ccut.plan_set_prefix_start(run.plan, start)
    assert ccut.plan_get_prefix_sharing(run.plan) and ccut.plan_get_prefix_start(run.plan) == start
    run.arena.zero_()
    run.simulate_subcircuits()
    torch.cuda.synchronize()
    pcuts = run.plan.cuts()
    for i in range(2):
        for r in range(16):
            ref = o["ostates"][oracle_key(pcuts, o["ocuts"], i, r)]
            got = to_np(run.variant_state(i, r))
            assert metrics.max_abs_error(ref, got) < fp32_tol(13), (prec, bits, i, r)
            assert metrics.one_minus_fidelity(ref, got) < 1e-9, (prec, bits, i, r)


@pytest.mark.parametrize("fusion", [False, True])
def test_deep_segment_in_one_block_splits_passes(lib, fusion):
    """A deep segment program in blocks that hold the whole segment (q = 28 in 14 + 14,
    d = 60, two cuts, 2^14-amplitude blocks, flat schedule): one pass would need more LDS
    for its op headers and stage heads than the CU has beside the block, so the schedule
    splits it into consecutive passes over the same qubits; the variant states match the
    oracle's, with register-stage fusion off and on."""
    ccut, pipeline = lib
    q, d, n, c = 28, 60, 2, 2
    sizes = [14, 14]
    g = brickwork(q, d, n, c, seed=6)
    ocuts = cutting.find_cuts(q, g, sizes)
    ostates = cutting.variant_states(q, g, sizes, ocuts)
    run = pipeline.CutRun(q, g, n)
    ccut.plan_set_block_bits(run.plan, 14)
    ccut.plan_set_prefix_sharing(run.plan, 0)
    ccut.plan_set_fusion(run.plan, fusion)
    assert ccut.plan_get_block_bits(run.plan) == 14
    assert ccut.plan_stats(run.plan)["passes"] > n      # more than one pass per segment
    need = run.plan.info()["arena_bytes"]
    if need > run.arena.numel():
        run.arena = torch.empty(need, dtype=torch.uint8, device=run.psi.device)
    run.arena.zero_()
    run.simulate_subcircuits()
    torch.cuda.synchronize()
    pcuts = run.plan.cuts()
    for i in range(n):
        for r in range(2 ** c):
            ref = ostates[oracle_key(pcuts, ocuts, i, r)]
            got = to_np(run.variant_state(i, r))
            assert metrics.max_abs_error(ref, got) < fp32_tol(14), (fusion, i, r)
            assert metrics.one_minus_fidelity(ref, got) < 1e-9, (fusion, i, r)


@pytest.mark.parametrize("prec,bits,prefix,start", [("fp16x3", 13, 0, 0), ("fp16x3", 12, 1, 2), ("fp16x3", 11, 1, 0),
                                                     ("fp32", 12, 0, 0), ("fp16x3", 9, 0, 0)])
def test_gate_fusion_matches_oracle(lib, prec, bits, prefix, start):
    """Register-stage gate fusion (one 16x16 matrix per run of gates confined to a stage's
    register qubits, composed on the device per slot choice; CZ pairs outside the register set
    applied at the stage's end) gives the oracle's subcircuit states: MFMA and float32 stages,
    flat and tree schedules, several passes, and blocks below the MFMA minimum."""
    ccut, pipeline = lib
    o = _q26_oracle()
    run = pipeline.CutRun(26, o["g"], 2)
    ccut.plan_set_sim_precision(run.plan, prec)
    ccut.plan_set_block_bits(run.plan, bits)
    ccut.plan_set_prefix_sharing(run.plan, prefix)
    if prefix:
        ccut.plan_set_prefix_start(run.plan, start)
    ccut.plan_set_fusion(run.plan, True)
    assert ccut.plan_get_fusion(run.plan)
    run.arena.zero_()
    run.simulate_subcircuits()
    torch.cuda.synchronize()
    pcuts = run.plan.cuts()
    worst = 0.0
    for i in range(2):
        for r in range(16):
            ref = o["ostates"][oracle_key(pcuts, o["ocuts"], i, r)]
            got = to_np(run.variant_state(i, r))
            worst = max(worst, metrics.max_abs_error(ref, got))
            assert metrics.one_minus_fidelity(ref, got) < 1e-9, (prec, bits, i, r)
    print(f"fused {prec} bits {bits} prefix {prefix}/{start}: worst max-abs {worst:.3e}", flush=True)
    assert worst < fp32_tol(13)


@pytest.mark.parametrize("q,n,c,kind", [(15, 3, 6, "brickwork"), (12, 3, 4, "staircase")])
def test_gate_fusion_full_pipeline(lib, q, n, c, kind):
    """Fused stages through the whole pipeline (three segments, CX cuts with H S H on the
    target side) against the oracle's plain sum."""
    ccut, pipeline = lib
    g = brickwork(q, 12, n, c, seed=q + c) if kind == "brickwork" else staircase(q, c // (n - 1))
    sizes = equal_blocks(q, n)
    run = pipeline.CutRun(q, g, n, sizes)
    ccut.plan_set_fusion(run.plan, True)
    psi = to_np(run.run("fp32"))
    ref = cutting.cut_simulate(q, g, sizes)
    check_state(ref, psi, q, f"fused q{q} n{n} c{c} {kind}")


@pytest.mark.parametrize("q,n,c,kind,start", [(20, 2, 8, "brickwork", 0), (12, 3, 4, "staircase", 0),
                                              (15, 3, 6, "brickwork", 0), (20, 2, 8, "brickwork", 3),
                                              (15, 3, 6, "brickwork", 4)])
def test_prefix_sharing_full_pipeline(lib, q, n, c, kind, start):
    """Tree simulation + merge against the oracle's plain sum, many cuts per segment,
    three segments with interleaved boundary slots (the middle one with more slots
    than the tree start, the outer ones with fewer), and CX cuts (H S H on targets)."""
    ccut, pipeline = lib
    g = brickwork(q, 12, n, c, seed=q + c) if kind == "brickwork" else staircase(q, c // (n - 1))
    sizes = equal_blocks(q, n)
    run = pipeline.CutRun(q, g, n, sizes)
    ccut.plan_set_prefix_sharing(run.plan, 1)
    ccut.plan_set_prefix_start(run.plan, start)
    psi = to_np(run.run("fp32"))
    ref = cutting.cut_simulate(q, g, sizes)
    check_state(ref, psi, q, f"tree q{q} n{n} c{c} {kind}")


def test_bench_config_sampled(lib):
    """The measured workload (q=28, 14+14, d=20, c_total=6): sampled amplitudes vs the oracle,
    unit norm, and the full cut state against the full uncut state on the GPU."""
    ccut, pipeline = lib
    q, d, n, c = 28, 20, 2, 6
    g = brickwork(q, d, n, c, seed=0)
    run = pipeline.CutRun(q, g, n)
    psi = run.run("fp32")
    sizes = [14, 14]
    ocuts = cutting.find_cuts(q, g, sizes)
    ostates = cutting.variant_states(q, g, sizes, ocuts)
    rng = np.random.default_rng(1)
    xs = sorted(set(int(x) for x in rng.integers(0, 2 ** q, size=400)) | {0, 2 ** q - 1})
    want = cutting.amplitudes(xs, sizes, ocuts, ostates)
    got = to_np(psi[torch.tensor(xs, device=psi.device)])
    assert np.max(np.abs(got - want)) < fp32_tol(q)
    ref = pipeline.uncut(q, g)
    stats = ccut.norm_fidelity(psi, ref, q, stream=torch.cuda.current_stream())
    print("q28 cut vs uncut:", stats, flush=True)
    assert abs(stats["norm2"] - 1) < 1e-5
    assert 1 - stats["fidelity"] < 1e-9
    assert stats["max_abs"] < 2 * fp32_tol(q)


def test_q32_three_segment_chain_sampled(lib):
    """The three-segment workload (q=32 in 10/11/11, d=30, 3+3 cuts, 80 variants) merged
    by the chain with the automatic precision: sampled amplitudes vs the oracle's plain
    sum over all 64 terms, and the whole 2^32 state against the uncut simulation."""
    ccut, pipeline = lib
    q, d, n, sizes, cb = 32, 30, 3, [10, 11, 11], [3, 3]
    g = brickwork(q, d, n, 6, seed=0, seg_sizes=sizes, cuts_per_boundary=cb)
    run = pipeline.CutRun(q, g, n, sizes)
    assert run.info["n_sub"] == 80
    psi = run.run("auto")
    ocuts = cutting.find_cuts(q, g, sizes)
    ostates = cutting.variant_states(q, g, sizes, ocuts)
    rng = np.random.default_rng(3)
    xs = sorted(set(int(x) for x in rng.integers(0, 2 ** q, size=300)) | {0, 2 ** q - 1})
    want = cutting.amplitudes(xs, sizes, ocuts, ostates)
    got = to_np(psi[torch.tensor(xs, device=psi.device)])
    err = np.max(np.abs(got - want))
    ref = pipeline.uncut(q, g)
    stats = ccut.norm_fidelity(psi, ref, q, stream=torch.cuda.current_stream())
    del ref
    print(f"q32 n3 chain: sampled max-abs vs oracle {err:.3e}; vs uncut {stats}", flush=True)
    # both stages have K = 8: the automatic precision is fp16x2 (bound below)
    assert err < split_tol(q, "fp16x2")
    assert abs(stats["norm2"] - 1) < 1e-5
    assert 1 - stats["fidelity"] < 1e-6
    assert stats["max_abs"] < split_tol(q, "fp16x2")


def test_norm_fidelity_matches_numpy(lib):
    ccut, pipeline = lib
    q = 16
    rng = np.random.default_rng(3)
    a = (rng.normal(size=2 ** q) + 1j * rng.normal(size=2 ** q)).astype(np.complex64)
    b = (a + 1e-3 * (rng.normal(size=2 ** q) + 1j * rng.normal(size=2 ** q))).astype(np.complex64)
    ta, tb = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    s = ccut.norm_fidelity(ta, tb, q)
    a64, b64 = a.astype(np.complex128), b.astype(np.complex128)
    assert abs(s["norm2"] - np.vdot(a64, a64).real) < 1e-9 * s["norm2"]
    assert abs(s["ref_norm2"] - np.vdot(b64, b64).real) < 1e-9 * s["ref_norm2"]
    assert abs(s["overlap"] - np.vdot(b64, a64)) < 1e-9 * abs(s["overlap"])
    assert s["max_abs"] == pytest.approx(np.max(np.abs(a64 - b64)), rel=1e-12)
    s0 = ccut.norm_fidelity(ta, None, q)
    assert s0["ref_norm2"] == 0 and s0["max_abs"] == pytest.approx(np.max(np.abs(a64)), rel=1e-12)


def test_deterministic_repeat(lib):
    ccut, pipeline = lib
    q = 16
    g = brickwork(q, 10, 2, 4, seed=9)
    run = pipeline.CutRun(q, g, 2)
    a = run.run("fp32").clone()
    b = run.run("fp32").clone()
    assert torch.equal(torch.view_as_real(a), torch.view_as_real(b))


def test_gpu_error_paths(lib):
    ccut, pipeline = lib
    q = 10
    g = brickwork(q, 4, 2, 2, seed=0)
    plan = ccut.cut_plan(q, g, 2)
    info = plan.info()
    small = torch.empty(info["arena_bytes"] - 8, dtype=torch.uint8, device="cuda")
    with pytest.raises(ccut.CcutError) as e:
        ccut.simulate_subcircuits(plan, small)
    assert e.value.code == ccut.ENOSPC
    arena = torch.empty(info["arena_bytes"], dtype=torch.uint8, device="cuda")
    psi = torch.empty(2 ** q - 1, dtype=torch.complex64, device="cuda")
    with pytest.raises(ccut.CcutError) as e:
        ccut.merge_full_state(plan, arena, psi, "fp32")
    assert e.value.code == ccut.ENOSPC
    with pytest.raises(ccut.CcutError) as e:
        ccut.merge_full_state(plan, arena, torch.empty(2 ** q, dtype=torch.complex64, device="cuda"), 7)
    assert e.value.code == ccut.EINVAL


# ------------------------------------------------------------ split-precision MFMA merge
# Splitting a float32 value into hi + lo halves keeps ~16 (bfloat16) or ~22 (float16)
# significant bits; dropping lo.lo leaves a relative error per product of ~2^-16 for
# bfloat16, so an amplitude carries ~1e-5 relative error and 1 - F ~ 1e-9.  The bar is
# the 1 - F <= 1e-6 of the metric and max-abs <= 1e-3 * 2^{-q/2}.  fp16x2 rounds the
# low-qubit factor once to float16 (relative error <= 2^-11, RMS ~2.8e-4): 1 - F ~ 1e-7
# and, over 2^20 amplitudes of up to ~4 * 2^{-q/2}, max-abs ~5e-3 * 2^{-q/2}; its
# max-abs bound is 1e-2 * 2^{-q/2}.

def split_tol(q, prec="bf16x3"):
    return (1e-2 if prec == "fp16x2" else 1e-3) * 2 ** (-q / 2)


@pytest.mark.parametrize("c", [2, 4, 6, 8])
@pytest.mark.parametrize("prec", ["bf16x3", "fp16x3", "fp16x2"])
def test_q20_split_precision_merge(lib, c, prec):
    ccut, pipeline = lib
    q, d, n = 20, 20, 2
    g = brickwork(q, d, n, c, seed=c)
    run = pipeline.CutRun(q, g, n)
    psi = to_np(run.run(prec))
    ref = cutting.cut_simulate(q, g, [10, 10])
    err = metrics.max_abs_error(ref, psi)
    inf = metrics.one_minus_fidelity(ref, psi)
    print(f"q20 c{c} {prec}: max-abs {err:.3e} 1-F {inf:.3e}", flush=True)
    assert inf <= 1e-6 and err <= split_tol(q, prec)


def test_unsplit_bf16_is_the_inaccurate_control(lib):
    ccut, pipeline = lib
    q, d, n, c = 20, 20, 2, 6
    g = brickwork(q, d, n, c, seed=3)
    run = pipeline.CutRun(q, g, n)
    ref = cutting.cut_simulate(q, g, [10, 10])
    inf_plain = metrics.one_minus_fidelity(ref, to_np(run.run("bf16")))
    inf_split = metrics.one_minus_fidelity(ref, to_np(run.run("bf16x3")))
    print(f"unsplit bf16 1-F {inf_plain:.3e}, split {inf_split:.3e}", flush=True)
    assert inf_split * 100 < inf_plain


@pytest.mark.parametrize("q,n,sizes,cuts", [
    (14, 2, [7, 7], [6]),          # exactly one 128 x 256 MFMA tile
    (22, 3, [7, 7, 8], [3, 3]),    # chain: stage 1 batched over the upper boundary
    (17, 2, [7, 10], [3]),         # K = 8: inner dimension padded to one 16-step
    (16, 2, [8, 8], [1]),          # K = 2, padded
])
def test_mfma_shapes(lib, q, n, sizes, cuts):
    ccut, pipeline = lib
    g = brickwork(q, 8, n, sum(cuts), seed=q, seg_sizes=sizes, cuts_per_boundary=cuts)
    run = pipeline.CutRun(q, g, n, sizes)
    ref = statevector.simulate(q, g)
    for prec in ("bf16x3", "fp16x3", "fp16x2"):
        psi = to_np(run.run(prec))
        err, inf = metrics.max_abs_error(ref, psi), metrics.one_minus_fidelity(ref, psi)
        print(f"q{q} {sizes} {prec}: max-abs {err:.3e} 1-F {inf:.3e}", flush=True)
        assert inf <= 1e-6 and err <= split_tol(q, prec), prec


def test_bench_config_split_precision(lib):
    ccut, pipeline = lib
    q, d, n, c = 28, 20, 2, 6
    g = brickwork(q, d, n, c, seed=0)
    run = pipeline.CutRun(q, g, n)
    ref = pipeline.uncut(q, g)
    sizes = [14, 14]
    ocuts = cutting.find_cuts(q, g, sizes)
    ostates = cutting.variant_states(q, g, sizes, ocuts)
    rng = np.random.default_rng(2)
    xs = sorted(set(int(x) for x in rng.integers(0, 2 ** q, size=400)))
    want = cutting.amplitudes(xs, sizes, ocuts, ostates)
    for prec in ("bf16x3", "fp16x3", "fp16x2", "auto"):
        psi = run.run(prec)
        got = to_np(psi[torch.tensor(xs, device=psi.device)])
        st = ccut.norm_fidelity(psi, ref, q)
        print(f"q28 {prec}: sampled max-abs {np.max(np.abs(got - want)):.3e}, 1-F vs uncut "
              f"{1 - st['fidelity']:.3e}", flush=True)
        assert np.max(np.abs(got - want)) < split_tol(q, prec)
        assert 1 - st["fidelity"] <= 1e-6


def test_large_k_split_precision_sampled(lib):
    """The large-K configuration (q = 30, 15 + 15, d = 20, K = 256) at full size: the plan's
    default GEMM there is the LDS-staged variant; 300 sampled amplitudes against the
    oracle's variant states (Alg. 3 term by term) and 1 - F against the uncut state."""
    ccut, pipeline = lib
    q, d, n, c = 30, 20, 2, 8
    g = brickwork(q, d, n, c, seed=0)
    run = pipeline.CutRun(q, g, n)
    assert ccut.plan_get_merge(run.plan)["variant"] == 5
    ref = pipeline.uncut(q, g)
    sizes = [15, 15]
    ocuts = cutting.find_cuts(q, g, sizes)
    ostates = cutting.variant_states(q, g, sizes, ocuts)
    rng = np.random.default_rng(5)
    xs = sorted(set(int(x) for x in rng.integers(0, 2 ** q, size=300)))
    want = cutting.amplitudes(xs, sizes, ocuts, ostates)
    for prec in ("fp16x3", "bf16x3", "fp16x2"):
        psi = run.run(prec)
        got = to_np(psi[torch.tensor(xs, device=psi.device)])
        st = ccut.norm_fidelity(psi, ref, q)
        print(f"q30 K256 {prec}: sampled max-abs {np.max(np.abs(got - want)):.3e}, 1-F vs uncut "
              f"{1 - st['fidelity']:.3e}", flush=True)
        assert np.max(np.abs(got - want)) < split_tol(q, prec)
        assert 1 - st["fidelity"] <= 1e-6


@pytest.mark.parametrize("d", [10, 20])
def test_bench_config_tuned(lib, d):
    """The measured workload in the launch configuration the bench runs: simulation groups
    as split-fp16 MFMA, 2^12-amplitude blocks (several LDS passes per 14-qubit state), the
    prefix tree from level c - 1 = 5, 512-thread workgroups, the column-stationary merge GEMM
    and AUTO = fp16x3; then the configuration the autotuner picks on this device.  Both at
    q = 28 (14 + 14), c_total = 6, seed 0: >= 400 sampled amplitudes against the oracle's
    plain sum at the split-merge bar, 1 - F <= 1e-6 and unit norm against the uncut state."""
    ccut, pipeline = lib
    q, n, c = 28, 2, 6
    sizes = [14, 14]
    g = brickwork(q, d, n, c, seed=0)
    ocuts = cutting.find_cuts(q, g, sizes)
    ostates = cutting.variant_states(q, g, sizes, ocuts)
    rng = np.random.default_rng(28 + d)
    xs = sorted(set(int(x) for x in rng.integers(0, 2 ** q, size=420)) | {0, 2 ** q - 1})
    want = cutting.amplitudes(xs, sizes, ocuts, ostates)
    ref = pipeline.uncut(q, g)
    run = pipeline.CutRun(q, g, n)
    stream = torch.cuda.current_stream()

    def check(label):
        need = run.plan.info()["arena_bytes"]     # other block sizes need other table room
        if need > run.arena.numel():
            run.arena = torch.empty(need, dtype=torch.uint8, device=run.psi.device)
        psi = run.run("auto")
        got = to_np(psi[torch.tensor(xs, device=psi.device)])
        err = np.max(np.abs(got - want))
        st = ccut.norm_fidelity(psi, ref, q, stream=stream)
        print(f"q28 d{d} {label}: sampled max-abs {err:.3e} (bar {split_tol(q):.1e}), 1-F vs uncut "
              f"{1 - st['fidelity']:.3e}, norm drift {abs(st['norm2'] - 1):.2e}", flush=True)
        assert len(xs) >= 400
        assert err <= split_tol(q), label
        assert 1 - st["fidelity"] <= 1e-6, label
        assert abs(st["norm2"] - 1) < 1e-5, label

    ccut.plan_set_sim_precision(run.plan, "fp16x3")
    ccut.plan_set_block_bits(run.plan, 12)
    ccut.plan_set_prefix_sharing(run.plan, 1)
    ccut.plan_set_prefix_start(run.plan, c - 1)
    ccut.plan_set_launch(run.plan, threads=512)
    ccut.plan_set_merge(run.plan, 6, 0)
    assert ccut.plan_get_auto_precision(run.plan) == "fp16x3"
    assert ccut.plan_get_block_bits(run.plan) == 12 and ccut.plan_get_prefix_start(run.plan) == c - 1
    assert ccut.plan_stats(run.plan)["passes"] > 2      # 2^14 states in 2^12 blocks: multi-pass
    check("bench configuration")
    ccut.autotune(run.plan, run.arena, run.psi, reps=2, stream=stream)
    check(f"autotuned {ccut.plan_get_launch(run.plan)} merge {ccut.plan_get_merge(run.plan)} "
          f"{ccut.plan_get_auto_precision(run.plan)}")


def absolute_term_sums(xs, sizes, cuts, states):
    """T[x] = sum over the combinations m of |alpha_m| prod_i |psi_i^(m)[x_i]|: the bound on
    every sum the merge forms for amplitude x, before cancellation."""
    n = len(sizes)
    off = cutting.segment_offsets(sizes)
    adj = [cutting.adjacent_cuts(cuts, i) for i in range(n)]
    combos = list(cutting.combinations(cuts))
    weights = [abs(cutting.alpha(m, cuts)) for m in combos]
    out = np.zeros(len(xs))
    for t, x in enumerate(xs):
        local = [(int(x) >> off[i]) & ((1 << sizes[i]) - 1) for i in range(n)]
        for m, w in zip(combos, weights):
            term = w
            for i in range(n):
                term *= abs(states[(i, tuple(m[j] for j in adj[i]))][local[i]])
            out[t] += term
    return out


@pytest.mark.parametrize("d", [10, 40])
def test_fp16x2_error_follows_the_term_sum(lib, d):
    """fp16x2 rounds each weighted low-segment value once to float16 (relative error at
    most 2^-11) and keeps the high-segment values to ~2^-22, so the error of amplitude x
    is at most 2^-11 T[x] plus float32 accumulation; the bar 2^-10 T[x] + 1e-4 2^{-q/2}
    also holds for shallow circuits, whose amplitudes are far from uniform in size (the
    bound 1e-2 2^{-q/2} assumes scrambled states and is not used here)."""
    ccut, pipeline = lib
    q, n, c = 28, 2, 6
    sizes = [14, 14]
    g = brickwork(q, d, n, c, seed=1)
    run = pipeline.CutRun(q, g, n)
    psi = run.run("fp16x2")
    ocuts = cutting.find_cuts(q, g, sizes)
    ostates = cutting.variant_states(q, g, sizes, ocuts)
    rng = np.random.default_rng(d)
    xs = sorted(set(int(x) for x in rng.integers(0, 2 ** q, size=400)))
    want = cutting.amplitudes(xs, sizes, ocuts, ostates)
    tsum = absolute_term_sums(xs, sizes, ocuts, ostates)
    got = to_np(psi[torch.tensor(xs, device=psi.device)])
    err = np.abs(got - want)
    ratio = np.max(err / (2.0 ** -10 * tsum + 1e-4 * 2 ** (-q / 2)))
    ref = pipeline.uncut(q, g)
    st = ccut.norm_fidelity(psi, ref, q)
    print(f"q28 d{d} fp16x2: sampled max-abs {err.max():.3e}, max err / bar {ratio:.3f}, "
          f"max |amp| / 2^(-q/2) {np.max(np.abs(want)) * 2 ** (q / 2):.1f}, "
          f"1-F vs uncut {1 - st['fidelity']:.3e}", flush=True)
    assert ratio <= 1.0
    assert 1 - st["fidelity"] <= 1e-6


def test_library_generator_feeds_the_pipeline(lib):
    """Gates from the library's own generator (ccut_brickwork) run through the cut
    pipeline and give the oracle's state."""
    ccut, pipeline = lib
    q, d, n, c = 16, 8, 2, 4
    g = ccut.brickwork_gates(q, d, n, c, 9)
    psi = to_np(pipeline.CutRun(q, g, n).run("fp32"))
    ref = statevector.simulate(q, brickwork(q, d, n, c, 9))
    assert metrics.max_abs_error(ref, psi) <= 1e-4 * 2 ** (-q / 2)


def test_q34_indices_beyond_32_bits(lib):
    """q = 34 (17 + 17, 128 GiB output): amplitude indices above 2^32 in the merge's
    tiles, the split operands and the reductions.  Sampled amplitudes (the highest
    indices included) against the oracle's plain sum, and the FP64 norm of the whole
    state."""
    ccut, pipeline = lib
    if torch.cuda.get_device_properties(0).total_memory < (200 << 30):
        pytest.skip("needs a device with more than 200 GiB")
    torch.cuda.empty_cache()                  # blocks cached by earlier tests
    q, d, n, c = 34, 6, 2, 4
    sizes = [17, 17]
    g = brickwork(q, d, n, c, seed=5)
    run = pipeline.CutRun(q, g, n)
    psi = run.run("auto")                     # K = 16: the fp16x2 GEMM
    stats = ccut.norm_fidelity(psi, None, q, stream=torch.cuda.current_stream())
    ocuts = cutting.find_cuts(q, g, sizes)
    ostates = cutting.variant_states(q, g, sizes, ocuts)
    rng = np.random.default_rng(34)
    top = 2 ** q - 1
    xs = sorted(set(int(x) for x in rng.integers(0, 2 ** q, size=200))
                | {0, 2 ** 32 - 1, 2 ** 32, 2 ** 33 + 12345, top - 1, top})
    want = cutting.amplitudes(xs, sizes, ocuts, ostates)
    tsum = absolute_term_sums(xs, sizes, ocuts, ostates)
    got = to_np(psi[torch.tensor(xs, device=psi.device)])
    ratio = np.max(np.abs(got - want) / (2.0 ** -10 * tsum + 1e-4 * 2 ** (-q / 2)))
    print(f"q34: sampled err / bar {ratio:.3f}, norm drift {abs(stats['norm2'] - 1):.2e}", flush=True)
    del psi, run
    torch.cuda.empty_cache()
    assert ratio <= 1.0
    assert abs(stats["norm2"] - 1) < 1e-5
