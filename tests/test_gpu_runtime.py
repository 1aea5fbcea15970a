"""Batching, launch configuration, HIP-graph replay and autotuning: every
configuration must give bit-identical results to the default launch path."""

import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from inputs import brickwork  # noqa: E402
from oracle import metrics, statevector  # noqa: E402

from .gpu_util import to_np  # noqa: E402


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_01443_amd import ccut, pipeline
    return ccut, pipeline


def arena_copy(run):
    torch.cuda.synchronize()
    return run.arena[: run.info["state_bytes"]].clone()


@pytest.mark.parametrize("q,n,sizes,cuts", [(20, 2, [10, 10], [6]), (32, 3, [10, 11, 11], [3, 3]),
                                            (30, 2, [15, 15], [2])])
def test_launch_configurations_bit_identical(lib, q, n, sizes, cuts):
    """One launch for all variants vs persistent grids vs one launch per variant (uneven sizes too)."""
    ccut, pipeline = lib
    g = brickwork(q, 6, n, sum(cuts), seed=4, seg_sizes=sizes, cuts_per_boundary=cuts)
    run = pipeline.CutRun(q, g, n, sizes, psi=torch.empty(8, dtype=torch.complex64, device="cuda"))
    run.simulate_subcircuits()
    ref = arena_copy(run)
    for threads, cap, pv in [(1024, 0, False), (512, 64, False), (256, 200, False), (256, 0, True),
                             (1024, 0, True)]:
        ccut.plan_set_launch(run.plan, threads, cap, pv)
        run.arena[: run.info["state_bytes"]].zero_()
        run.simulate_subcircuits()
        assert torch.equal(arena_copy(run), ref), (threads, cap, pv)


def test_graph_replay_matches_direct(lib):
    ccut, pipeline = lib
    q, n = 20, 2
    g = brickwork(q, 10, n, 6, seed=2)
    run = pipeline.CutRun(q, g, n)
    direct = run.run("auto").clone()
    s = torch.cuda.Stream()
    graph = ccut.Graph(run.plan, run.arena, run.psi, "auto", stream=s)
    for rep in range(3):
        run.psi.zero_()
        run.arena.zero_()
        scratch = pipeline.uncut(16, brickwork(16, 4, 2, 1, seed=rep))   # eager work between replays
        torch.cuda.synchronize()
        graph.launch(s)
        s.synchronize()
        assert torch.equal(torch.view_as_real(run.psi), torch.view_as_real(direct)), rep
        del scratch
    graph.free()


def test_graph_rebind_runs_other_plans(lib):
    """One captured graph replays the pipelines of other plans of the same layout (the same
    brickwork family with other angles) after ccut_graph_rebind: each replay's state is
    bit-identical to that plan's direct launches, with eager work and synchronizations
    between replays; a plan of another shape is refused."""
    ccut, pipeline = lib
    q, n, d, c = 20, 2, 10, 6
    runs = {seed: pipeline.CutRun(q, brickwork(q, d, n, c, seed=seed), n) for seed in (2, 3, 4)}
    base = runs[2]
    want = {}
    for seed, r in runs.items():   # direct launches, all in the base run's buffers
        ccut.simulate_subcircuits(r.plan, base.arena, stream=torch.cuda.current_stream())
        ccut.merge_full_state(r.plan, base.arena, base.psi, "auto", stream=torch.cuda.current_stream())
        want[seed] = base.psi.clone()
    assert not torch.equal(want[2], want[3])
    s = torch.cuda.Stream()
    graph = ccut.Graph(base.plan, base.arena, base.psi, "auto", stream=s)
    for rep, seed in enumerate((3, 4, 2, 4)):
        base.psi.zero_()
        scratch = pipeline.uncut(16, brickwork(16, 4, 2, 1, seed=rep))   # eager work between replays
        torch.cuda.synchronize()
        graph.rebind(runs[seed].plan, s)
        graph.launch(s)
        s.synchronize()
        assert torch.equal(torch.view_as_real(base.psi), torch.view_as_real(want[seed])), (rep, seed)
        del scratch
    other = ccut.cut_plan(q, ccut.gate_array(brickwork(q, d, n, c - 2, seed=2)), n)
    with pytest.raises(ccut.CcutError) as e:
        graph.rebind(other, s)
    assert e.value.code == ccut.EINVAL
    graph.free()


def test_autotune_keeps_results_and_caches(lib, tmp_path):
    ccut, pipeline = lib
    q, n = 22, 2
    g = brickwork(q, 10, n, 6, seed=6)
    run = pipeline.CutRun(q, g, n)
    before = run.run("bf16x3").clone()
    best = ccut.autotune(run.plan, run.arena, run.psi, reps=2, stream=torch.cuda.current_stream())
    cfg = ccut.plan_get_launch(run.plan)
    print("autotuned", cfg, f"{best:.3f} ms", flush=True)
    assert best > 0 and cfg["threads"] in (256, 512, 1024)
    after = run.run("bf16x3")
    # the tuned block size and prefix-sharing mode regroup the gates (rounding order),
    # so the state agrees to float32 rounding rather than bit for bit
    diff = (after - before).abs().max().item()
    assert diff < 1e-4 * 2 ** (-q / 2), diff
    path = str(tmp_path / "tune.txt")
    ccut.autotune_save(path)
    assert os.path.getsize(path) > 0
    ccut.autotune_load(path)
    fresh = ccut.cut_plan(q, g, n)                 # same shape: starts from the cached entry
    assert ccut.plan_get_launch(fresh) == {**cfg, "per_variant": 0}
    assert ccut.plan_get_prefix_sharing(fresh) == ccut.plan_get_prefix_sharing(run.plan)
    assert ccut.plan_get_prefix_start(fresh) == ccut.plan_get_prefix_start(run.plan)
    # every saved line must load back: rewrite the entry with other threads and a tree
    # from level 5 (prefix field 6) and check that a fresh plan takes both
    # the cache is process-wide: other tests may have tuned other shapes; this plan's line
    # is the one entry for q = 22
    lines = [ln.split() for ln in open(path) if not ln.startswith("#") and ln.split()[0].split("|")[1] == f"q{q}"]
    assert len(lines) == 1 and len(lines[0]) == 9
    key, fields = lines[0][0], lines[0][1:]
    assert ccut.plan_get_auto_precision(fresh) == ccut.plan_get_auto_precision(run.plan)
    assert int(fields[7]) == ccut.PRECISIONS[ccut.plan_get_auto_precision(run.plan)]
    fields[0] = "256" if fields[0] != "256" else "1024"
    fields[6] = "6"
    fields[7] = str(ccut.PREC_BF16X3 if int(fields[7]) != ccut.PREC_BF16X3 else ccut.PREC_FP16X3)
    edited = str(tmp_path / "edited.txt")
    with open(edited, "w") as f:
        f.write(key + " " + " ".join(fields) + "\n")
    ccut.autotune_load(edited)
    fresh = ccut.cut_plan(q, g, n)
    assert ccut.plan_get_launch(fresh)["threads"] == int(fields[0])
    assert ccut.plan_get_prefix_sharing(fresh) and ccut.plan_get_prefix_start(fresh) == 5
    assert ccut.PRECISIONS[ccut.plan_get_auto_precision(fresh)] == int(fields[7])
    # a line written before the split-arithmetic field existed still loads (fp16x3 then)
    old = str(tmp_path / "old.txt")
    with open(old, "w") as f:
        f.write(key + " " + " ".join(fields[:7]) + "\n")
    ccut.autotune_load(old)
    assert ccut.plan_get_auto_precision(ccut.cut_plan(q, g, n)) == "fp16x3"


@pytest.mark.parametrize("prec,c", [("bf16x3", 6), ("fp16x3", 6), ("bf16", 6), ("fp16x2", 6),
                                    ("fp16x2", 3), ("bf16", 5), ("fp16x2", 7), ("fp16x3", 8), ("bf16x3", 8)])
def test_merge_gemm_variants_bit_identical(lib, prec, c):
    """Store path (direct / LDS transpose), tile height, persistent grids, the
    R-stationary, LDS-staged and column-stationary kernels change only data movement: every
    variant writes the same bits, also at K = 8, 32, 128 and 256 (c = 3, 5, 7, 8: one,
    four, sixteen and thirty-two MFMA steps; from sixteen on the R-stationary strip
    runs the tiled kernel instead)."""
    ccut, pipeline = lib
    q, n = 22, 2
    g = brickwork(q, max(6, c), n, c, seed=12)
    run = pipeline.CutRun(q, g, n)
    run.simulate_subcircuits()
    ref = None
    for variant in range(7):
        for cap in (0, 37, 512):
            ccut.plan_set_merge(run.plan, variant, cap)
            run.psi.zero_()
            out = run.merge(prec).clone()
            if ref is None:
                ref = out
            assert torch.equal(torch.view_as_real(out), torch.view_as_real(ref)), (variant, cap)


@pytest.mark.parametrize("prec", ["fp16x3", "fp16x2"])
def test_merge_gemm_repeatable(lib, prec):
    """Every GEMM variant writes the same bits run after run (a 16-byte epilogue store
    whose first data register a vector write reused one instruction later had made a few
    words differ from run to run in the f16 modes): q = 24, K = 64, four runs each."""
    ccut, pipeline = lib
    q, n, c = 24, 2, 6
    g = brickwork(q, 6, n, c, seed=3)
    run = pipeline.CutRun(q, g, n)
    run.simulate_subcircuits()
    ref = None
    for variant in range(7):
        ccut.plan_set_merge(run.plan, variant, 0)
        for rep in range(4):
            run.psi.zero_()
            out = run.merge(prec).clone()
            if ref is None:
                ref = out
            assert torch.equal(torch.view_as_real(out), torch.view_as_real(ref)), (variant, rep)


@pytest.mark.parametrize("prec", ["fp16x3", "fp16x2", "bf16x3"])
def test_merge_gemm_variants_bit_identical_chain(lib, prec):
    """Three segments (8 + 8 + 8 qubits, 2 + 2 cuts): the chain's first stage is a batch of
    four merges with one weighted factor per batch entry; every GEMM variant writes the same
    bits there and in the final stage, the R-stationary kernel splits its rows over
    several workgroups per strip at these small shapes (the column-stationary kernel
    too), and the LDS-staged kernel runs its persistent grid over the batch."""
    ccut, pipeline = lib
    q, n = 24, 3
    g = brickwork(q, 8, n, 4, seed=5)
    run = pipeline.CutRun(q, g, n)
    run.simulate_subcircuits()
    ref = None
    for variant in range(7):
        ccut.plan_set_merge(run.plan, variant, 0)
        run.psi.zero_()
        out = run.merge(prec).clone()
        if ref is None:
            ref = out
        assert torch.equal(torch.view_as_real(out), torch.view_as_real(ref)), variant


def test_kernel_timing_families_and_mask(lib):
    """Kernel timing: one cut pipeline records its kernel families (one split launch for
    the one GEMM merge stage), the mask restricts timing to the named families, and a
    reset clears the totals."""
    ccut, pipeline = lib
    q, n = 20, 2
    run = pipeline.CutRun(q, brickwork(q, 8, n, 6, seed=4), n)
    run.run("fp16x2")                         # tables staged, clocks up
    torch.cuda.synchronize()
    ccut.profile_reset()
    ccut.profile_mask(None)
    ccut.profile_enable(True)
    try:
        run.simulate_subcircuits()
        run.merge("fp16x2")
        torch.cuda.synchronize()
        prof = ccut.profile_read()
        assert set(prof) == set(ccut.PROFILE_KERNELS)
        assert prof["sim"][0] >= 1 and prof["sim"][1] > 0
        assert prof["split"][0] == 1 and prof["merge_gemm"][0] == 1
        assert prof["merge_f32"][0] == 0 and prof["reduce"][0] == 0
        ccut.profile_reset()
        ccut.profile_mask(["merge_gemm"])
        run.simulate_subcircuits()
        run.merge("fp16x2")
        torch.cuda.synchronize()
        prof = ccut.profile_read()
        assert prof["merge_gemm"][0] == 1 and prof["merge_gemm"][1] > 0
        assert all(v[0] == 0 for k, v in prof.items() if k != "merge_gemm")
        ccut.profile_reset()
        assert all(v == (0, 0.0) for v in ccut.profile_read().values())
    finally:
        ccut.profile_enable(False)
        ccut.profile_mask(None)
