"""GPU parity of Schmidt-rank-4 (and rank-2 Pauli-rotation) cuts, through the C-ABI.

The device path cuts SWAP, iSWAP, RXX, RYY, RZZ and fused rotation runs with the
Pauli form of Eq. (schmidt); the oracle uses its own SVD decomposition.  The two
decompositions differ term by term, so parity is on what is unique: the merged
state (equal to the uncut state, Sec. III) and expectation values.  Tolerances
are those of the CZ tests: float32 merge 1 - F <= 1e-9 and max-abs <=
1e-4 * 2^{-q/2}; automatic (split) merge max-abs <= 1e-2 * 2^{-q/2}.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from inputs import Gate, brickwork, equal_blocks  # noqa: E402
from oracle import cutting, metrics, statevector  # noqa: E402
from oracle.expectation import expval  # noqa: E402

from .gpu_util import to_np  # noqa: E402

KINDS = ["SWAP", "ISWAP", "RXX", "RYY", "RZZ", "CAN"]


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_01443_amd import ccut, pipeline
    return ccut, pipeline


def fp32_tol(q):
    return 1e-4 * 2 ** (-q / 2)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("n,q,c", [(2, 14, 3), (3, 15, 4)])
def test_schmidt_cut_pipeline_matches_oracle(lib, kind, n, q, c):
    ccut, pipeline = lib
    g = brickwork(q, 8, n, c, seed=q + n, boundary_gate=kind)
    sizes = equal_blocks(q, n)
    ref = statevector.simulate(q, g)
    run = pipeline.CutRun(q, g, n, sizes)
    for prefix in (0, 1):
        ccut.plan_set_prefix_sharing(run.plan, prefix)
        psi = to_np(run.run("fp32"))
        err, inf = metrics.max_abs_error(ref, psi), metrics.one_minus_fidelity(ref, psi)
        print(f"{kind} n{n} q{q} prefix {prefix}: K={run.info['n_terms']} max-abs {err:.2e} 1-F {inf:.2e}",
              flush=True)
        assert err < fp32_tol(q) and inf < 1e-9
    psi = to_np(run.run("auto"))
    assert metrics.max_abs_error(ref, psi) < 1e-2 * 2 ** (-q / 2)
    assert metrics.one_minus_fidelity(ref, psi) < 1e-6


@pytest.mark.parametrize("prec", ["fp32", "fp16x3"])
def test_swap_cuts_multipass_sampled(lib, prec):
    """q = 26 (13 + 13, d = 8, three SWAP cuts: 64 variants per segment, K = 64) with
    the states split into two LDS blocks: sampled amplitudes against the oracle's
    plain sum over its own Schmidt terms, and the whole state against the uncut run."""
    ccut, pipeline = lib
    q, n, sizes = 26, 2, [13, 13]
    g = brickwork(q, 8, n, 3, seed=11, boundary_gate="SWAP")
    run = pipeline.CutRun(q, g, n, sizes)
    assert run.info["n_terms"] == 64 and run.info["c_seg"][:2] == [6, 6]
    ccut.plan_set_sim_precision(run.plan, prec)
    psi = run.run("fp32")
    ocuts = cutting.find_cuts(q, g, sizes)
    ostates = cutting.variant_states(q, g, sizes, ocuts)
    rng = np.random.default_rng(5)
    xs = sorted(set(int(x) for x in rng.integers(0, 2 ** q, size=300)) | {0, 2 ** q - 1})
    want = cutting.amplitudes(xs, sizes, ocuts, ostates)
    got = to_np(psi[torch.tensor(xs, device=psi.device)])
    err = np.max(np.abs(got - want))
    ref = pipeline.uncut(q, g)
    st = ccut.norm_fidelity(psi, ref, q, stream=torch.cuda.current_stream())
    print(f"q26 SWAP {prec}: sampled max-abs {err:.2e}; vs uncut 1-F {1 - st['fidelity']:.2e}", flush=True)
    assert err < fp32_tol(q)
    assert 1 - st["fidelity"] < 1e-9 and st["max_abs"] < 2 * fp32_tol(q)


@pytest.mark.parametrize("bulk", ["SWAP", "ISWAP", "RXX", "RYY", "RZZ", "CAN"])
def test_uncut_with_two_qubit_kinds(lib, bulk):
    """The uncut baseline applies the new kinds inside a register (exact CX
    decompositions): against the oracle's dense 4 x 4 application."""
    ccut, pipeline = lib
    for q in (10, 17):
        g = brickwork(q, 6, 1, 0, seed=q, bulk_gate=bulk)
        ref = statevector.simulate(q, g)
        psi = to_np(pipeline.uncut(q, g))
        err = metrics.max_abs_error(ref, psi)
        print(f"uncut {bulk} q{q}: max-abs {err:.2e}", flush=True)
        assert err < fp32_tol(q) and metrics.one_minus_fidelity(ref, psi) < 1e-9


def test_fused_rotation_run_and_mixed_kinds(lib):
    """A general interaction (RXX RYY RZZ run, fused into one rank-4 cut) next to CZ,
    CX and SWAP cuts on the same boundary, three segments."""
    ccut, pipeline = lib
    q, sizes = 12, [4, 4, 4]
    g = [Gate("H", j) for j in range(q)] + [Gate("T", j) for j in range(0, q, 3)]
    g += [Gate("RXX", 3, 4, 0.4), Gate("RYY", 3, 4, 1.3), Gate("RZZ", 4, 3, 2.2), Gate("CZ", 2, 5),
          Gate("RYRZ", 4, -1, 0.9, 0.2), Gate("SWAP", 7, 8), Gate("CX", 8, 7), Gate("ISWAP", 3, 4),
          Gate("RY", 0, -1, 0.3), Gate("RZZ", 7, 8, 0.6), Gate("CX", 1, 2), Gate("SWAP", 6, 9)]
    run = pipeline.CutRun(q, g, 3, sizes)
    cuts = run.plan.cuts()
    assert [cu["n_gates"] for cu in cuts if cu["gate_index"] == 16] == [3]
    ref = statevector.simulate(q, g)
    for prefix in (0, 1):
        ccut.plan_set_prefix_sharing(run.plan, prefix)
        psi = to_np(run.run("fp32"))
        assert metrics.max_abs_error(ref, psi) < fp32_tol(q)


@pytest.mark.parametrize("kind", ["SWAP", "CAN", "RZZ"])
def test_expectations_with_schmidt_cuts(lib, kind):
    """Pauli expectation values from the subcircuits (no merge) with rank-4 cuts:
    against the oracle's full-state definition, TOL 2e-5 as for CZ cuts."""
    ccut, pipeline = lib
    q, n = 14, 3
    g = brickwork(q, 6, n, 4, seed=21, boundary_gate=kind)
    ref = statevector.simulate(q, g)
    run = pipeline.CutRun(q, g, n, psi=torch.empty(8, dtype=torch.complex64, device="cuda"), sim_only=True)
    run.simulate_subcircuits()
    work = torch.empty(max(ccut.expectation_work_bytes(run.plan), 8), dtype=torch.uint8, device="cuda")
    rng = np.random.default_rng(7)
    labels = ["I" * q, "Z" * q, "X" * q] + ["".join(rng.choice(list("IXYZ"), q)) for _ in range(6)]
    for j in (3, 4, 5, 9):
        lab = ["I"] * q
        lab[j] = "Z"
        lab[(j + 1) % q] = "X"
        labels.append("".join(lab))
    for lab in labels:
        v = ccut.expectation_pauli(run.plan, run.arena, lab, work, stream=torch.cuda.current_stream())
        assert abs(v - expval(ref, q, lab)) < 2e-5, lab
