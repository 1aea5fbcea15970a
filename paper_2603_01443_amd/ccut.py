"""ctypes binding of libccut.so (argument marshalling only).

Every function here has the name of a C entry point of include/ccut.h
without its ``ccut_`` prefix and forwards to it unchanged: all computation
happens in the HIP library.  Device buffers are passed as integer addresses
(``tensor.data_ptr()``) with their byte sizes, or as objects exposing
``data_ptr()`` / ``numel()`` / ``element_size()`` (PyTorch tensors); streams as
integer ``hipStream_t`` handles (``torch.cuda.current_stream().cuda_stream``)
or None for the default stream.

The library must have been built in-tree (``__graft_entry__.build()``);
importing this module without it raises ImportError.
"""

from __future__ import annotations

import ctypes
import os
from typing import Iterable, List, Optional, Sequence

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libccut.so")

MAX_SEG = 8

OK, EINVAL, EUNCUTTABLE, ENOSPC, ENOMEM, EHIP, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6

PREC_AUTO, PREC_FP32, PREC_BF16X3, PREC_FP16X3, PREC_BF16, PREC_FP16X2 = -1, 0, 1, 2, 3, 4
PRECISIONS = {"auto": PREC_AUTO, "fp32": PREC_FP32, "bf16x3": PREC_BF16X3, "fp16x3": PREC_FP16X3,
              "bf16": PREC_BF16, "fp16x2": PREC_FP16X2}

GATE_KIND = {
    "H": 0, "X": 1, "Y": 2, "Z": 3, "S": 4, "SDG": 5, "T": 6, "TDG": 7,
    "RX": 8, "RY": 9, "RZ": 10, "RYRZ": 11, "CZ": 16, "CX": 17,
    "SWAP": 18, "ISWAP": 19, "RXX": 20, "RYY": 21, "RZZ": 22,
}

GATE_DTYPE = np.dtype([("kind", "<i4"), ("q0", "<i4"), ("q1", "<i4"), ("reserved", "<i4"),
                       ("p0", "<f8"), ("p1", "<f8")])


class CcutError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ccut error {code}: {msg}")
        self.code = code


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("q", ctypes.c_int32), ("n_seg", ctypes.c_int32), ("c_total", ctypes.c_int32),
        ("n_gates", ctypes.c_int32),
        ("seg_size", ctypes.c_int32 * MAX_SEG), ("seg_offset", ctypes.c_int32 * MAX_SEG),
        ("c_seg", ctypes.c_int32 * MAX_SEG), ("c_boundary", ctypes.c_int32 * MAX_SEG),
        ("n_sub", ctypes.c_int64), ("n_terms", ctypes.c_int64),
        ("seg_state_offset", ctypes.c_uint64 * MAX_SEG),
        ("state_bytes", ctypes.c_uint64), ("arena_bytes", ctypes.c_uint64), ("psi_bytes", ctypes.c_uint64),
        ("sim_arena_bytes", ctypes.c_uint64),
    ]


class CutInfo(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int32) for name in
                ("gate_index", "kind", "boundary", "q_low", "q_high", "target_high", "bit_low", "bit_high",
                 "n_bits", "n_gates")]


def _load():
    # PyTorch-ROCm ships its own libamdhip64.so.7.  Loading torch first makes this
    # library bind to that same runtime, so the process holds one HIP runtime
    # whichever module the caller imports first.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")
    lib = ctypes.CDLL(_LIB_PATH)
    vp, u64, i32, i64 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64
    sig = {
        "ccut_cut_plan": [i32, vp, i64, i32, vp, ctypes.POINTER(vp)],
        "ccut_plan_info": [vp, ctypes.POINTER(PlanInfo)],
        "ccut_plan_cut": [vp, i32, ctypes.POINTER(CutInfo)],
        "ccut_cut_weight": [i32, ctypes.POINTER(ctypes.c_double)],
        "ccut_plan_cut_terms": [vp, i32, ctypes.POINTER(ctypes.c_double)],
        "ccut_plan_prepare": [vp],
        "ccut_simulate_subcircuits": [vp, vp, u64, vp],
        "ccut_merge_full_state": [vp, vp, u64, vp, u64, i32, vp],
        "ccut_simulate_uncut": [i32, vp, i64, vp, u64, vp],
        "ccut_norm_fidelity": [vp, vp, i32, ctypes.POINTER(ctypes.c_double), vp],
        "ccut_norm_fidelity_noalloc": [vp, vp, i32, vp, vp],
        "ccut_expectation_work_bytes": [vp, ctypes.POINTER(u64)],
        "ccut_expectation_pauli": [vp, vp, u64, ctypes.c_char_p, vp, u64, ctypes.POINTER(ctypes.c_double), vp],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    fp, dp = ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_double)
    more = {
        "ccut_threshold_ctotal": [i32, i32, dp],
        "ccut_speedup_margin": [i32, i32, vp, dp],
        "ccut_cost_features": [i32, i32, i32, i32, fp],
        "ccut_mlp_work_bytes": [i64, i32, ctypes.POINTER(u64)],
        "ccut_mlp_predict": [vp, vp, i64, vp, vp],
        "ccut_mlp_grad": [vp, vp, vp, i64, vp, u64, vp, fp, vp],
        "ccut_mlp_train": [vp, vp, vp, i64, i32, ctypes.c_float, vp, u64, fp, vp],
        "ccut_decide": [i32, i32, i32, vp, ctypes.c_double, ctypes.c_double, ctypes.POINTER(i32), dp, vp],
        "ccut_brickwork": [i32, i32, i32, i32, vp, vp, u64, vp, i64, ctypes.POINTER(i64)],
        "ccut_staircase": [i32, i32, i32, vp, i64, ctypes.POINTER(i64)],
    }
    for name, args in more.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    for name, args in {
        "ccut_plan_set_launch": [vp, i32, i32, i32, i32],
        "ccut_plan_get_launch": [vp, ctypes.POINTER(i32)],
        "ccut_plan_set_merge": [vp, i32, i32],
        "ccut_plan_get_merge": [vp, ctypes.POINTER(i32)],
        "ccut_plan_set_auto_precision": [vp, i32],
        "ccut_plan_get_auto_precision": [vp, ctypes.POINTER(i32)],
        "ccut_plan_set_block_bits": [vp, i32],
        "ccut_plan_set_sim_precision": [vp, i32],
        "ccut_plan_set_prefix_sharing": [vp, i32],
        "ccut_plan_set_prefix_start": [vp, i32],
        "ccut_plan_get_prefix_start": [vp, ctypes.POINTER(i32)],
        "ccut_plan_get_prefix_sharing": [vp, ctypes.POINTER(i32)],
        "ccut_plan_set_fusion": [vp, i32],
        "ccut_plan_get_fusion": [vp, ctypes.POINTER(i32)],
        "ccut_plan_get_sim_precision": [vp, ctypes.POINTER(i32)],
        "ccut_plan_get_block_bits": [vp, ctypes.POINTER(i32)],
        "ccut_plan_stats": [vp, ctypes.POINTER(i64)],
        "ccut_plan_work": [vp, ctypes.POINTER(ctypes.c_double)],
        "ccut_autotune": [vp, vp, u64, vp, u64, i32, vp, dp],
        "ccut_autotune_save": [ctypes.c_char_p],
        "ccut_autotune_load": [ctypes.c_char_p],
        "ccut_graph_create": [vp, vp, u64, vp, u64, i32, vp, ctypes.POINTER(vp)],
        "ccut_graph_launch": [vp, vp],
        "ccut_graph_rebind": [vp, vp, vp],
    }.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.ccut_graph_free.argtypes = [vp]
    lib.ccut_graph_free.restype = None
    lib.ccut_profile_enable.argtypes = [i32]
    lib.ccut_profile_enable.restype = ctypes.c_int
    lib.ccut_profile_read.argtypes = [i32, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_char_p)]
    lib.ccut_profile_read.restype = ctypes.c_int
    lib.ccut_profile_reset.argtypes = []
    lib.ccut_profile_reset.restype = ctypes.c_int
    lib.ccut_profile_mask.argtypes = [ctypes.c_uint32]
    lib.ccut_profile_mask.restype = ctypes.c_int
    lib.ccut_plan_free.argtypes = [vp]
    lib.ccut_plan_free.restype = None
    lib.ccut_last_error.restype = ctypes.c_char_p
    lib.ccut_version.restype = ctypes.c_char_p
    return lib


_lib = _load()


def library_path() -> str:
    return _LIB_PATH


def _check(rc: int) -> None:
    if rc != OK:
        raise CcutError(rc, _lib.ccut_last_error().decode())


def _ptr(x) -> int:
    if x is None:
        return 0
    if hasattr(x, "data_ptr"):
        return int(x.data_ptr())
    return int(x)


def _nbytes(x, nbytes: Optional[int]) -> int:
    if nbytes is not None:
        return int(nbytes)
    if hasattr(x, "numel"):
        return int(x.numel() * x.element_size())
    raise ValueError("byte size required for a raw device address")


def _stream(s) -> int:
    if s is None:
        return 0
    if hasattr(s, "cuda_stream"):
        return int(s.cuda_stream)
    return int(s)


def gate_array(gates: Iterable) -> np.ndarray:
    """Packs (kind, q0, q1, p0, p1) tuples into the 32-byte ccut_gate_t layout (an array
    already in that layout is returned as a contiguous copy)."""
    if isinstance(gates, np.ndarray) and gates.dtype == GATE_DTYPE:
        return np.ascontiguousarray(gates).copy()
    gates = list(gates)
    arr = np.zeros(len(gates), dtype=GATE_DTYPE)
    for i, g in enumerate(gates):
        kind, q0 = g[0], g[1]
        q1 = g[2] if len(g) > 2 else -1
        p0 = g[3] if len(g) > 3 else 0.0
        p1 = g[4] if len(g) > 4 else 0.0
        arr[i] = (GATE_KIND[kind] if isinstance(kind, str) else int(kind), q0, q1, 0, p0, p1)
    return arr


class Plan:
    """Owner of an opaque ccut_plan_t (freed on garbage collection)."""

    def __init__(self, handle: int, q: int):
        self._h = ctypes.c_void_p(handle)
        self.q = q

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    def info(self) -> dict:
        inf = PlanInfo()
        _check(_lib.ccut_plan_info(self._h, ctypes.byref(inf)))
        n = inf.n_seg
        return {
            "q": inf.q, "n_seg": n, "c_total": inf.c_total, "n_gates": inf.n_gates,
            "seg_size": list(inf.seg_size[:n]), "seg_offset": list(inf.seg_offset[:n]),
            "c_seg": list(inf.c_seg[:n]), "c_boundary": list(inf.c_boundary[:max(0, n - 1)]),
            "n_sub": inf.n_sub, "n_terms": inf.n_terms,
            "seg_state_offset": list(inf.seg_state_offset[:n]),
            "state_bytes": inf.state_bytes, "arena_bytes": inf.arena_bytes, "psi_bytes": inf.psi_bytes,
            "sim_arena_bytes": inf.sim_arena_bytes,
        }

    def cuts(self) -> List[dict]:
        out = []
        for j in range(self.info()["c_total"]):
            c = CutInfo()
            _check(_lib.ccut_plan_cut(self._h, j, ctypes.byref(c)))
            out.append({f: getattr(c, f) for f, _ in CutInfo._fields_})
        return out

    def cut_terms(self, j: int) -> List[complex]:
        """Weights of cut j's 2^{n_bits} terms (term t = its variant bits as an integer)."""
        out = (ctypes.c_double * 8)()
        _check(_lib.ccut_plan_cut_terms(self._h, j, out))
        n = 1 << self.cuts()[j]["n_bits"]
        return [complex(out[2 * t], out[2 * t + 1]) for t in range(n)]

    def free(self) -> None:
        if self._h and self._h.value:
            _lib.ccut_plan_free(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def cut_plan(q: int, gates, n_seg: int, seg_sizes: Optional[Sequence[int]] = None) -> Plan:
    arr = gates if isinstance(gates, np.ndarray) and gates.dtype == GATE_DTYPE else gate_array(gates)
    arr = np.ascontiguousarray(arr)
    sizes = None
    if seg_sizes is not None:
        sizes = (ctypes.c_int32 * len(seg_sizes))(*seg_sizes)
    h = ctypes.c_void_p(0)
    _check(_lib.ccut_cut_plan(q, arr.ctypes.data, len(arr), n_seg, sizes, ctypes.byref(h)))
    return Plan(h.value, q)


def _gates_from(call) -> np.ndarray:
    """Runs a generator entry point twice: a size query, then the fill."""
    n = ctypes.c_int64(0)
    _check(call(None, 0, ctypes.byref(n)))
    arr = np.zeros(n.value, dtype=GATE_DTYPE)
    _check(call(arr.ctypes.data if n.value else None, n.value, ctypes.byref(n)))
    return arr


def brickwork_gates(q: int, d: int, n_seg: int, c_total: int, seed: int,
                    seg_sizes: Optional[Sequence[int]] = None,
                    cuts_per_boundary: Optional[Sequence[int]] = None) -> np.ndarray:
    """The library's seeded brickwork (ccut_brickwork) as a ccut_gate_t array."""
    sizes = (ctypes.c_int32 * n_seg)(*seg_sizes) if seg_sizes is not None else None
    cuts = (ctypes.c_int32 * max(1, n_seg - 1))(*cuts_per_boundary) if cuts_per_boundary is not None else None
    return _gates_from(lambda out, cap, n: _lib.ccut_brickwork(q, d, n_seg, c_total, sizes, cuts,
                                                               seed & 0xFFFFFFFFFFFFFFFF, out, cap, n))


def staircase_gates(q: int, copies: int, tx_layers: int = 0) -> np.ndarray:
    """The paper's Fig. 1 staircase family (ccut_staircase) as a ccut_gate_t array."""
    return _gates_from(lambda out, cap, n: _lib.ccut_staircase(q, copies, tx_layers, out, cap, n))


def plan_prepare(plan: Plan) -> None:
    _check(_lib.ccut_plan_prepare(plan.handle))


def cut_weight(bit: int) -> complex:
    out = (ctypes.c_double * 2)()
    _check(_lib.ccut_cut_weight(bit, out))
    return complex(out[0], out[1])


def simulate_subcircuits(plan: Plan, arena, arena_bytes: Optional[int] = None, stream=None) -> None:
    _check(_lib.ccut_simulate_subcircuits(plan.handle, _ptr(arena), _nbytes(arena, arena_bytes), _stream(stream)))


def merge_full_state(plan: Plan, arena, psi, precision="fp32", arena_bytes: Optional[int] = None,
                     psi_bytes: Optional[int] = None, stream=None) -> None:
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    _check(_lib.ccut_merge_full_state(plan.handle, _ptr(arena), _nbytes(arena, arena_bytes), _ptr(psi),
                                      _nbytes(psi, psi_bytes), prec, _stream(stream)))


def simulate_uncut(q: int, gates, psi, psi_bytes: Optional[int] = None, stream=None) -> None:
    arr = gates if isinstance(gates, np.ndarray) and gates.dtype == GATE_DTYPE else gate_array(gates)
    arr = np.ascontiguousarray(arr)
    _check(_lib.ccut_simulate_uncut(q, arr.ctypes.data, len(arr), _ptr(psi), _nbytes(psi, psi_bytes),
                                    _stream(stream)))


def norm_fidelity(psi, ref, q: int, stream=None) -> dict:
    out = (ctypes.c_double * 5)()
    _check(_lib.ccut_norm_fidelity(_ptr(psi), _ptr(ref), q, out, _stream(stream)))
    n2p, n2r, ore, oim, mx = out[:]
    res = {"norm2": n2p, "ref_norm2": n2r, "overlap": complex(ore, oim), "max_abs": mx}
    if ref is not None and n2p > 0 and n2r > 0:
        res["fidelity"] = (ore * ore + oim * oim) / (n2p * n2r)
    return res


def norm_fidelity_noalloc(psi, ref, q: int, out, stream=None) -> None:
    """Allocation-free form: the five float64 results go to the device buffer `out`."""
    _check(_lib.ccut_norm_fidelity_noalloc(_ptr(psi), _ptr(ref), q, _ptr(out), _stream(stream)))


PROF_KERNELS = 8
MLP_PARAMS = 4931
MLP_IN = 8


def expectation_work_bytes(plan: Plan) -> int:
    out = ctypes.c_uint64(0)
    _check(_lib.ccut_expectation_work_bytes(plan.handle, ctypes.byref(out)))
    return int(out.value)


def expectation_pauli(plan: Plan, arena, pauli: str, work, arena_bytes: Optional[int] = None,
                      work_bytes: Optional[int] = None, stream=None) -> complex:
    """<Psi|P|Psi> of the cut state from the subcircuit states (character j of `pauli` on qubit j)."""
    out = (ctypes.c_double * 2)()
    _check(_lib.ccut_expectation_pauli(plan.handle, _ptr(arena), _nbytes(arena, arena_bytes), pauli.encode(),
                                       _ptr(work), _nbytes(work, work_bytes), out, _stream(stream)))
    return complex(out[0], out[1])


def threshold_ctotal(q: int, n: int) -> float:
    out = ctypes.c_double()
    _check(_lib.ccut_threshold_ctotal(q, n, ctypes.byref(out)))
    return out.value


def speedup_margin(q: int, n: int, cuts_per_boundary: Sequence[int]) -> float:
    arr = (ctypes.c_int32 * max(1, len(cuts_per_boundary)))(*cuts_per_boundary)
    out = ctypes.c_double()
    _check(_lib.ccut_speedup_margin(q, n, arr, ctypes.byref(out)))
    return out.value


def cost_features(q: int, d: int, n: int, c_total: int) -> List[float]:
    out = (ctypes.c_float * MLP_IN)()
    _check(_lib.ccut_cost_features(q, d, n, c_total, out))
    return list(out)


def mlp_work_bytes(rows: int, epochs: int) -> int:
    out = ctypes.c_uint64()
    _check(_lib.ccut_mlp_work_bytes(rows, epochs, ctypes.byref(out)))
    return out.value


def mlp_predict(params, x, y, rows: int, stream=None) -> None:
    _check(_lib.ccut_mlp_predict(_ptr(params), _ptr(x), rows, _ptr(y), _stream(stream)))


def mlp_grad(params, x, t, rows: int, work, grad, work_bytes: Optional[int] = None, stream=None) -> float:
    loss = ctypes.c_float()
    _check(_lib.ccut_mlp_grad(_ptr(params), _ptr(x), _ptr(t), rows, _ptr(work), _nbytes(work, work_bytes),
                              _ptr(grad), ctypes.byref(loss), _stream(stream)))
    return loss.value


def mlp_train(params, x, t, rows: int, epochs: int, lr: float, work, work_bytes: Optional[int] = None,
              stream=None) -> np.ndarray:
    losses = np.zeros(max(epochs, 1), dtype=np.float32)
    _check(_lib.ccut_mlp_train(_ptr(params), _ptr(x), _ptr(t), rows, epochs, lr, _ptr(work),
                               _nbytes(work, work_bytes), losses.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                               _stream(stream)))
    return losses[:epochs]


# Guard margin of the learned decision validated on held-out measured rows (results/cost_model.json):
# from 0.1 on, no held-out decision was slower than the closed-form rule's.
DECIDE_MARGIN = 0.1


def decide(q: int, d: int, c_total: int, params=None, budget_s: float = 0.0, margin: float = DECIDE_MARGIN,
           stream=None):
    """(choice, predicted seconds): choice 0 = no cut, n >= 2 segments, -1 = over budget.
    margin: leave the closed-form choice only for a predicted gain above this fraction."""
    choice = ctypes.c_int32()
    pred = ctypes.c_double()
    _check(_lib.ccut_decide(q, d, c_total, _ptr(params) if params is not None else None, budget_s, margin,
                            ctypes.byref(choice), ctypes.byref(pred), _stream(stream)))
    return choice.value, pred.value


def profile_enable(on: bool = True) -> None:
    _check(_lib.ccut_profile_enable(1 if on else 0))


PROFILE_KERNELS = ("sim", "merge_f32", "split", "tables", "merge_gemm", "reduce", "mlp", "expect")


def profile_mask(kernels=None) -> None:
    """Time only the named kernel families while profiling is on (None: all)."""
    mask = 0xFFFFFFFF if kernels is None else sum(1 << PROFILE_KERNELS.index(k) for k in kernels)
    _check(_lib.ccut_profile_mask(mask))


def profile_reset() -> None:
    _check(_lib.ccut_profile_reset())


def profile_read() -> dict:
    """{family: (launches, total_ms)} accumulated since the last reset."""
    out = {}
    for k in range(PROF_KERNELS):
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        name = ctypes.c_char_p()
        _check(_lib.ccut_profile_read(k, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(name)))
        out[name.value.decode()] = (n.value, ms.value)
    return out


def plan_set_launch(plan: Plan, threads: int = 256, grid_cap: int = 0, per_variant: bool = False,
                    mfma_min_terms: int = -1) -> None:
    _check(_lib.ccut_plan_set_launch(plan.handle, threads, grid_cap, 1 if per_variant else 0, mfma_min_terms))


def plan_set_merge(plan: Plan, epilogue: int = 0, grid_cap: int = 0) -> None:
    _check(_lib.ccut_plan_set_merge(plan.handle, epilogue, grid_cap))


def plan_get_merge(plan: Plan) -> dict:
    out = (ctypes.c_int32 * 2)()
    _check(_lib.ccut_plan_get_merge(plan.handle, out))
    return {"variant": out[0], "grid_cap": out[1]}


def plan_set_auto_precision(plan: Plan, precision) -> None:
    """Split arithmetic CCUT_PREC_AUTO uses on MFMA: "fp16x3", "bf16x3" or (opt-in) "fp16x2"."""
    p = PRECISIONS[precision] if isinstance(precision, str) else precision
    _check(_lib.ccut_plan_set_auto_precision(plan.handle, p))


def plan_get_auto_precision(plan: Plan) -> str:
    out = ctypes.c_int32()
    _check(_lib.ccut_plan_get_auto_precision(plan.handle, ctypes.byref(out)))
    return {v: k for k, v in PRECISIONS.items()}[out.value]


def resolved_precision(plan: Plan, precision, k: int) -> str:
    """The arithmetic merge_full_state runs for a stage of k terms under `precision`."""
    if precision not in ("auto", PREC_AUTO):
        return precision if isinstance(precision, str) else {v: n for n, v in PRECISIONS.items()}[precision]
    kmin = plan_get_launch(plan)["mfma_min_terms"]
    return plan_get_auto_precision(plan) if k >= (kmin if kmin >= 0 else 8) else "fp32"


def plan_set_block_bits(plan: Plan, bits: int) -> None:
    """LDS block size of the simulation (2^bits amplitudes; 0 = automatic)."""
    _check(_lib.ccut_plan_set_block_bits(plan.handle, int(bits)))


SIM_PRECISIONS = {"fp32": 0, "fp16x3": 1}


def plan_set_sim_precision(plan: Plan, precision) -> None:
    """Gate arithmetic of the subcircuit simulation: "fp32" (vector ALUs) or "fp16x3" (MFMA groups)."""
    p = SIM_PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    _check(_lib.ccut_plan_set_sim_precision(plan.handle, p))


def plan_get_sim_precision(plan: Plan) -> str:
    out = ctypes.c_int32(0)
    _check(_lib.ccut_plan_get_sim_precision(plan.handle, ctypes.byref(out)))
    return {v: k for k, v in SIM_PRECISIONS.items()}[int(out.value)]


def plan_set_prefix_sharing(plan: Plan, mode: int) -> None:
    """Prefix sharing in the subcircuit simulation: 0 off, 1 on, -1 automatic."""
    _check(_lib.ccut_plan_set_prefix_sharing(plan.handle, int(mode)))


def plan_set_fusion(plan: Plan, on: bool) -> None:
    """Register-stage gate fusion (ccut_plan_set_fusion)."""
    _check(_lib.ccut_plan_set_fusion(plan.handle, int(on)))


def plan_get_fusion(plan: Plan) -> bool:
    out = ctypes.c_int32()
    _check(_lib.ccut_plan_get_fusion(plan.handle, ctypes.byref(out)))
    return bool(out.value)


def plan_get_prefix_sharing(plan: Plan) -> bool:
    out = ctypes.c_int32(0)
    _check(_lib.ccut_plan_get_prefix_sharing(plan.handle, ctypes.byref(out)))
    return bool(out.value)


def plan_set_prefix_start(plan: Plan, level: int) -> None:
    """First level of the prefix-sharing tree (the slots below it run flat)."""
    _check(_lib.ccut_plan_set_prefix_start(plan.handle, int(level)))


def plan_get_prefix_start(plan: Plan) -> int:
    out = ctypes.c_int32(0)
    _check(_lib.ccut_plan_get_prefix_start(plan.handle, ctypes.byref(out)))
    return int(out.value)


def plan_get_block_bits(plan: Plan) -> int:
    out = ctypes.c_int32(0)
    _check(_lib.ccut_plan_get_block_bits(plan.handle, ctypes.byref(out)))
    return int(out.value)


def plan_stats(plan: Plan) -> dict:
    out = (ctypes.c_int64 * 8)()
    _check(_lib.ccut_plan_stats(plan.handle, out))
    keys = ("passes", "stages", "device_ops", "dense_ops", "diag_ops", "fused_ops", "launches", "jobs")
    return dict(zip(keys, out[:]))


def plan_work(plan: Plan) -> dict:
    """Work the simulation launches execute under the plan's current schedule."""
    out = (ctypes.c_double * 5)()
    _check(_lib.ccut_plan_work(plan.handle, out))
    return {"dense_amp_ops": out[0], "diag_amp_ops": out[1], "perm_amp_ops": out[2],
            "amps_moved": out[3], "flat_dense_amp_ops": out[4]}


def plan_get_launch(plan: Plan) -> dict:
    out = (ctypes.c_int32 * 4)()
    _check(_lib.ccut_plan_get_launch(plan.handle, out))
    return {"threads": out[0], "grid_cap": out[1], "per_variant": out[2], "mfma_min_terms": out[3]}


def autotune(plan: Plan, arena, psi, reps: int = 3, arena_bytes: Optional[int] = None,
             psi_bytes: Optional[int] = None, stream=None) -> float:
    best = ctypes.c_double()
    _check(_lib.ccut_autotune(plan.handle, _ptr(arena), _nbytes(arena, arena_bytes), _ptr(psi),
                              _nbytes(psi, psi_bytes), reps, _stream(stream), ctypes.byref(best)))
    return best.value


def autotune_save(path: str) -> None:
    _check(_lib.ccut_autotune_save(path.encode()))


def autotune_load(path: str) -> None:
    _check(_lib.ccut_autotune_load(path.encode()))


class Graph:
    """Owner of a captured pipeline graph (ccut_graph_t)."""

    def __init__(self, plan: Plan, arena, psi, precision="auto", stream=None,
                 arena_bytes: Optional[int] = None, psi_bytes: Optional[int] = None):
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        h = ctypes.c_void_p(0)
        _check(_lib.ccut_graph_create(plan.handle, _ptr(arena), _nbytes(arena, arena_bytes), _ptr(psi),
                                      _nbytes(psi, psi_bytes), prec, _stream(stream), ctypes.byref(h)))
        self._h = h

    def rebind(self, plan: Plan, stream=None) -> None:
        """Next replays on `stream` run `plan` (same launch layout as the captured plan)."""
        _check(_lib.ccut_graph_rebind(self._h, plan.handle, _stream(stream)))

    def launch(self, stream=None) -> None:
        _check(_lib.ccut_graph_launch(self._h, _stream(stream)))

    def free(self) -> None:
        if self._h and self._h.value:
            _lib.ccut_graph_free(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def version() -> str:
    return _lib.ccut_version().decode()
