"""Device buffers for one cut run, held in PyTorch tensors (memory and streams only).

``CutRun`` owns a plan, an arena (subcircuit states + merge workspace) and the
2^q output, and calls the C-ABI stages in order:
cut_plan (T_pre) -> simulate_subcircuits (T_sub) -> merge_full_state (T_merge).
``uncut`` runs the baseline simulate_uncut (T_orig) into its own buffer.
"""

from __future__ import annotations

from typing import Optional, Sequence

import torch

from . import ccut


def _stream():
    return torch.cuda.current_stream().cuda_stream


class CutRun:
    def __init__(self, q: int, gates, n_seg: int, seg_sizes: Optional[Sequence[int]] = None,
                 device: str = "cuda:0", psi: Optional[torch.Tensor] = None, sim_only: bool = False):
        self.q = q
        self.device = torch.device(device)
        self.gates = ccut.gate_array(gates)
        self.plan = ccut.cut_plan(q, self.gates, n_seg, seg_sizes)
        self.info = self.plan.info()
        with torch.cuda.device(self.device):
            # sim_only: room for the simulation (and expectation values) only, no merge workspace
            size = self.info["sim_arena_bytes"] if sim_only else self.info["arena_bytes"]
            self.arena = torch.empty(max(size, 8), dtype=torch.uint8, device=self.device)
            self.psi = psi if psi is not None else torch.empty(1 << q, dtype=torch.complex64, device=self.device)
            ccut.plan_prepare(self.plan)

    def simulate_subcircuits(self) -> None:
        ccut.simulate_subcircuits(self.plan, self.arena, stream=_stream())

    def merge(self, precision="fp32") -> torch.Tensor:
        ccut.merge_full_state(self.plan, self.arena, self.psi, precision, stream=_stream())
        return self.psi

    def run(self, precision="fp32") -> torch.Tensor:
        self.simulate_subcircuits()
        return self.merge(precision)

    def variant_state(self, seg: int, r: int) -> torch.Tensor:
        """View of segment seg's variant r in the arena (complex64, 2^{q_seg})."""
        nq = self.info["seg_size"][seg]
        off = self.info["seg_state_offset"][seg] + r * 8 * (1 << nq)
        return self.arena[off:off + 8 * (1 << nq)].view(torch.complex64)


def uncut(q: int, gates, device: str = "cuda:0", out: Optional[torch.Tensor] = None) -> torch.Tensor:
    dev = torch.device(device)
    psi = out if out is not None else torch.empty(1 << q, dtype=torch.complex64, device=dev)
    ccut.simulate_uncut(q, ccut.gate_array(gates), psi, stream=_stream())
    return psi
