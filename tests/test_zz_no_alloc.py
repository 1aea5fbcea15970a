"""The allocation-free reduction entry point (ccut_norm_fidelity_noalloc) against
ccut_norm_fidelity, whose kernels it shares: its partials sit in the library's fixed
device array instead of an allocated buffer.  Two calls in a row, the second on a
smaller state, so the second reads only partials it wrote itself."""

import sys

import numpy as np
import pytest

from paper_2603_01443_amd import ccut


def _case(msg):
    print(f"no-alloc reduction: {msg}", file=sys.stderr, flush=True)


@pytest.mark.gpu
def test_noalloc_reduction_matches_the_allocating_entry_point():
    import torch

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    gen = torch.Generator().manual_seed(11)
    for q, with_ref in ((20, True), (13, True), (13, False), (0, True)):
        _case(f"q={q} ref={'yes' if with_ref else 'no'}")
        n = 1 << q
        psi_h = torch.randn(n, dtype=torch.complex64, generator=gen) * 2 ** (-q / 2)
        ref_h = psi_h + 1e-3 * torch.randn(n, dtype=torch.complex64, generator=gen) * 2 ** (-q / 2)
        psi = psi_h.to(dev)
        ref = ref_h.to(dev) if with_ref else None
        want = ccut.norm_fidelity(psi, ref, q, stream=stream)
        out = torch.full((5,), float("nan"), dtype=torch.float64, device=dev)
        ccut.norm_fidelity_noalloc(psi, ref, q, out, stream=stream)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        exp = np.array([want["norm2"], want["ref_norm2"], want["overlap"].real, want["overlap"].imag,
                        want["max_abs"]])
        # same kernels and the same block count: the fixed summation order gives the same bits
        assert np.array_equal(got, exp), (q, got, exp)
        # and the float64 definitions on the host (float64 sums of float32 products)
        p = psi_h.numpy().astype(np.complex128)
        r = ref_h.numpy().astype(np.complex128) if with_ref else np.zeros_like(p)
        host = np.array([np.vdot(p, p).real, np.vdot(r, r).real, np.vdot(r, p).real, np.vdot(r, p).imag,
                         np.max(np.abs(p - r))])
        scale = np.array([host[0], max(host[1], 1e-300), np.sqrt(host[0] * host[1]) + 1e-300,
                          np.sqrt(host[0] * host[1]) + 1e-300, max(host[4], 1e-300)])
        assert np.all(np.abs(got - host) <= 1e-9 * scale), (q, got, host)


def test_noalloc_reduction_rejects_states_beyond_the_array():
    """q above CCUT_MAX_Q is refused on the host before anything is launched."""
    with pytest.raises(ccut.CcutError) as e:
        ccut.norm_fidelity_noalloc(1 << 20, None, 36, 1 << 20)
    assert e.value.code == ccut.EINVAL
