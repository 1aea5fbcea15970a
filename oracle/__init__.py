"""Plain complex128 CPU oracle for circuit cutting in state-vector simulation.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls, links
or executes anything in this package: only ``tests/``, the smoke check in
``__graft_entry__.py`` and the ``cpu_baseline`` leg of ``bench.py`` may use
it.  It shares no code with the HIP path (``paper_2603_01443_amd/``); the
two meet only in the seeded circuit generators of ``inputs/``.

What it computes, following the paper (arXiv 2603.01443):

* ``statevector`` - gate-by-gate simulation of a circuit on |0...0>, the
  uncut baseline T_orig (Sec. III.A) and the StateVectorSimulate step of
  Algorithm 2.
* ``cutting`` - preprocessing (Algorithm 1: boundary gates, fragments,
  2^{c_i} variants per segment with S or S^dagger at each cut, HSH on a CX
  target), variant simulation (Algorithm 2), and the merge (Algorithm 3) as
  the plain sum over every global combination of cut terms, using the CZ
  decomposition of Eq. (CZ).
* ``metrics`` - norm, overlap, fidelity and max-abs error in float64.
* ``threshold`` - the closed-form cut thresholds of Sec. IV
  (Eqs. speedup_depth_free, threshold_n2, threshold_nge3, threshold_with_D,
  Table II).
* ``mlp`` - float64 forward, loss, backward and Adam step of the 8-64-64-3
  cost-model network.  The network is not part of the paper: parity
  unpinned with respect to the paper; its gradients are pinned by central
  finite differences.

Everything is float64 / complex128, written for readability, not speed.
"""
