"""MI355X (gfx950) circuit cutting for classical state-vector simulation.

The compute path is the HIP library ``libccut.so`` (sources in ``csrc/``,
C ABI in ``include/ccut.h``); ``ccut`` is its ctypes binding and
``pipeline`` keeps device buffers in PyTorch tensors.  Import ``ccut``
explicitly: it fails loudly when the library has not been built.
"""
