"""MI355X-native many-replica Metropolis annealer for sparse Ising / MaxCut.

The compute path is the HIP library ``libising.so`` (built from ``csrc/``)
behind a C ABI declared in ``include/ising.h``; :mod:`.binding` is a thin
ctypes layer over it.  Importing this package does not load the library;
``from paper_2311_09275_amd import binding`` does, and fails loudly when the
library has not been built.
"""
__all__ = ["binding", "instances", "ttt"]
