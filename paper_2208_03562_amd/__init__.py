"""MI355X-native hot path of the preconditioned rectangular central-moment
lattice Boltzmann method (PRC-LBM, arXiv 2208.03562).

``capi`` is the ctypes binding of the C ABI (``include/prc.h``); ``solver``
wraps it with PyTorch-owned device buffers.  Both load ``libprc.so`` lazily so
that CPU-only tooling can import the package; any compute call without the
built library raises.
"""
__all__ = ["capi", "solver"]
