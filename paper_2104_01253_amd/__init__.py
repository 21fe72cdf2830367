"""MI355X-native DCGS2 Arnoldi-QR expansion (one global reduction per step).

The compute path is the C-ABI library ``libdcgs2.so`` (hand-written HIP for
gfx950, built from ``csrc/``); ``binding`` marshals torch device tensors into
it.  See ``include/dcgs2.h`` for the interface.
"""
__all__ = ["binding", "synth"]
