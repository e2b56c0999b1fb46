"""MI355X-native kinematical powder-XRD hot path (gfx950 HIP kernels behind a C ABI).

Importing the package loads nothing; ``paper_2602_11709_amd.api`` loads the
HIP library and fails loudly when it has not been built.
"""

__all__ = ["synth"]
