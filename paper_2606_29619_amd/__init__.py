"""MI355X-native hot path of the one-domain porous-media lattice Boltzmann method
(Gusev & Karlin, arXiv 2606.29619): hand-written HIP kernels for gfx950 behind a C-ABI library
(``include/lbm.h``), with a thin ctypes binding of the same names in ``capi``.

The binding loads ``liblbm.so`` lazily on first use and fails loudly when it is missing; there is
no CPU fallback.
"""
__all__ = ["capi", "workloads"]
