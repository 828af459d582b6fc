"""MI355X-native variable-density pressure Poisson solver.

Solves div((1/rho) grad p) = b on a uniform triply periodic staggered grid with
the iteration of Pouransari, Mortazavi & Mani (arXiv:1601.05448, section
"Poisson equation"), in hand-written HIP kernels for gfx950 behind a C ABI
(``include/poisson.h``).  The Python side is argument marshalling only; see
``paper_1601_05448_amd.poisson``.

Submodules are imported lazily so that ``paper_1601_05448_amd.inputs`` (the
seeded input generators) can be used without loading the GPU library.
"""
__all__ = ["inputs", "poisson"]
