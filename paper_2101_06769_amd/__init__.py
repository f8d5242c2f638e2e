"""MI355X-native hot path of the multiphase lattice Boltzmann solver of
arXiv 2101.06769: cumulant pressure-based flow populations coupled to
conservative Allen-Cahn phase-field populations, as HIP kernels for gfx950
behind a C ABI (``libmplb.so``).

``inputs`` (seeded case generators) imports nothing else from this package;
the GPU binding lives in ``mplb`` and loads the shared library on first use.
"""
