"""MI355X-native forced lattice-Boltzmann step (arXiv 2212.07494).

The compute path lives in the HIP library built from ``csrc/`` (``liblbm.so``);
:mod:`paper_2212_07494_amd.lbm` is a thin ctypes binding with the C-ABI's names and
:mod:`paper_2212_07494_amd.inputs` builds seeded synthetic inputs.  Submodules are
imported on demand (``from paper_2212_07494_amd import lbm``), so ``inputs`` stays
usable where the library is not built.
"""
