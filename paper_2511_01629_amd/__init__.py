"""MI355X-native constraint-penalization lattice Boltzmann for rigid particles
(Millet & Liberge, arXiv 2511.01629).

The compute path is the HIP library `liblbmpen.so` (kernels for gfx950 behind
the C ABI declared in include/lbm.h).  `paper_2511_01629_amd.lbm` is the thin
ctypes binding; `paper_2511_01629_amd.workloads` holds the seeded inputs.
Importing the package loads nothing; the binding loads the library on first
use and raises if it has not been built.
"""
