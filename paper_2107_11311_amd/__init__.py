"""MI355X-native hot path of Behler-Parrinello ANN-potential molecular dynamics
with the Chebyshev descriptor (arXiv:2107.11311, Sec. II): GPU neighbour list,
descriptors, per-species atomic networks, force back-propagation and velocity
Verlet, behind the C ABI declared in include/aenet_gpu.h.

Importing the package loads nothing; the HIP library is loaded on first use by
paper_2107_11311_amd.aenet (see aenet.load()).
"""
__all__ = ["inputs"]
