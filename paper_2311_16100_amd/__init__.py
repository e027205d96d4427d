"""MI355X (gfx950) implementation of the known-pose Fourier-slice refinement
of Toader, Brubaker & Lederman, "Efficient high-resolution refinement in
cryo-EM with stochastic gradient descent" (arXiv:2311.16100).

The compute path is the HIP library libcryosgd.so behind the C ABI of
include/cryosgd.h; `binding` is its thin ctypes wrapper over torch device
tensors.  Submodules are imported on use so that importing the package does
not load the GPU library.
"""
__all__ = ["binding", "build"]
