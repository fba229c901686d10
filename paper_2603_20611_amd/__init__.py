"""MI355X-native Focus-Gaussian slice renderer (GaussianPile hot path).

The compute path is the HIP library ``libgaussianpile.so`` (gfx950), reached
through the C-ABI declared in ``include/gaussianpile.h``.  ``binding`` loads it
with ctypes and fails loudly when it is missing; ``render`` wraps it in a
``torch.autograd.Function``; ``synth`` draws the seeded synthetic workloads.
Importing the package itself loads nothing.
"""
__all__ = ["binding", "render", "synth"]
