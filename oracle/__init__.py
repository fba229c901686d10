"""CPU oracle of the Focus-Gaussian slice renderer (GaussianPile, Sec. 4).

TEST INFRASTRUCTURE ONLY.  This package is imported by the test-suite, by the
smoke check and by the CPU-baseline leg of the benchmark, and by nothing else.
The product path (the HIP library and its Python binding) never imports, links
or executes it, and it shares no code with that path.

  spec32  binary32 emulation of tile membership (axial cull + tile footprint)
  focus   float64 literal-route renderer, autograd gradient, Adam

Every function is pinned by CPU tests (tests/test_oracle_pins.py) against
closed forms, quadrature of the paper's convolution integral, the two limits of
the model, brute force on tiny grids, finite differences and textbook
properties of Adam.
"""
from . import spec32, focus  # noqa: F401
