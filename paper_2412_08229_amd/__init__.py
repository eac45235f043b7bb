"""MI355X (gfx950) engine for the neural-collision-operator lattice Boltzmann
method (arXiv 2412.08229).

The compute path is the HIP library ``libnco.so`` (C ABI in include/nco.h);
``Lattice`` is a thin wrapper over it.  ``inputs`` holds the seeded synthetic
workloads.  Importing the package does not load the library; the first call
that needs it does, and fails loudly if it has not been built.
"""
from .lattice import Lattice, n_bins  # noqa: F401
