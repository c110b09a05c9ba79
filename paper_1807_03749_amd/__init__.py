"""MI355X (gfx950) coupled cluster Monte Carlo step: HIP kernels behind a C ABI.

The data-parallel hot path of CCMC (Spencer et al., arXiv:1807.03749) -- cluster
selection, collapse, spawning with full non-composite and multi-spawn sampling, death and
annihilation into a device-resident sorted excitor store -- runs in ``libccmc.so``;
``ccmc.py`` is its ctypes binding and ``driver.py`` the host-side run loop.
"""
