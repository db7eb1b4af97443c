"""MI355X (gfx950) implementation of the improved random batch Ewald (IRBE)
non-bonded force: random batch list short range + random batch Ewald long range
(Liang, Xu, Zhao, arXiv:2204.13595).

The compute path is the HIP library ``libirbe.so`` behind the C ABI of
``include/irbe.h``; :mod:`paper_2204_13595_amd.irbe` is its Python binding.
Importing the package does not load the library; the binding loads it on first
use and raises if it is missing.
"""

__all__ = ["irbe", "inputs"]
