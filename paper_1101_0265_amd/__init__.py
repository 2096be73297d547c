"""Scale-and-fold density-matrix purification on MI355X (gfx950).

The compute path is the HIP library ``libsnf.so`` behind the C ABI in ``include/snf.h``;
``paper_1101_0265_amd.snf`` is its ctypes binding.  ``hamiltonians`` makes seeded synthetic
inputs.  Importing the package does not load the library (so CPU-only tools can use the
input generators); the first call through ``snf`` does, and fails loudly if it is missing.
"""

__all__ = ["snf", "hamiltonians"]
