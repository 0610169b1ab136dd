"""Reverse Cuthill-McKee ordering on one AMD Instinct MI355X.

The ordering runs in the HIP library ``librcm.so`` (C ABI in include/rcm.h);
``paper_1610_08128_amd.rcm`` is its Python binding and
``paper_1610_08128_amd.inputs`` holds the seeded synthetic workload
generators.  Importing the package loads neither torch nor the library.
"""

__all__ = ["rcm", "inputs", "build"]
