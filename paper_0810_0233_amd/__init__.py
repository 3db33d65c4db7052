"""MI355X-native Cartesian fast multipole method for point-dipole fields.

The compute path is the HIP library ``libccfmm.so`` (built from ``csrc/``),
reached through the C ABI in ``include/ccfmm.h``; ``ccfmm`` is its thin
ctypes binding.  ``inputs`` holds the seeded synthetic workloads.  Importing
the package does not load the library; ``ccfmm.lib()`` does, and fails loudly
when it is missing.
"""
