"""MI355X-native sparse state-vector simulator (arXiv 2105.01533, Sec. 3).

The product is ``libsparsesim.so`` (HIP kernels for gfx950 behind the C-ABI in
``include/sparsesim.h``); ``paper_2105_01533_amd.sim`` is its ctypes binding and
``paper_2105_01533_amd.workloads`` the seeded circuit generators.  Importing
the package itself loads nothing.
"""
