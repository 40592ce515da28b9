"""MI355X-native triangle centrality (Burkhardt, arXiv 2105.00110).

The compute path is the HIP library ``libtc.so`` behind the C ABI in
``include/tc.h``; ``paper_2105_00110_amd.tc`` is its thin ctypes binding and
``graphgen`` the seeded input generators.
"""
__all__ = ["tc", "graphgen"]
