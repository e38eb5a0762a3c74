"""MI355X-native Cherenkov photon propagation through a RICH-like detector.

The compute path is the HIP library ``librich.so`` behind the C ABI declared
in ``include/rich.h``; ``paper_2309_12496_amd.rich`` is its Python binding and
``paper_2309_12496_amd.inputs`` holds the seeded synthetic workloads.
Importing the package itself loads nothing.
"""
