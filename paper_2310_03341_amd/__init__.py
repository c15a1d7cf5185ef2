"""MI355X-native dense BdG eigensolver (arXiv:2310.03341 hot path).

``paper_2310_03341_amd.api`` is the Python binding of libbdg.so (the C-ABI in
include/bdg.h); ``paper_2310_03341_amd.inputs`` holds the seeded synthetic
workload generators.  Importing the package does not load the library.
"""
__all__ = ["api", "inputs", "build"]
