"""MI355X-native SMAME solver (arXiv 2012.03525): HIP kernels behind a C ABI.

Importing the package loads nothing; `paper_2012_03525_amd.acm` opens the
compiled library `libacm.so` (built by `paper_2012_03525_amd.build`) and
raises if it is missing.
"""
__all__ = ["acm", "inputs", "build"]
