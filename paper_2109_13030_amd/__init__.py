"""MI355X-native batched alternating-minimization trajectory optimizer
(arXiv 2109.13030): a HIP library behind a C-ABI plus a thin Python binding.

Importing the package loads nothing; ``paper_2109_13030_amd.am`` loads the
compiled library on first use and fails loudly when it is missing.
"""
__all__ = ["inputs", "am"]
