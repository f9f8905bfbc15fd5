"""MadFlow's per-event integrand (arXiv:2106.10279) as a gfx950 HIP library.

The product is libmadflow_mi355x.so (C ABI in include/mf.h); this package
is its thin Python binding.  Importing `paper_2106_10279_amd.api` loads the
library and fails loudly when it has not been built.
"""

__all__ = ["api", "build"]
