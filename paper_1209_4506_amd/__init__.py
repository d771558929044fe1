"""MI355X-native periodic Hartree (FFT-Poisson) solve with a Gaussian density splat.

The compute path is the HIP library ``libhartree.so`` (built from ``csrc/``)
behind the C ABI declared in ``include/hartree.h``; ``hartree`` is its thin
Python binding.  ``inputs`` draws the seeded synthetic workloads.  Importing
the package loads nothing; importing ``paper_1209_4506_amd.hartree`` loads the
library and fails loudly if it is missing.
"""
__all__ = ["inputs"]
