"""MI355X-native field-dependent PSF operator (Milani & Douglas, arXiv 2106.09122).

The operator lives in ``libpsflib.so`` (hand-written HIP for gfx950, C ABI
declared in ``include/psflib.h``); :mod:`paper_2106_09122_amd.psflib` is its
Python binding (``from paper_2106_09122_amd import psflib``).  Importing it
fails loudly if the library has not been built.
"""
