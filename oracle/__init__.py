"""FP64 CPU oracle for the PSF-library operator -- test infrastructure only.

Imported by ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg
of ``bench.py``; never by the product package.
"""
from .psf_oracle import *  # noqa: F401,F403
