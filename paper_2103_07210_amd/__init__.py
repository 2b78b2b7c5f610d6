"""MI355X-native FT-GCR: fault-tolerant preconditioned GCR(k) on a
lat-lon-height sphere grid (Gillard & Benacchio, arXiv 2103.07210).

The solver lives in the HIP library ``libftgcr.so`` behind the C ABI declared
in ``include/ftgcr.h``; :mod:`.ftgcr` is the thin ctypes binding and
:mod:`.inputs` the seeded synthetic-input generators.  Importing this package
loads nothing; the binding loads the library on first use and raises if it is
missing.
"""

__all__ = ["ftgcr", "inputs"]
