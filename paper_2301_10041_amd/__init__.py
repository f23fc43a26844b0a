"""MI355X-native hot path of the DLM fictitious-domain FSI solver (Boffi, Credali,
Gastaldi, Scacchi).

The compute path is the C-ABI library ``libfsi.so`` (hand-written HIP for gfx950)
declared in ``include/fsi.h``; :mod:`paper_2301_10041_amd.fsi` is its thin ctypes
binding.  Importing this package loads nothing: the binding loads the library on
first use and raises if it is missing.
"""
