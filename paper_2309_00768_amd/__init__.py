"""Space-time block-preconditioned FGMRES for linearised resistive MHD on MI355X.

The compute path is the C-ABI library ``libst.so`` (hand-written HIP for gfx950);
``binding`` is its thin ctypes layer.  ``inputs`` holds the seeded synthetic
workloads.  Importing the package loads nothing; ``binding`` loads the library
on first use and raises if it is missing.
"""
