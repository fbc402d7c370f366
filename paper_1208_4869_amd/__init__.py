"""MI355X-native complex Krylov solvers (BiCGSTAB, CGNR) for A x = y.

The work runs in hand-written gfx950 HIP kernels behind the C ABI declared in
``include/ccg.h`` (shared library ``libccg.so``).  ``paper_1208_4869_amd.ccg``
is the thin ctypes binding over it; ``inputs`` builds seeded synthetic systems.
"""
