"""MI355X (gfx950) AM-AMG-preconditioned FGMRES solver for the Schwinger-model Wilson-Dirac system.

The solver is the HIP library ``libamamg.so`` behind the C ABI of ``include/amamg.h``;
``paper_2608_03515_amd.amamg`` is its ctypes binding and ``paper_2608_03515_amd.build``
compiles it.  Importing this package does not load the library.
"""
