"""MI355X-native multigrid-preconditioned Bi-CGSTAB solver for the 2-D
Helmholtz equation with first-order Sommerfeld boundaries (the method of
Livshits, arXiv:1312.2880).

The compute path is the C-ABI library ``libhmg.so`` (hand-written HIP for
gfx950); ``paper_1312_2880_amd.hmg`` is its thin ctypes binding and raises if
the library is not built.  ``paper_1312_2880_amd.inputs`` holds the seeded
synthetic input generators only.
"""

__all__ = ["hmg", "inputs"]
