"""MI355X (gfx950) shifted solves for the Hermitian Wilson-Dirac operator.

The compute path is the HIP library ``libqmg.so`` (C interface in
``include/qmg.h``); ``paper_2004_08146_amd.qmg`` is a thin ctypes binding with
the same names.  Importing the binding raises if the library is not built.
"""
