"""FP64 CPU oracle for the shifted Wilson-Dirac solve -- TEST INFRASTRUCTURE.

This package is a plain, slow, direct NumPy transcription of the paper's
definitions (Frommer et al., "A multigrid accelerated eigensolver for the
Hermitian Wilson-Dirac operator in lattice QCD", arXiv:2004.08146).  It is
used only by ``tests/``, by ``__graft_entry__.smoke()`` and by the
``cpu_baseline`` leg of ``bench.py``.  The product path (the HIP library
and its Python binding) never imports it, and it imports nothing from the
product path.

All arithmetic is complex128.  Fields use the canonical layout documented in
``synth.fields``.  Pins tying every function to something other than itself
live in ``tests/test_oracle_*.py``; a function whose exact values had no such
pin would say "parity unpinned" in its docstring (none does).
"""
