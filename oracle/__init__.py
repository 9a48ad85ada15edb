"""ORACLE -- test infrastructure only.

A plain, slow, obviously correct FP64 CPU implementation of the SDME high-order
FEM hot path (arXiv 2104.13466): the 1D bases of Section 2 (``basis``), direct
element loops for the weak-form operators of Section 3 (``fem``, plain C), and
textbook drivers for PCG, Newton, Newmark and central differences of Section 4
(``solvers``).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import, call, link or execute anything in this package.  It
shares no code with the HIP library and never imports it.
"""
