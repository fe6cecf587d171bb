"""FP64 CPU oracle for the local graph-diffusion solvers -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the GPU library
``paper_2410_21634_amd`` and never imports it.

* :mod:`oracle.solvers` -- ctypes wrapper of ``gde_oracle.c`` (step-by-step
  LocalGD, LocalCH, FIFO push (APPR / AKatz / LocalSOR), HK level push and the
  replay checker).
* :mod:`oracle.exact`   -- dense / global FP64 references (closed forms,
  truncated series, eigenvalue bounds) written with numpy / scipy.
"""
