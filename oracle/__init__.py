"""CPU oracle for the vielbein lattice-Boltzmann hot path (TEST INFRASTRUCTURE ONLY).

This package is a plain, slow, high-precision / FP64 restatement of the method of
Busuioc & Ambrus (arXiv:1708.05944): vielbein lattice-Boltzmann models for flows in
curvilinear geometries.  It exists only so
that tests, the smoke check and the CPU-baseline leg of the benchmark can check the
HIP library against an independent implementation.

Rules that keep it independent:
  * nothing in the product package (``paper_1708_05944_amd``) imports, links or runs
    anything from here, and nothing here imports the product package (the seeded
    workload generators in ``paper_1708_05944_amd.workloads`` hold no method
    arithmetic and are the one shared module);
  * quadrature tables are built here in arbitrary precision (mpmath) from the
    paper's formulas; the library builds its own in long double by a different
    route (discretised Stieltjes), so the two share no table generator;
  * the time stepper is plain C (``couette_oracle.c``) with FP64 loops in the
    paper's order of operations, compiled with ``-ffp-contract=off``.
"""
