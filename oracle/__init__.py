"""Oracle for the linear lattice Boltzmann acoustic scheme (arXiv:1704.03172).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark may import, call, link or execute anything
in this package.  The product (the HIP library and its Python binding) never
imports it and shares no code with it.

Contents
  lb_oracle.c / lb_oracle.py  plain FP64 time stepping of the recurrence
                              (C loops, OpenMP over rows) and its Python
                              driver: moments, weights, equilibrium,
                              BGK/MRT collision, source, sponge, periodic
                              streaming, receivers, sum of rho.
  refine.py                   coarse/fine grid-refinement composite stepping
                              (Sec. IV) built on the grid driver.
  dispersion.py               Fourier-space update operator and closed-form
                              dispersion relations (Sec. III, Appendix E).
  analytic.py                 analytic 2D solution for a point source
                              (eq. exact solution) in the time domain.

Parity status per function is listed in each module header; nothing here is
"parity unpinned" except where a module header says so.
"""
