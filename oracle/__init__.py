"""Plain, slow, obviously-correct FP64 CPU oracle for the adaptive-ROM hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, links or
executes anything in this directory; only the test-suite, the smoke check and
the CPU-baseline leg of the benchmark call it.  It shares no code with the HIP
library: the only inputs both sides see come from the seeded generators in
``paper_2605_28684_amd.workloads``, which hold none of the method's arithmetic.

Modules
  fom      full-order model: fluxes, residual f(q), backward-Euler residual,
           exact Jacobian (complex step), Newton solve (paper Sec. 2, eq.
           fom_lmm; App. B; Burgers setup of Sec. 5.1)
  riemann  exact Riemann solver for the Sod pin (Toro, ch. 4)
  rom      preprocessing, POD, iSVD (Alg. 2), greedy DEIM, rebuild, Galerkin and
           hyper-reduced LSPG steps, state transfer, and the Alg. 1 driver
  react    the synthetic stiff ten-species advection-reaction model
"""
