"""CPU reference implementation ("oracle") of the DtN / Jacobian hot path.

TEST INFRASTRUCTURE ONLY: only tests/, the smoke check and the CPU-baseline leg of
the benchmark may import it.  The product path (paper_1210_5672_amd) never does,
and the two share no code.

  ww_oracle.py : FP64 reference (numpy, numpy.fft, scipy LU), every function cites
                 the passage of the paper it follows.
  xprec.py     : the same reference run in 34-digit mpmath arithmetic, to measure
                 the FP64 rounding floor on small problems.
  mesh_oracle.py : the non-uniform mesh x = xi(alpha) and the time segments with
                 regridding (Sec. 2.2 eq. (xi), (rho:def)), pinned by
                 tests/test_mesh_oracle.py.
  sdc_oracle.py : the SDC15 time stepper (Radau IIa nodes, RK4 predictor, Picard
                 sweeps; Sec. 2.2), pinned by tests/test_sdc_oracle.py.

Parity status: every function is pinned by tests/test_oracle_pins.py (closed forms,
printed linear periods, invariants, central differences, extended precision).
"""
