"""Plain FP64 CPU oracle of the steady-state Boltzmann SGS / preconditioned
fixed-point method (Cai, Dong, Hu, "Symmetric Gauss-Seidel Method with a
Preconditioned Fixed-Point Iteration for the Steady-State Boltzmann Equation").

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
calls this package; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it.  It shares no code, tables or
constants with the HIP path; the two meet only through the seeded input
generators in ``synth``.

Modules:
  grid        velocity grid, quadrature rules (Section 2.2; Section 4.2 setup)
  maxwellian  moments, discrete Maxwellian by Newton (eqs. moment,
              discrete_conservation, discrete_Gaussian)
  collision   Fourier-spectral collision operator, fast sigma-form and the
              sigma-exact spectral sum, steady-state correction (eq. discrete_Q)
  physical    direct physical-space quadrature of the truncated collision
              integral (eq. collision) for analytic inputs: an independent pin
  cell        inner problem (eq. inner_eqn): FP, PFP, and an independent
              theta-space Newton solve of its fixed point
  sweep       1D upwind finite volumes, diffuse walls, SGS scans, outer
              residual, mass constraint, FAS multigrid V-cycle
  mlp         small MLP forward/backward used by the learned warm start

Where a function has no independent pin it says "parity unpinned" in its
docstring.
"""
