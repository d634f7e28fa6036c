"""Reference oracle for the exponential-free open-GRAPE gradient.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, float64 CPU
implementation written from the paper (Boutin et al., "Resonator reset in
circuit QED by optimal control for large open quantum systems").  It exists
so that the HIP path can be checked against an independent computation.  It
shares no code with the GPU library and imports nothing from it; only the
tests, the smoke check and the benchmark's CPU-baseline leg may use it.

Modules
  rk        -- the method itself: Runge-Kutta propagation of rho and of the
               adjoint lambda, cost, first-order (GRAPE1) and exact
               discrete-adjoint gradients (Secs. II.B, III; Eqs. (3)-(15)).
  superop   -- the standard method the paper replaces: Liouville-space
               superoperators and matrix exponentials (Eqs. (5)-(7)), with
               this package's own Pade scaling-and-squaring exponential and
               Van Loan's block formula for exact gradients.
  closed    -- closed forms used as pins (amplitude damping, the moment
               recursion of the driven damped resonator, steady state
               Eq. (20)).
  extensions -- Gaussian control filter (App. A) and photon-number penalty
               (Eqs. (24), (25), App. B).

Every function is pinned by a CPU test against something other than
itself; see the test files whose names start with test_oracle.
"""
