"""CPU oracle for the shared-Jacobian, frequency-shifted block-sparse solve of the
implicit FNLH scheme (Wang, Weber, Radford, di Mare, Meyer: "Convergence Acceleration
of Favre-Averaged Non-Linear Harmonic Method", arXiv 2404.01407).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, FP64/complex128 NumPy
statement of what the GPU library computes.  Only the test-suite, the smoke check and
the CPU-baseline leg of the benchmark may import it; the product path never does.  It
shares no code with the GPU library: it takes meshes, states, right-hand sides and
colour orderings as plain arrays.

Modules
-------
flux       Euler + Spalart-Allmaras convective flux and its analytic Jacobian, the
           Rusanov spectral radius (stand-in for the paper's first-order approximate
           Jacobian, section "Generalized RK Scheme for The Mean Flow").
assemble   First-order residual Jacobian J, its diagonal part P and the implicit /
           explicit preconditioner matrix K (equation for K in the same section).
ordering   Colour classes (independent sets) that define the ILU ordering.
solve      Frequency-shifted systems K + i omega V I (section "Generalized RK Scheme
           for Time-Linearized Harmonic Flows"), block Jacobi / SGS / DILU / ILU(0)
           preconditioners and the iterative inexact solve of section "Solution Update";
           dense direct solves used as pins.
precision  Round-to-nearest-even storage rounding (FP32, BF16) of matrix blocks.
learned    Reference forward / backward / Adam of the per-edge message-passing
           preconditioner (a project addition, not in the paper).

Pins: every function is checked in tests/test_oracle_*.py against facts fixed by the
paper or by mathematics (dense solves, closed forms, homogeneity, complex-step
derivatives, omega = 0 and conjugate symmetry, the real 2x2 block form of the complex
system, ILU(0) defining property, brute-force dense iterates, finite differences).
Parity unpinned: the paper's end-to-end numbers (speed-ups, memory table), which need
the industrial solver and meshes.
"""
