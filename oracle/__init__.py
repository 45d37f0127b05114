"""CPU oracle for the nested MLMC hot path (Haas & Giles, "A nested MLMC framework
for efficient simulations on FPGAs", 2025).

TEST INFRASTRUCTURE ONLY.  Nothing in the library imports, links or calls this
package; only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark do.  It shares no code, tables or constants with the HIP path: every
value here is recomputed from the paper's definitions (mpmath / scipy / exact
integers / numpy with per-operation rounding), slowly and in the paper's order.

Modules
  philox      Philox4x32-10 block function and the counter layout of the uniform
              integers J of Section 3 (the paper names no generator).
  normal      U = 2^-D (J + 1/2), the exact inverse normal Phi^-1(U), and the
              Method-1 piecewise-constant table (Section 3.1).
  fixedpoint  fixed-point values (-1)^s 2^(e-d) n with round-to-nearest and
              saturation (Section 4.1), as exact integer arithmetic.
  paths       coupled fine/coarse Euler-Maruyama (Section 2.1, Algorithm 1) and
              Milstein GBM paths in FP64 / FP32 / FP16 / fixed point, payoffs.
  rngmethods  Methods 2 (sum of two small-table variables, least squares under a
              permutation, permuted coupled uniform) and 3 (piecewise linear on
              dyadic intervals) of Section 3.
  errmodel    rounding-error model of Sections 4-6: reverse-sweep sensitivities,
              V_indep / V_corr and their approximate-normal extension, the
              separable cost, Lagrange widths by golden-section search and the
              greedy integer rounding.
  mlmc        per-level sums, the nested split (Section 2.2), optimal sample
              allocation (Sections 2.1-2.2) and the adaptive driver.

Readings where the paper is silent are named R1..R23 in the docstrings; each is
listed in the repository's design notes.
"""
