"""Plain CPU FP64 / multiprecision oracle for the BURA method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package: only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark call it.  It shares no code with the HIP library; the only module
both sides use is the seeded input generator package ``synth``, which holds no
arithmetic of the method.

Contents (each file cites the passage of Harizanov, Lazarov, Marinov,
Margenov, Vutov, "Optimal solvers for linear systems with fractional powers
of sparse SPD matrices" (arXiv:1612.04846) that it follows):

* ``remez``    -- best uniform rational approximation r_alpha^beta of
                  t^(beta-alpha) on [0,1] by the modified Remez algorithm
                  (Section 3.2, Algorithm 1) in the Chebyshev basis of
                  eq. (eq1bua), and its partial-fraction form eq. (eq:simplified).
* ``operators``-- the scaled SPD grid matrices (Section 5.3 five-point
                  Laplacian, its 7-point 3D analogue and a variable-coefficient
                  flux-form variant) as scipy.sparse matrices, and the
                  spectral bound of eq. (algebraic).
* ``spectral`` -- exact A^-alpha f (eq. eqn:exacalg) and the BURA result
                  u_r = sum_j c_j (A - d_j I)^-1 f evaluated in the closed-form
                  sine eigenbasis of the constant-coefficient Laplacian.
* ``shifted``  -- u_r by k+1 shifted sparse solves, eq. (eq:Rgeneral).
* ``metrics``  -- relative errors and the error-lemma norms of eq. (12) (Lemma 2.1).
* ``multistep`` -- the multi-step BURA of Section 4.4 (sequential 1-BURA
                  steps) and its eigenvector errors.
* ``product``  -- the zero-pole product form of the remark in Section 2.2
                  (zeros, leading constant, factor-by-factor evaluation).
* ``quadrature`` -- the sinc quadrature u_Q of Bonito and Pasciak that
                  Section 5.3 compares the BURA against (its weights, shifts and
                  term counts), and its closed-form eigenbasis evaluation.
"""
