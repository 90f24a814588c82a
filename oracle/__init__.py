"""Plain, slow, FP64 CPU reference implementation of spaQR (Gnanasekaran & Darve,
"Hierarchical Orthogonal Factorization: Sparse Square Matrices").

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package; only the tests, the smoke check and the benchmark's CPU-baseline leg
do.  It shares no code with the GPU engine: its ordering, symbolic analysis,
factorization, apply and GMRES are written independently here, in Python and
NumPy, following the paper's steps in the paper's order.

Modules
  ordering  geometric modified nested dissection with interfaces (Sections 2.3, 4)
  spaqr     factorization (Algorithm 2: Sections 2.4-2.8) and the apply of
            Q^T and W^{-1}
  gmres     right-preconditioned flexible GMRES (Section 4)
  cpqr      partial column-pivoted Householder QR with the ratio rank rule

Every function is pinned by tests under tests/ against values fixed by the
paper or by mathematics (exact factorization at eps = 0, dense QR, LAPACK
routines, brute force on small grids); see the test files for the pins.
"""
