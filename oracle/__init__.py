"""Plain FP64 CPU oracle for the SIPG multigrid hot path (Cui & Kanschat,
"Multilevel Interior Penalty Methods on GPUs").

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
runs this package; only the test suite, the smoke check and the CPU-baseline
leg of the benchmark use it.  It shares no code with the HIP path: every
matrix, index set and iteration here is rebuilt from the paper's definitions
with NumPy/SciPy in double precision.

Modules
-------
basis       Q_k Lagrange basis on Gauss-Lobatto points (Appendix A)
sipg        SIPG operator: 1-D Kronecker factors (Sec. 2.2), an independent
            quadrature assembly of the bilinear form (Sec. 2.1, eq. bilinear_form),
            and a matrix-free Kronecker apply
transfer    prolongation by canonical embedding, restriction as its transpose (Sec. 3)
patches     vertex patches, the Dirichlet local space V_j and the 2^d colouring
            (Sec. 3.1, Fig. patch_coloring)
smoother    colourised multiplicative vertex-patch Schwarz step (Alg. 1): a dense
            by-definition version and a fast-diagonalisation version (Sec. 3.2)
multigrid   V-cycle (Sec. 3), preconditioned CG, right-preconditioned GMRES and
            the fractional iteration count (Sec. 3.3)
fdsolve     global fast-diagonalisation direct solver on the brick
rhs         load vectors, interpolants and L2 errors for manufactured solutions
adjoint     closed-form / dense adjoint of the differentiable solve
"""
