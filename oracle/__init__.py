"""Plain, slow FP64 CPU oracle for H-LU preconditioned GMRES on lowest-order
Nedelec discretisations of the time-harmonic Maxwell equations
(Parvizi, Khodadadian, Beuchler, Wick: "Hierarchical LU preconditioning for
the time-harmonic Maxwell equations", arXiv 2211.11303).

THIS PACKAGE IS TEST INFRASTRUCTURE. Only the test suite, the smoke check and
the CPU-baseline leg of the benchmark may import it. The product path (the
HIP library and its Python binding) never imports, links or calls anything
here, and nothing here imports the product path: the two share no code.

Modules, in the order of the method:

* ``mesh``      -- Kuhn-split cube mesh, interior edges (the unknowns), edge
                   midpoints (Sec. 2.1, Example 1 of Sec. 4).
* ``assemble``  -- Whitney edge basis, exact element integrals, the Galerkin
                   matrix ``A = K - kappa^2 M`` (eq. (5), eq. (8)).
* ``cluster``   -- geometric bisection cluster tree and eta-admissible block
                   tree (Sec. 3, Definition 1; eta = 2 as in Sec. 4).
* ``hmatrix``   -- H-matrix storage, truncated low-rank addition (truncated
                   SVD, Sec. 4), H-matrix products, H-LU factorisation
                   (Algorithm 1, step II) and H-triangular solves
                   (Algorithm 1, step III).
* ``hinverse``  -- approximate inverse B_H of the H-matrix by the Schulz
                   iteration in H-arithmetic (Sec. 3; truncated SVD, Sec. 4),
                   used as a preconditioner (Example 2).
* ``krylov``    -- preconditioned restarted GMRES (Sec. 4, Example 1) and the
                   preconditioned Richardson iteration of Algorithm 1, step III.

Every floating-point computation here is FP64.
"""
