"""Plain, slow FP64 CPU oracle for the SIPG-DG Poisson method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package: only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg
of ``bench.py`` use it.  It shares no code, tables or constants with the HIP
library in ``paper_2407_09621_amd``; both sides only share the seeded input
generators in ``paper_2407_09621_amd.inputs`` (random numbers, no method
arithmetic).

Contents (each module cites the passage of Cui, "Acceleration of
Tensor-Product Operations with Tensor Cores", arXiv 2407.09621, it follows):

* ``basis1d``   - GLL nodes, Gauss rules, Lagrange basis, 1D mass/stiffness
                  (Sec. 2 and 2.1).
* ``sipg``      - the SIPG matrix assembled by 3D/2D quadrature straight from
                  the bilinear form (Sec. 2, eq. bilinear_form), and a second,
                  independent derivation through the Kronecker-sum identity on
                  Cartesian meshes (Sec. 2.1, eq. tensorproduct_3d).
* ``mapped``    - the SIPG matrix on trilinear hexahedra (general geometry:
                  mapped cell integrals with per-point Jacobians, Sec. 2.1,
                  and physical face normals), by quadrature cell by cell.
* ``rhs``       - right-hand side and L2 error by tensor Gauss quadrature
                  (Sec. 7.2 manufactured solution).
* ``multigrid`` - transfers, multiplicative vertex-patch smoother with dense
                  patch solves, coarse solve, V-cycle (Sec. 7.1, Alg. v_cycle).
* ``fgmres``    - right-preconditioned flexible GMRES with modified
                  Gram-Schmidt (Sec. 7.1, 7.2).
* ``learned``   - the learned correction stage of this project (not in the
                  paper): grid mapping of DG coefficients, 3D convolutions,
                  ReLU, masked MSE and their exact gradients, Adam, the
                  solver-generated training pairs and the learned
                  preconditioner with its fallback rule.

Readings of passages the paper leaves open are listed in each function's
docstring.  Parity pins for each function live in ``tests/test_oracle_*.py``.
"""
