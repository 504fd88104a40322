"""FP64 CPU oracle for the explicit spectral-cell (SCM) wave step.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package.  The product path (the HIP library and
its Python binding) never imports it, and this package never imports the product
path: the two share nothing but the seeded input generators in ``workloads``.

Every function is a plain, slow, direct transcription of the mathematics, in float64,
with numpy/scipy primitives (matmul, eigh, eigsh) as its only building blocks.  Each
cites the passage of the paper it follows (section / equation / algorithm):

* ``basis``      - GLL/GL points and weights, 1-D Lagrange polynomials (Sec. 2.2).
* ``element``    - element stiffness and mass integrands, uncut reference cell,
                   isotropic elasticity by B^T D B (Sec. 2.2; elasticity is textbook).
* ``geometry``   - the indicator alpha^FCM and cell classification (Sec. 2.2).
* ``quadrature`` - space-tree quadrature of cut cells (Sec. 2.2).
* ``stabilize``  - eigenvalue (epsilon) stabilisation and HRZ lumping (Sec. 2.4, 2.6).
* ``problem``    - assembly of the whole discrete problem and the point load.
* ``timestep``   - critical time step, central differences with the Newmark start-up,
                   discrete energy (Sec. 2.3, eq. cdm, Alg. newmark).
* ``imex``       - the Newmark IMEX scheme: explicit/implicit DOF split, consistent
                   cut-DOF mass, trapezoidal Newmark on the cut DOFs (Sec. 2.5, Alg. imex).

Readings of the paper where it is silent are stated in the functions that take them.
Parity status: every function here is pinned by tests under ``tests/test_oracle_*``;
the choices that the paper does not fix (EVS threshold, lumping of a stabilised cut
cell, tree depth, point source) are pinned only by invariants, not by paper values.
"""
