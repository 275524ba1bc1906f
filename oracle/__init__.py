"""CPU oracle for the coarse Dirac operator S_bb = D_bb - D_br D_rr^{-1} D_rb.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import, call or link anything in this
package.  The product (the HIP library and its Python binding) never does,
and the two share no code.

Two tiers:

* ``oracle.dense``   -- O1, dense numpy/LAPACK in FP64 on tiny lattices:
  builds the Wilson-Dirac matrix entry by entry, permutes it (section 2,
  Permutation_block), partitions it into the 2x2 block form (section 1, step 1)
  and forms S_bb by a dense LU solve (section 1, the Schur complement formula).
* ``oracle.matfree`` -- O2, a plain C + OpenMP FP64 matrix-free stencil with a
  textbook restarted GCR for D_rr, for lattices too large for dense algebra.
  Built by ``oracle/build.py`` with gcc into ``oracle/liboracle.so``.
* ``oracle.ptc``     -- the gauge-covariant convolution network used as a
  preconditioner (forward, analytic Wirtinger backward, finite differences).
"""
