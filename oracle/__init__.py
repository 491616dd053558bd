"""CPU FP64 oracle for the Wilson-Dirac hopping term and the solvers around it.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import this
package: only the tests, the smoke check of the graft entry point and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP path
(it imports nothing from the ``paper_0710_2442_amd`` package), and the HIP
path never calls it.

Every routine is plain numpy in float64/complex128 (except the routines that
explicitly emulate a lower storage precision) and follows the paper's
definitions without blocking or fusion:

* ``gamma``       -- the Dirac matrices (an explicit chiral basis; the paper
                     leaves the basis open).
* ``wilson``      -- Eq. 3 (hopping term), D_W = 1 - kappa*H, parity-restricted
                     hops, the even-odd Schur operator, a dense brute-force
                     matrix and a per-site evaluation for sampled checks.
* ``free_field``  -- unit-link closed forms: plane-wave action, spectrum and
                     the momentum-space solution of D x = b.
* ``solvers``     -- CG on the normal equations (full and even-odd), FP64
                     defect correction with an emulated low-precision inner
                     solve, flexible GCR with a plain-CG fallback.
* ``ptc``         -- the gauge-covariant parallel-transport convolution
                     network: forward, analytic backward, loss and Adam.
* ``perf_model``  -- the paper's linear timing model (Eqs. 1-2) and its
                     Table 1 arithmetic.
* ``blas``        -- the caxpy / inner products of Sec. 4 written out.

Routines whose result has no independent pin say "parity unpinned" in their
docstring.
"""
