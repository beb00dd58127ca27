"""CPU oracle for diagonally-addressed (DA) CSR storage and its products.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only the tests, the smoke check and the benchmark's CPU-baseline leg do.  It
shares no code with the HIP library (no kernels, headers, helpers or tables);
the two meet only at the seeded inputs of the `workloads` package.

Everything is plain NumPy in float64 unless a function states otherwise, and
follows the paper's definitions in the order the paper states them:

storage   -- CSR checks, bandwidth (Eq. 2), the DA transform col - row
             (Sec. 2, Example 1), symmetric permutation, encode/decode.
rcm       -- reverse Cuthill-McKee with a George-Liu pseudo-peripheral start
             (the paper cites RCM in Sec. 2 and Sec. 3 but does not fix its
             details; the reading implemented here is documented there).
spmv      -- y <- alpha*A*x + beta*y (Sec. 4) for CSR and DA-CSR, and its
             multi-vector form.
traffic   -- the matrix traffic model (Eq. 3), the work count W, and the
             traffic ratios of Fig. 3.
cg        -- conjugate gradients in float64 and a float32-inner iterative
             refinement scheme (the multi-precision remark of Sec. 2).
mlp       -- a small multilayer perceptron (forward, loss, backward, update)
             used to pick kernel variants from sparsity features.
features  -- the sparsity features that selector consumes.

Pins: every function is checked in tests against values the paper prints,
closed forms, library routines or brute force; see the oracle tests.
"""
