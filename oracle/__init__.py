"""FP64 CPU oracle for the Tucker discrete-velocity S-model step.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, independent
reference the HIP path is checked against.  Only the test-suite, the smoke
check and the bench's CPU-baseline leg may import it; the product path
never calls it and shares no code with it (the two only take the same
seeded inputs from `synth`).

Two levels, both written from the paper (Chikitkin, Kornev, Titarev,
"Numerical solution of the Boltzmann equation with S-model collision
integral using tensor decompositions"):

  O1  `dvm.step_full`    - the plain definition: full N^3 tensors, the
                           discrete velocity method (Alg. 1, Alg. 2), then
                           truncated HOSVD by LAPACK SVDs of the unfoldings.
  O2  `tucker_dvm.step`  - the same step in Tucker form: moments by
                           convolution (Op5), the low-rank S-model
                           equilibrium, flux terms by Hadamard products and
                           sums (Op3, Op2) and one rounding (Op4) per cell.

Readings of points where the paper is silent or garbled are listed in the
module docstrings where they are used.  Parity unpinned: the rank-6 face
estimate of |xi.e| on oblique faces (the paper gives no construction and
its figure is missing); it is pinned only by the HOSVD error bound.
"""
