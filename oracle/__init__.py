"""Plain FP64 CPU oracle for randomized far-field compression.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import this package:
only the test suite, the smoke check and the CPU-baseline leg of the benchmark
use it. It shares no code with the GPU library (no kernels, headers, helpers or
tables); the only thing both sides consume is the seeded input generator
module, which holds no arithmetic of the method.

Everything here is written for obviousness rather than speed: numpy float64,
no blocking or fusion beyond what the definitions state, one function per
step of the method of March & Biros, "Far-Field Compression for Fast Kernel
Summation Methods in High Dimensions":

  kernels     Gaussian, Laplace and polynomial kernels (Section 4.2-4.4)
  direct      direct kernel summation u = Kq (Section 1, eq. e:sum)
  sampling    counter-based uniform row sampling without replacement
              (Section 4.1.3, uniform sampling; Theorem thm_column_sampling_approx2)
  cpqr_id     interpolative decomposition via column-pivoted QR
              (Section 2.1.3, Definition of the ID, Theorem thm_compute_id;
              Appendix 6.1)
  tree        binary ball tree used to group the points (Section 2)
  skeleton    per-node sampled ID with nested skeletons (Section 2.2)
  evaluate    equivalent charges and far-field application (eq. e:id)
  leverage    statistical leverage scores (Section 3, Definition of leverage)
  theory      closed forms: Silverman bandwidth, sampling bounds (Section 3, 4.2)
  proposal    features, MLP and weighted sampling for the learned proposal

Functions whose result has no independent pin say "parity unpinned" in their
docstring.
"""
