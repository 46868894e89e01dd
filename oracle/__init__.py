"""Plain, slow, FP64 CPU oracle of the paper's MPM step and reduced-order
model step.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark import, call or execute anything here.  It
shares no code with the HIP library (no kernels, headers, helpers, tables or
constant generators), and nothing in the product path imports it.

Modules:
  mpm      Algorithm 1 / Algorithm 5 transfers (C core in mpm_oracle.c)
  decoder  g(X; xhat), dg/dX, dg/dxhat
  project  Algorithms 6 and 7 (velocity least squares, Gauss-Newton)
  sampler  sample-point selection (stratified, SplitMix64)
  rom      Algorithms 2 and 3, initial latents, initial-condition
           correction fields, error metrics
  train    training loss and its gradients
  encoder  the encoder network of Section 4.1 / Table 1 and its gradient

Parity status: every function above is pinned by the CPU test suite
against closed forms, invariants or brute force, except the accuracy of a
trained reduced model on a full scene, which has no closed form and is
judged against the full-order model only (parity unpinned).
"""
