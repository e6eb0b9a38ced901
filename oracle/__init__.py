"""Plain FP64 CPU oracle of the relativistic particle-mesh step.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The product path (the
HIP library and its Python binding) never imports, links or calls it, and this
package shares no code with that path.

Modules:
  pm   -- background, CIC deposit, metric solves, gather/kick/drift, step driver
  pk   -- matter power spectrum estimator
  cnn  -- the 3-layer 3D convolutional closure (forward, backward, Adam) in FP64
"""
