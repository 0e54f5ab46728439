"""FP64 CPU oracle of the lensless RF volumetric render (GeRaF, arXiv 2605.29097).

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the benchmark's
CPU-baseline leg import this package; the product package never does, and this
package never imports the product package.  The GPU path and this oracle share
nothing but the seeded input generators of the ``synth`` module.

Modules:
  render    signal tracing, matched filter, loss and their adjoints (C core + numpy)
  mlp       SDF network forward / gradient / double backward (torch float64, CPU)
  sampling  lensless primary-ray sampling and its counter-based generator
  optim     AdamW with cosine schedule (numpy)
"""
