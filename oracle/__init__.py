"""FP64 CPU oracle for the fast-hyperspectral-reconstruction hot path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The product path
(the HIP library and its Python binding) never imports, links or calls it,
and this package imports nothing from the product path.

Everything here is plain, slow and obviously correct: numpy in float64,
written from the paper's statement of each step, with no blocking, fusion
or reordering beyond what the definition states.

Modules and the passages they follow:
  normalize  -- eq. (2) -log normalisation; Appendix A offset correction
  nnls       -- non-negative least squares (the row problem of eq. (4)/(8))
  nmf        -- eq. (4) NMF: multiplicative updates, ANLS, NNDSVD init, HALS
  projector  -- the linear projection operator A of eq. (3)/(5)
  cgls       -- eq. (5) data term minimised per channel
  expand     -- eq. (6) subspace expansion; eq. (7)-(9) FMD tail
  mlp        -- learned warm start (no counterpart in the paper)
  metrics    -- relative objective, canonical factor form, SNR of eq. (11)
"""
