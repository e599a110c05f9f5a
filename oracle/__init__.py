"""Plain FP64 CPU oracle for IRLS + PCG L1 phase unwrapping.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library
and its Python binding) may import, call or link this package; only the
tests, the smoke check and the CPU-baseline leg of the benchmark do.  It
shares no code with the GPU path: the only common module is ``synth``
(seeded inputs, none of the method's arithmetic).

Layout and notation follow the paper (arXiv 2401.09961):

* ``reduced``  -- the weighted 5-point form D^T Omega D U = D^T Omega G that
  the GPU path implements (the augmented system of Proposition 1 with the
  slack variables eliminated), IRLS weights C / max(|DU - G|, eps).
* ``paper_form`` -- Algorithm 1 and Algorithm 2 verbatim in (U, V^v, V^h)
  with tau, delta and the block-diagonal preconditioner of Section 3.3.
* ``schedule`` -- the adaptive CG-iteration rule of Section 4.3.

Everything is numpy/scipy in float64, written for readability, not speed.
Parity status of every function is listed in each module's header; the
one result with no independent pin ("parity unpinned") is the pointwise
U of non-Itoh problems, whose minimiser need not be unique.
"""
from . import reduced, paper_form, schedule  # noqa: F401
