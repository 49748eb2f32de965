"""FP64 CPU oracle for MN-BaB bounding (test infrastructure only).

This package is the reference against which the GPU path is checked.  Only the
test-suite, the smoke entry point and the benchmark's CPU-baseline leg may use
it; the product path never imports it.  It is written from the paper
(Ferrari et al., ICLR 2022, arXiv 2205.00263), Section 3, plainly and slowly,
in float64 numpy, with scipy only for the LP / convex-hull cross-checks.

Modules
    net      -- network arithmetic: affine maps, their adjoints, forward pass, IBP
    backsub  -- back-substitution (Eq. 2 and Eq. 5), concretisation (Eq. 6), x*
    optimize -- DeepPoly root pass, parameter sets, analytic gradient, Adam
    bab      -- branch_split, branching score, BaB loop
    lp       -- LP of the same relaxation (weak / strong duality pins)
    enum     -- exact minimum by activation-pattern enumeration
    mnc      -- exact 3-neuron ReLU hull constraints (MNC input data)
    cost     -- the split-cost model of Appendix B
    branching -- active constraint score and cost adjusted branching (Section 3.4)
"""
from . import net, backsub, optimize, bab, lp, enum, mnc, cost, branching  # noqa: F401
