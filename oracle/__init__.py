"""CPU FP64 oracle for Power Bundle Adjustment (Weber, Demmel, Chan, Cremers,
"Power Bundle Adjustment for Large-Scale 3D Reconstruction", arXiv 2204.12834).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only the tests, the smoke check and the CPU-baseline leg of
the benchmark use it.  It shares no code with the HIP library and imports
nothing from the product package.

It is a plain, slow, obviously-correct NumPy implementation in float64 of what
the hot path computes, one module per stage of a Levenberg-Marquardt iteration:

  camera   residuals r_i and Jacobian blocks J_p (2x9), J_l (2x3)  (Sec. 4, 4.1)
  robust   Huber loss and its IRLS weights (an extension; not in the paper)
  normal   block-diagonal U, V, right-hand sides b_p, b_l, damping  (Sec. 4.1,
           eq. normal)
  schur    matrix-free W / W^T products, reduced right-hand side, power-series
           solve with the stop rule, back-substitution  (Sec. 4.2, 4.3, eqs.
           Schur, S_approx, x_approx, qcriterion, back_substitution)
  dense    dense H, S, P and spectral quantities for tiny problems
           (Sec. 3 Prop. 1, Sec. 4.3 Lemma 1 and Prop. 2)
  lm       the Levenberg-Marquardt outer loop (Sec. 5.1 "LM loop")
  adjoint  implicit differentiation of one damped step (an extension)

Readings taken where the paper is silent or garbled are listed in each
function's docstring.
"""
from . import camera, robust, normal, schur, dense, lm, adjoint  # noqa: F401
