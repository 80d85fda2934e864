"""MI355X (gfx950) implementation of the hot path of Power Bundle Adjustment
(Weber, Demmel, Chan, Cremers, arXiv 2204.12834): the power-series solve of
the reduced camera system inside each Levenberg-Marquardt step, with the
residual / Jacobian evaluation and the damped block inverses that feed it.

The computation lives in libpoba.so (HIP, C ABI in include/poba.h); the
Python side only marshals arguments.  `synth` generates seeded synthetic
scenes.
"""

__all__ = ["solver", "synth"]


def __getattr__(name):
    if name in ("solver", "Problem", "LMOptions", "project"):
        from . import solver
        return solver if name == "solver" else getattr(solver, name)
    raise AttributeError(name)
