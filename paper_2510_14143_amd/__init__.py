"""MI355X (gfx950) Richardson-Lucy deconvolution: HIP kernels behind a C ABI.

`rl` is the binding of include/rl.h (librlmi.so, built by `build`), `synth`
draws seeded synthetic input volumes.
"""
from . import rl  # noqa: F401
from .rl import BatchPlan, Plan, RLError  # noqa: F401
