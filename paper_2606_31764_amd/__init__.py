"""MI355X-native NURBS Splatting render path (sample -> bin -> composite and its adjoint).

The kernels live in ``libnsplat.so`` (HIP for gfx950, built by ``build.py``);
``render`` wraps its C ABI for PyTorch tensors and ``synth`` draws seeded
workloads shaped like the paper's.
"""
from . import synth  # noqa: F401

__all__ = ["synth", "render", "build"]
