"""MI355X (gfx950) Gaussian Mesh Renderer: forward and backward of the mesh-to-Gaussian splatting
rasteriser as hand-written HIP kernels behind the C ABI of include/gmr.h (libgmr.so).

Importing the package loads libgmr.so and fails if it has not been built; there is no fallback.
"""
# torch first: libgmr.so then binds to the HIP runtime torch has already loaded, so the library
# and torch's allocator and streams share one runtime (loading the library first pulled in a second
# runtime, which found no device)
import torch  # noqa: F401

from . import _lib
from ._lib import GMRError, gmr_options

_lib.load()

from .render import (Batch, GraphAdamLoop, GraphStep, Handle, MeshGraph, ReconLoop, ReconWeights, Renderer,  # noqa: E402
                     adam_step, copy_options, default_options, options_dict, render, vector_adam_step)

__all__ = ["Batch", "GraphAdamLoop", "GraphStep", "Handle", "MeshGraph", "ReconLoop", "ReconWeights", "Renderer", "adam_step",
           "copy_options", "default_options", "options_dict", "render", "vector_adam_step", "GMRError",
           "gmr_options"]
