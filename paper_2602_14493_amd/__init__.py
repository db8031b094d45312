"""MI355X (gfx950) Gaussian Mesh Renderer: forward and backward of the mesh-to-Gaussian splatting
rasteriser as hand-written HIP kernels behind the C ABI of include/gmr.h (libgmr.so).

Importing the package loads libgmr.so and fails if it has not been built; there is no fallback.
"""
from . import _lib
from ._lib import GMRError, gmr_options

_lib.load()

from .render import (Batch, GraphAdamLoop, Handle, MeshGraph, ReconLoop, ReconWeights, Renderer,  # noqa: E402
                     adam_step, copy_options, default_options, options_dict, render, vector_adam_step)

__all__ = ["Batch", "GraphAdamLoop", "Handle", "MeshGraph", "ReconLoop", "ReconWeights", "Renderer", "adam_step",
           "copy_options", "default_options", "options_dict", "render", "vector_adam_step", "GMRError",
           "gmr_options"]
