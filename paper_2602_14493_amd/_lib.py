"""ctypes binding of libgmr.so: the C ABI declared in include/gmr.h, same names, argument
marshalling only.  Loading fails loudly when the library has not been built -- there is no
fallback implementation."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgmr.so")

c_float, c_int32, c_int64, c_size_t, c_void_p = ctypes.c_float, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_void_p

GMR_OK, GMR_ERR_INVALID_ARG, GMR_ERR_WORKSPACE, GMR_ERR_CAPACITY, GMR_ERR_UNSUPPORTED, GMR_ERR_HIP = range(6)
NOALLOC_WORKSPACE_BYTES = 64 << 20   # GMR_NOALLOC_WORKSPACE_BYTES of gmr.h


class gmr_camera(ctypes.Structure):
    _fields_ = [("R", c_float * 9), ("t", c_float * 3), ("fx", c_float), ("fy", c_float), ("cx", c_float),
                ("cy", c_float), ("width", c_int32), ("height", c_int32), ("near_plane", c_float),
                ("far_plane", c_float)]


class gmr_options(ctypes.Structure):
    _fields_ = [("cov_mode", c_int32), ("dilation", c_float), ("alpha_min", c_float), ("alpha_max", c_float),
                ("t_eps", c_float), ("bg", c_float * 3), ("tile_w", c_int32), ("tile_h", c_int32),
                ("raster_mode", c_int32), ("px_per_lane", c_int32), ("lane_lists", c_int32),
                ("sh_degree", c_int32), ("composited_lists", c_int32), ("instance_capacity", c_int64)]


class gmr_batch(ctypes.Structure):
    _fields_ = [("num_meshes", c_int32), ("num_views", c_int32), ("vert_offsets_host", c_void_p),
                ("face_offsets_host", c_void_p), ("view_mesh_host", c_void_p), ("cams_host", c_void_p)]


class gmr_counters(ctypes.Structure):
    _fields_ = [("instances", c_int64), ("capacity", c_int64), ("overflow", c_int32), ("overflow_any", c_int32),
                ("pairs_fwd", c_int64), ("pairs_bwd", c_int64), ("loss", c_float), ("loss_sil", c_float),
                ("peak_instances", c_int64)]


# name -> (restype, argtypes)
_SIGS = {
    "gmr_default_options": (gmr_options, []),
    "gmr_create": (c_int32, [ctypes.POINTER(c_void_p), c_int32]),
    "gmr_destroy": (c_int32, [c_void_p]),
    "gmr_status_string": (ctypes.c_char_p, [c_int32]),
    "gmr_last_error": (ctypes.c_char_p, []),
    "gmr_view_table_size": (c_int32, [ctypes.POINTER(gmr_batch), ctypes.POINTER(gmr_options), ctypes.POINTER(c_size_t)]),
    "gmr_view_table_fill": (c_int32, [ctypes.POINTER(gmr_batch), ctypes.POINTER(gmr_options), c_void_p, c_size_t]),
    "gmr_workspace_size": (c_int32, [ctypes.POINTER(gmr_batch), ctypes.POINTER(gmr_options), ctypes.POINTER(c_size_t),
                                     ctypes.POINTER(c_size_t)]),
    "gmr_build_adjacency": (c_int32, [c_void_p, c_int64, c_int64, c_void_p, c_void_p]),
    "gmr_render_fwd": (c_int32, [c_void_p, ctypes.POINTER(gmr_batch), ctypes.POINTER(gmr_options), c_void_p,
                                 c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t,
                                 c_void_p]),
    "gmr_render_fwd_noalloc": (c_int32, [c_void_p, ctypes.POINTER(gmr_batch), ctypes.POINTER(gmr_options), c_void_p,
                                         c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                         c_void_p]),
    "gmr_render_bwd": (c_int32, [c_void_p, ctypes.POINTER(gmr_batch), ctypes.POINTER(gmr_options), c_void_p,
                                 c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                 c_int32, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "gmr_render_bwd_l2": (c_int32, [c_void_p, ctypes.POINTER(gmr_batch), ctypes.POINTER(gmr_options), c_void_p,
                                    c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_float, c_void_p, c_void_p,
                                    c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "gmr_render_step_l2": (c_int32, [c_void_p, ctypes.POINTER(gmr_batch), ctypes.POINTER(gmr_options), c_void_p,
                                     c_void_p, c_void_p, c_void_p, c_void_p, c_float, c_void_p, c_void_p, c_void_p,
                                     c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "gmr_render_step_recon": (c_int32, [c_void_p, ctypes.POINTER(gmr_batch), ctypes.POINTER(gmr_options), c_void_p,
                                        c_void_p, c_void_p, c_void_p, c_void_p, c_float, c_void_p, c_float, c_void_p,
                                        c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                        c_void_p, c_size_t, c_void_p]),
    "gmr_render_bwd_recon": (c_int32, [c_void_p, ctypes.POINTER(gmr_batch), ctypes.POINTER(gmr_options), c_void_p,
                                       c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_float, c_void_p, c_float,
                                       c_void_p, c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                                       c_size_t, c_void_p]),
    "gmr_workspace_view": (c_int32, [ctypes.POINTER(gmr_batch), ctypes.POINTER(gmr_options), ctypes.POINTER(c_size_t),
                                     ctypes.POINTER(c_size_t), ctypes.POINTER(c_size_t), ctypes.POINTER(c_size_t)]),
    "gmr_read_counters": (c_int32, [c_void_p, c_size_t, ctypes.POINTER(gmr_counters), c_void_p]),
    "gmr_profile_enable": (c_int32, [c_void_p, c_int32]),
    "gmr_profile_read": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p]),
    "gmr_adam_step": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_int64, c_float, c_float, c_float, c_float,
                                c_void_p, c_void_p]),
    "gmr_mesh_graph_size": (c_int32, [c_void_p, c_int64, c_int64, ctypes.POINTER(c_int64)]),
    "gmr_build_mesh_graph": (c_int32, [c_void_p, c_int64, c_int64, c_int64, c_void_p, c_void_p, c_void_p]),
    "gmr_regularizers_scratch_size": (c_int32, [c_int64, c_int64, ctypes.POINTER(c_size_t)]),
    "gmr_regularizers": (c_int32, [c_void_p, c_int64, c_void_p, c_int64, c_void_p, c_void_p, c_float, c_float,
                                   c_float, c_void_p, c_size_t, c_void_p, c_void_p, c_void_p]),
    "gmr_vector_adam_step": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_int64, c_float, c_float, c_float,
                                       c_float, c_void_p, c_void_p]),
    "gmr_autotune": (c_int32, [c_void_p, ctypes.POINTER(gmr_batch), ctypes.POINTER(gmr_options), c_void_p, c_void_p,
                               c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_int32, ctypes.POINTER(gmr_options),
                               ctypes.POINTER(c_float), c_void_p]),
}

EXPORTED = tuple(_SIGS)
_lib = None


class GMRError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn} failed with status {status}: {msg}")
        self.status = status


def load() -> ctypes.CDLL:
    """Load the in-tree libgmr.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libgmr.so is not built ({LIB_PATH}); run __graft_entry__.build() or "
                               "python paper_2602_14493_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(fn: str, status: int) -> None:
    if status != GMR_OK:
        msg = load().gmr_last_error().decode(errors="replace")
        raise GMRError(fn, status, msg)


def call(fn: str, *args) -> None:
    check(fn, getattr(load(), fn)(*args))
