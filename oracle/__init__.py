"""FP64 CPU oracle of the Gaussian Mesh Renderer hot path (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the bench's CPU-baseline
leg may use this package; the product path (``paper_2602_14493_amd``) never imports it, and the
two share no code.  The arithmetic lives in ``gmr_oracle.cpp`` (see its header for what each
function follows in the paper); this module only marshals arrays, builds the library with g++,
and adds the plain L2 loss (Sec. 3.1, colour loss = mean squared error) and an FP64
central-difference harness.  ``oracle.recon`` holds the reconstruction step around the renderer
(silhouette BCE, edge-length and Laplacian regularisers, VectorAdam), in NumPy float64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gmr_oracle.cpp")
_LIB_PATH = os.path.join(_HERE, "libgmr_oracle.so")
_lib = None
_lock = threading.Lock()

f32 = np.float32


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (never hipcc)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = ctypes.CDLL(_LIB_PATH)
            P = ctypes.c_void_p
            i64, i32 = ctypes.c_long, ctypes.c_int
            L.gmro_convert.argtypes = [i64, P, i64, P, P, i32, P, P, P, P]
            L.gmro_convert.restype = i64
            L.gmro_convert_closed.argtypes = [i64, P, i64, P, i32, P, P, P]
            L.gmro_convert_closed.restype = i64
            L.gmro_face_steps.argtypes = [P, P, P, i32, P]
            L.gmro_face_steps.restype = i32
            L.gmro_project_one.argtypes = [P, P, P, ctypes.c_double, ctypes.c_double, P]
            L.gmro_project_one.restype = i32
            L.gmro_gaussians.argtypes = [i64, P, i64, P, P, P, P, P]
            L.gmro_gaussians.restype = i64
            L.gmro_render.argtypes = [i64, P, i64, P, P, i64, P, P, P, P, P, P, P, P]
            L.gmro_render.restype = i64
            L.gmro_render_adjoint.argtypes = [i64, P, i64, P, P, i64, P, P, P, P, P, P, P, P]
            L.gmro_render_adjoint.restype = i64
            L.gmro_tile_lists.argtypes = [i64, P, i64, P, P, i64, P, P, i32, i32, P, P, P, i64]
            L.gmro_tile_lists.restype = i64
            L.gmro_sh_basis.argtypes = [i32, i64, P, P]
            L.gmro_sh_basis.restype = i64
            L.gmro_num_threads.restype = i32
            _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _colours(colors, nv: int, params: "Params") -> np.ndarray:
    """Colour input as float32, checked against the colour model: [V,3] at degree 0, else
    [V, (degree + 1)^2, 3] coefficients (coefficient 0 is the colour itself)."""
    C = _c(colors, f32)
    k = (params.sh_degree + 1) ** 2
    if C.size != nv * 3 * k:
        raise ValueError(f"colours must hold {k} x 3 values per vertex for sh_degree {params.sh_degree}")
    return C


@dataclass
class Params:
    """Renderer constants.  Thresholds are the float32-rounded values (a pixel where two clamped
    Gaussians overlap has T(1-a) = (1 - a_max)^2, right at the stop threshold; rounding both sides'
    constants identically keeps that decision the same)."""
    cov_mode: int = 0                    # 0: Eq. 13 (area matched), 1: Eq. 15 (embedded Sigma2D),
    #                                      2: the "3DGS-based" edge-frame baseline (Sec. 3.1, Baselines)
    dilation: float = float(f32(0.3))    # screen-space low-pass, px^2
    alpha_min: float = float(f32(1.0 / 255.0))
    alpha_max: float = float(f32(0.99))
    t_eps: float = float(f32(1e-4))
    bg: tuple = (0.0, 0.0, 0.0)
    d_ext: float = 1e-6                  # px
    d_alpha: float = 1e-5                # relative
    alpha_err: float = 2e-6              # relative error bound of a float32 alpha
    nsig: float = 3.0
    sh_degree: int = 0                   # 0: Eq. 16 colours [V,3]; 1-3: coefficients [V,(d+1)^2,3]

    def array(self) -> np.ndarray:
        return np.array([self.cov_mode, self.dilation, self.alpha_min, self.alpha_max, self.t_eps,
                         *self.bg, self.d_ext, self.d_alpha, self.alpha_err, self.nsig, self.sh_degree],
                        dtype=np.float64)


def sh_basis(degree: int, dirs) -> np.ndarray:
    """The view-dependent colour basis (Y[0] = 1, then real harmonics of degree 1..degree) on unit
    directions [n,3]; returns [n, (degree + 1)^2]."""
    d = _c(np.asarray(dirs).reshape(-1, 3), np.float64)
    out = np.zeros((len(d), 16))
    lib().gmro_sh_basis(int(degree), len(d), _p(d), _p(out))
    return out[:, :(degree + 1) ** 2]


def num_threads() -> int:
    return int(lib().gmro_num_threads())


# ------------------------------------------------------------------------------------------------
# conversion (Sec. 2.2)
# ------------------------------------------------------------------------------------------------

def convert(verts, faces, colors, cov_mode: int = 0):
    """Literal conversion of every face.  Returns mu [F,3], Sigma [F,3,3], colour [F,3], valid [F]."""
    V, Fc = _c(verts, f32), _c(faces, np.int32)
    C = _c(colors, f32)
    nf = len(Fc)
    mu = np.zeros((nf, 3)); S = np.zeros((nf, 9)); col = np.zeros((nf, 3)); valid = np.zeros(nf, np.uint8)
    lib().gmro_convert(len(V), _p(V), nf, _p(Fc), _p(C), cov_mode, _p(mu), _p(S), _p(col), _p(valid))
    return mu, S.reshape(nf, 3, 3), col, valid.astype(bool)


def convert_closed(verts, faces, cov_mode: int = 0):
    V, Fc = _c(verts, f32), _c(faces, np.int32)
    nf = len(Fc)
    mu = np.zeros((nf, 3)); S = np.zeros((nf, 9)); valid = np.zeros(nf, np.uint8)
    lib().gmro_convert_closed(len(V), _p(V), nf, _p(Fc), cov_mode, _p(mu), _p(S), _p(valid))
    return mu, S.reshape(nf, 3, 3), valid.astype(bool)


_STEP_FIELDS = [("x_axis", 3), ("y_axis", 3), ("n_f", 3), ("xj", 1), ("xk", 1), ("yk", 1), ("mux", 1),
                ("muy", 1), ("Exx", 1), ("Exy", 1), ("Eyy", 1), ("S2", 3), ("l1", 1), ("l2", 1), ("u1", 2),
                ("u2", 2), ("xp", 3), ("yp", 3), ("area", 1), ("kappa", 1), ("mu", 3), ("S", 9)]


def face_steps(vi, vj, vk, cov_mode: int = 0):
    """Every intermediate of the literal route for one triangle (double inputs), or None."""
    a, b, c = (_c(x, np.float64) for x in (vi, vj, vk))
    out = np.zeros(64)
    if not lib().gmro_face_steps(_p(a), _p(b), _p(c), cov_mode, _p(out)):
        return None
    d, k = {}, 0
    for name, n in _STEP_FIELDS:
        d[name] = out[k] if n == 1 else out[k:k + n].copy()
        k += n
    d["S"] = d["S"].reshape(3, 3)
    return d


def project_one(mu, S, cam_arr, dilation=Params.dilation, nsig=3.0):
    """EWA projection of one Gaussian; returns dict(u, v, conic, rx, ry, depth) or None."""
    out = np.zeros(8)
    m, s, c = _c(mu, np.float64), _c(np.asarray(S).reshape(9), np.float64), _c(cam_arr, np.float64)
    if not lib().gmro_project_one(_p(m), _p(s), _p(c), dilation, nsig, _p(out)):
        return None
    return dict(u=out[0], v=out[1], conic=out[2:5].copy(), rx=out[5], ry=out[6], depth=out[7])


def gaussians(verts, faces, colors, cam_arr, params: Params | None = None):
    """Per-face screen-space Gaussians for one view: array [F,12] = ok u v a b c rx ry depth r g b."""
    params = params or Params()
    V, Fc = _c(verts, f32), _c(faces, np.int32)
    C = _colours(colors, len(V), params)
    out = np.zeros((len(Fc), 12))
    lib().gmro_gaussians(len(V), _p(V), len(Fc), _p(Fc), _p(C), _p(_c(cam_arr, np.float64)),
                         _p(params.array()), _p(out))
    return out


# ------------------------------------------------------------------------------------------------
# rendering (per view, no tiles) and its adjoint
# ------------------------------------------------------------------------------------------------

def render_view(verts, faces, colors, cam_arr, params: Params | None = None, gid_base: int = 0,
                window=None, want_hash=False):
    """Render one view of one mesh.  Returns (rgb [h,w,3], Tf [h,w], ncomp [h,w], mask [h,w])
    over window = (x0, y0, x1, y1) (default: the whole image); with want_hash also a per-pixel
    hash [h,w] of the composited face sequence."""
    params = params or Params()
    cam_arr = _c(cam_arr, np.float64)
    W, H = int(cam_arr[16]), int(cam_arr[17])
    win = np.array(window if window is not None else (0, 0, W, H), dtype=np.int32)
    win = np.array([max(0, win[0]), max(0, win[1]), min(W, win[2]), min(H, win[3])], dtype=np.int32)
    w, h = max(0, int(win[2] - win[0])), max(0, int(win[3] - win[1]))
    V, Fc = _c(verts, f32), _c(faces, np.int32)
    C = _colours(colors, len(V), params)
    rgb = np.zeros((h, w, 3)); Tf = np.zeros((h, w)); nc = np.zeros((h, w), np.int32)
    mask = np.zeros((h, w), np.uint8)
    lh = np.zeros((h, w), np.uint64) if want_hash else None
    lib().gmro_render(len(V), _p(V), len(Fc), _p(Fc), _p(C), gid_base, _p(cam_arr), _p(params.array()),
                      _p(win), _p(rgb), _p(Tf), _p(nc), _p(mask), _p(lh))
    if want_hash:
        return rgb, Tf, nc, mask.astype(bool), lh
    return rgb, Tf, nc, mask.astype(bool)


def adjoint_view(verts, faces, colors, cam_arr, g_rgb, g_alpha=None, params: Params | None = None,
                 gid_base: int = 0, window=None, want_screen_grads=False):
    """Exact adjoint of render_view: returns (dV [V,3], dC shaped like colors) (and the per-face
    screen-space gradients [F,8] when want_screen_grads)."""
    params = params or Params()
    cam_arr = _c(cam_arr, np.float64)
    W, H = int(cam_arr[16]), int(cam_arr[17])
    win = np.array(window if window is not None else (0, 0, W, H), dtype=np.int32)
    win = np.array([max(0, win[0]), max(0, win[1]), min(W, win[2]), min(H, win[3])], dtype=np.int32)
    V, Fc = _c(verts, f32), _c(faces, np.int32)
    C = _colours(colors, len(V), params)
    g_rgb = _c(g_rgb, np.float64)
    g_alpha = None if g_alpha is None else _c(g_alpha, np.float64)
    dV = np.zeros((len(V), 3)); dC = np.zeros(C.shape)
    gG = np.zeros((len(Fc), 8)) if want_screen_grads else None
    lib().gmro_render_adjoint(len(V), _p(V), len(Fc), _p(Fc), _p(C), gid_base, _p(cam_arr),
                              _p(params.array()), _p(win), _p(g_rgb), _p(g_alpha), _p(dV), _p(dC), _p(gG))
    if want_screen_grads:
        return dV, dC, gG
    return dV, dC


def tile_lists_view(verts, faces, colors, cam_arr, tile_w, tile_h, params: Params | None = None,
                    gid_base: int = 0):
    """Per-tile lists of global ids ordered by (float32 depth, id), plus per-entry ambiguity codes
    (0 certain, 1 member but near the extent margin, 2 non-member near the margin)."""
    params = params or Params()
    cam_arr = _c(cam_arr, np.float64)
    W, H = int(cam_arr[16]), int(cam_arr[17])
    nt = ((W + tile_w - 1) // tile_w) * ((H + tile_h - 1) // tile_h)
    V, Fc = _c(verts, f32), _c(faces, np.int32)
    C = _colours(colors, len(V), params)
    off = np.zeros(nt + 1, np.int64)
    cap = 1 << 16
    while True:
        ids = np.zeros(cap, np.int32); amb = np.zeros(cap, np.uint8)
        n = lib().gmro_tile_lists(len(V), _p(V), len(Fc), _p(Fc), _p(C), gid_base, _p(cam_arr),
                                  _p(params.array()), tile_w, tile_h, _p(off), _p(ids), _p(amb), cap)
        if n <= cap:
            return off, ids[:n], amb[:n]
        cap = int(n)


# ------------------------------------------------------------------------------------------------
# whole workloads (views laid out back to back, row-major, like the GPU output)
# ------------------------------------------------------------------------------------------------

def render_workload(wl, params: Params | None = None, verts=None, views=None, colors=None):
    """Render every view of a workloads.Workload.  Returns flat (rgb [P,3], Tf [P], ncomp [P],
    mask [P]) with the views back to back."""
    params = params or Params()
    verts = wl.verts if verts is None else verts
    colors = wl.colors if colors is None else colors
    views = range(wl.num_views) if views is None else views
    rgbs, tfs, ncs, masks = [], [], [], []
    cams = wl.cam_array()
    for v in views:
        m = int(wl.view_mesh[v])
        v0, v1 = int(wl.vert_offsets[m]), int(wl.vert_offsets[m + 1])
        f0, f1 = int(wl.face_offsets[m]), int(wl.face_offsets[m + 1])
        rgb, tf, nc, mk = render_view(verts[v0:v1], wl.faces[f0:f1] - v0, colors[v0:v1], cams[v],
                                      params, gid_base=f0)
        rgbs.append(rgb.reshape(-1, 3)); tfs.append(tf.reshape(-1)); ncs.append(nc.reshape(-1))
        masks.append(mk.reshape(-1))
    return np.concatenate(rgbs), np.concatenate(tfs), np.concatenate(ncs), np.concatenate(masks)


def adjoint_workload(wl, g_rgb, g_alpha=None, params: Params | None = None, verts=None, colors=None):
    """Adjoint over every view of a workload; g_rgb [P,3] and g_alpha [P] in the flat layout."""
    params = params or Params()
    verts = wl.verts if verts is None else verts
    colors = wl.colors if colors is None else colors
    dV = np.zeros((len(verts), 3)); dC = np.zeros(np.shape(colors), np.float64)
    cams = wl.cam_array()
    po = wl.pixel_offsets()
    for v in range(wl.num_views):
        m = int(wl.view_mesh[v])
        v0, v1 = int(wl.vert_offsets[m]), int(wl.vert_offsets[m + 1])
        f0, f1 = int(wl.face_offsets[m]), int(wl.face_offsets[m + 1])
        W, H = wl.cams[v].width, wl.cams[v].height
        gr = g_rgb[po[v]:po[v + 1]].reshape(H, W, 3)
        ga = None if g_alpha is None else g_alpha[po[v]:po[v + 1]].reshape(H, W)
        dv, dc = adjoint_view(verts[v0:v1], wl.faces[f0:f1] - v0, colors[v0:v1], cams[v], gr, ga, params,
                              gid_base=f0)
        dV[v0:v1] += dv
        dC[v0:v1] += dc
    return dV, dC


def l2_loss(rgb, target, weight=None):
    """Colour loss of Sec. 3.1 (mean squared error over every channel of every pixel of every view),
    optionally with per-pixel weights; returns (loss, dL/drgb)."""
    rgb = np.asarray(rgb, np.float64)
    target = np.asarray(target, np.float64)
    n = rgb.size
    diff = rgb - target
    if weight is not None:
        w = np.asarray(weight, np.float64).reshape(-1, 1)
        return float((w * diff * diff).sum() / n), 2.0 * w * diff / n
    return float((diff * diff).sum() / n), 2.0 * diff / n


def fd_vertex_grad(loss_fn, verts, vid: int, h: float = 1e-6, decision_fn=None, max_halvings: int = 3):
    """FP64 central difference of loss_fn(verts) w.r.t. vertex vid's 3 coordinates.  The vertex is
    moved in float64 and handed over as float32, so h must be representable: the perturbed vertex
    is rounded to float32 and the actual step is used.  decision_fn(verts) returns a hashable
    summary of every discrete decision (composited lists); when the + and - evaluations disagree
    with the base, h is halved (up to max_halvings times), else the coordinate is reported as None."""
    base = np.asarray(verts, np.float64)
    dec0 = decision_fn(base.astype(f32)) if decision_fn else None
    g = []
    for k in range(3):
        hh = h
        for _ in range(max_halvings + 1):
            vp = base.copy(); vm = base.copy()
            vp[vid, k] = float(f32(base[vid, k] + hh))
            vm[vid, k] = float(f32(base[vid, k] - hh))
            step = vp[vid, k] - vm[vid, k]
            vpf, vmf = vp.astype(f32), vm.astype(f32)
            if decision_fn is None or (decision_fn(vpf) == dec0 and decision_fn(vmf) == dec0):
                g.append((loss_fn(vpf) - loss_fn(vmf)) / step)
                break
            hh /= 2.0
        else:
            g.append(None)
    return g
