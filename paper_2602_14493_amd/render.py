"""Thin Python layer over libgmr: batch description, workspace / capacity management, the
torch.autograd.Function, and the hipGraph-captured Adam optimisation step.

Every stage of the forward and backward pass runs in libgmr's HIP kernels; this module only
allocates device memory through torch, hands pointers and the current stream to the C ABI, and
reads the device counters when asked.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import call, gmr_batch, gmr_camera, gmr_counters, gmr_options

_DEFAULT_HEADROOM = 1.25


def _ptr(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def default_options(**kw) -> gmr_options:
    """gmr_default_options() with fields overridden by keyword (bg takes a 3-sequence)."""
    o = _lib.load().gmr_default_options()
    for k, v in kw.items():
        if k == "bg":
            for i in range(3):
                o.bg[i] = float(v[i])
        else:
            setattr(o, k, v)
    return o


def options_dict(o: gmr_options) -> dict:
    d = {k: getattr(o, k) for k, _ in gmr_options._fields_ if k != "bg"}
    d["bg"] = tuple(o.bg)
    return d


def copy_options(o: gmr_options, **kw) -> gmr_options:
    n = gmr_options()
    ctypes.memmove(ctypes.addressof(n), ctypes.addressof(o), ctypes.sizeof(gmr_options))
    for k, v in kw.items():
        if k == "bg":
            for i in range(3):
                n.bg[i] = float(v[i])
        else:
            setattr(n, k, v)
    return n


class Handle:
    """gmr_create / gmr_destroy for one device."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        call("gmr_create", ctypes.byref(h), int(device))
        self.ptr = h
        self.device = device

    def __del__(self):
        try:
            if getattr(self, "ptr", None):
                _lib.load().gmr_destroy(self.ptr)
        except Exception:
            pass


class Batch:
    """Host description of a batch of meshes and views (see gmr_batch).  cams: array [NV, 20]
    laid out as R(9) t(3) fx fy cx cy W H near far."""

    def __init__(self, vert_offsets, face_offsets, view_mesh, cams):
        self.vert_offsets = np.ascontiguousarray(vert_offsets, dtype=np.int64)
        self.face_offsets = np.ascontiguousarray(face_offsets, dtype=np.int64)
        self.view_mesh = np.ascontiguousarray(view_mesh, dtype=np.int32)
        cams = np.asarray(cams, dtype=np.float64).reshape(-1, 20)
        self.cams = (gmr_camera * len(cams))()
        for i, c in enumerate(cams):
            cc = self.cams[i]
            for k in range(9):
                cc.R[k] = float(c[k])
            for k in range(3):
                cc.t[k] = float(c[9 + k])
            cc.fx, cc.fy, cc.cx, cc.cy = (float(x) for x in c[12:16])
            cc.width, cc.height = int(c[16]), int(c[17])
            cc.near_plane, cc.far_plane = float(c[18]), float(c[19])
        self.sizes = [(int(c[16]), int(c[17])) for c in cams]
        self.c = gmr_batch(len(self.vert_offsets) - 1, len(cams), self.vert_offsets.ctypes.data,
                           self.face_offsets.ctypes.data, self.view_mesh.ctypes.data,
                           ctypes.cast(self.cams, ctypes.c_void_p))
        self.num_pixels = int(sum(w * h for w, h in self.sizes))
        self.num_verts = int(self.vert_offsets[-1])
        self.num_faces = int(self.face_offsets[-1])

    @classmethod
    def from_workload(cls, wl) -> "Batch":
        return cls(wl.vert_offsets, wl.face_offsets, wl.view_mesh, wl.cam_array())

    def view(self, v: int) -> "Batch":
        """The single-view batch of view v (its mesh only), for per-view launches."""
        m = int(self.view_mesh[v])
        v0, v1 = int(self.vert_offsets[m]), int(self.vert_offsets[m + 1])
        f0, f1 = int(self.face_offsets[m]), int(self.face_offsets[m + 1])
        cam = np.zeros(20)
        c = self.cams[v]
        cam[:9] = list(c.R)
        cam[9:12] = list(c.t)
        cam[12:20] = [c.fx, c.fy, c.cx, c.cy, c.width, c.height, c.near_plane, c.far_plane]
        b = Batch([0, v1 - v0], [0, f1 - f0], [0], cam[None])
        b.mesh_range = (v0, v1, f0, f1)
        return b


@dataclass
class Counters:
    instances: int
    capacity: int
    overflow: bool
    pairs_fwd: int = 0
    pairs_bwd: int = 0
    loss: float = 0.0
    loss_sil: float = 0.0
    peak_instances: int = 0      # largest count of any list build since the previous read
    overflow_any: bool = False   # any of those builds overflowed


class Renderer:
    """One batch + options bound to device buffers: the view table, the vertex adjacency, and a
    workspace sized by the instance capacity (grown on overflow).

    faces: int32 [F,3] global vertex indices (host numpy or torch)."""

    def __init__(self, batch: Batch, faces, options: gmr_options | None = None, device: int = 0,
                 handle: Handle | None = None, headroom: float = _DEFAULT_HEADROOM):
        self.batch = batch
        self.device = torch.device("cuda", device)
        self.handle = handle or Handle(device)
        self.opts = copy_options(options if options is not None else default_options())
        self.headroom = headroom
        faces_np = faces.detach().cpu().numpy() if torch.is_tensor(faces) else np.asarray(faces)
        faces_np = np.ascontiguousarray(faces_np, dtype=np.int32)
        if faces_np.shape != (batch.num_faces, 3):
            raise ValueError(f"faces must be [{batch.num_faces}, 3], got {faces_np.shape}")
        self.faces = torch.from_numpy(faces_np).to(self.device)
        off = np.zeros(batch.num_verts + 1, np.int32)
        ent = np.zeros(3 * batch.num_faces, np.int32)
        call("gmr_build_adjacency", faces_np.ctypes.data, batch.num_faces, batch.num_verts, off.ctypes.data,
             ent.ctypes.data)
        self.adj_off = torch.from_numpy(off).to(self.device)
        self.adj_ent = torch.from_numpy(ent).to(self.device)
        self._set_table()
        if self.opts.instance_capacity <= 0:
            # a small first guess keeps small batches on the one-launch list build (the first
            # forward measures the count and grows the capacity if it was too small)
            self.opts.instance_capacity = max(1 << 12, 4 * batch.num_faces * max(1, batch.c.num_views))
            self.opts.instance_capacity = min(self.opts.instance_capacity, 1 << 26)
        self.capacity_checked = False
        self.ws = None

    # -- plumbing --------------------------------------------------------------------------------
    def _set_table(self):
        n = ctypes.c_size_t()
        call("gmr_view_table_size", ctypes.byref(self.batch.c), ctypes.byref(self.opts), ctypes.byref(n))
        host = np.zeros(n.value, np.uint8)
        call("gmr_view_table_fill", ctypes.byref(self.batch.c), ctypes.byref(self.opts), host.ctypes.data, n.value)
        self.table = torch.from_numpy(host).to(self.device)

    def set_options(self, options: gmr_options):
        cap = self.opts.instance_capacity
        self.opts = copy_options(options)
        if self.opts.instance_capacity <= 0:
            self.opts.instance_capacity = cap
        self._set_table()
        self.ws = None
        self.capacity_checked = False

    def sizes(self):
        ws = ctypes.c_size_t()
        saved = ctypes.c_size_t()
        call("gmr_workspace_size", ctypes.byref(self.batch.c), ctypes.byref(self.opts), ctypes.byref(ws),
             ctypes.byref(saved))
        return ws.value, saved.value

    def new_workspace(self) -> torch.Tensor:
        ws, _ = self.sizes()
        w = torch.empty(ws, dtype=torch.uint8, device=self.device)
        w[:256].zero_()   # arms the peak instance counter (the rest needs no initialisation)
        return w

    def new_saved(self) -> torch.Tensor:
        _, saved = self.sizes()
        return torch.empty(saved, dtype=torch.uint8, device=self.device)

    def counters(self, ws: torch.Tensor) -> Counters:
        c = gmr_counters()
        call("gmr_read_counters", _ptr(ws), ws.numel(), ctypes.byref(c), _stream(self.device))
        return Counters(int(c.instances), int(c.capacity), bool(c.overflow), int(c.pairs_fwd), int(c.pairs_bwd),
                        float(c.loss), float(c.loss_sil), int(c.peak_instances), bool(c.overflow_any))

    def check_colors(self, colors, verts=None):
        """Colours hold (sh_degree + 1)^2 x 3 floats per vertex ([V,3] at degree 0); vertices [V,3];
        both float32 on this renderer's device (the kernels index them by the batch's sizes)."""
        k = (int(self.opts.sh_degree) + 1) ** 2
        if colors.numel() != self.batch.num_verts * 3 * k or colors.dtype != torch.float32:
            raise ValueError(f"colors must be float32 with {k} x 3 values per vertex (sh_degree "
                             f"{self.opts.sh_degree}), got {tuple(colors.shape)} {colors.dtype}")
        if verts is not None and (verts.numel() != self.batch.num_verts * 3 or verts.dtype != torch.float32):
            raise ValueError(f"verts must be float32 [{self.batch.num_verts}, 3], got {tuple(verts.shape)} "
                             f"{verts.dtype}")
        for t in (colors, verts):
            if t is not None and t.device != self.device:
                raise ValueError(f"inputs must be on {self.device}, got {t.device}")

    # -- raw calls (no capacity management) --------------------------------------------------------
    def fwd_raw(self, verts, colors, rgb, alpha, saved, ws):
        call("gmr_render_fwd", self.handle.ptr, ctypes.byref(self.batch.c), ctypes.byref(self.opts), _ptr(self.table),
             _ptr(verts), _ptr(self.faces), _ptr(colors), _ptr(rgb), _ptr(alpha), _ptr(saved), _ptr(ws), ws.numel(),
             _stream(self.device))

    def step_l2_raw(self, verts, colors, target, loss_weight, rgb, alpha, saved, ws, d_verts, d_colors, loss=None):
        """gmr_render_step_l2: forward + fused L2 backward from one list build (see the header)."""
        call("gmr_render_step_l2", self.handle.ptr, ctypes.byref(self.batch.c), ctypes.byref(self.opts),
             _ptr(self.table), _ptr(verts), _ptr(self.faces), _ptr(colors), _ptr(target), float(loss_weight),
             _ptr(rgb), _ptr(alpha), _ptr(saved), _ptr(self.adj_off), _ptr(self.adj_ent), _ptr(d_verts),
             _ptr(d_colors), _ptr(loss), _ptr(ws), ws.numel(), _stream(self.device))

    def step_recon_raw(self, verts, colors, target, color_weight, mask, sil_weight, rgb, alpha, saved, ws, d_verts,
                       d_colors, losses=None):
        """gmr_render_step_recon: forward + colour and silhouette backward from one list build."""
        call("gmr_render_step_recon", self.handle.ptr, ctypes.byref(self.batch.c), ctypes.byref(self.opts),
             _ptr(self.table), _ptr(verts), _ptr(self.faces), _ptr(colors), _ptr(target), float(color_weight),
             _ptr(mask), float(sil_weight), _ptr(rgb), _ptr(alpha), _ptr(saved), _ptr(self.adj_off),
             _ptr(self.adj_ent), _ptr(d_verts), _ptr(d_colors), _ptr(losses), _ptr(ws), ws.numel(),
             _stream(self.device))

    def bwd_raw(self, verts, colors, d_rgb, d_alpha, saved, ws, recompute, d_verts, d_colors):
        call("gmr_render_bwd", self.handle.ptr, ctypes.byref(self.batch.c), ctypes.byref(self.opts), _ptr(self.table),
             _ptr(verts), _ptr(self.faces), _ptr(colors), _ptr(d_rgb), _ptr(d_alpha), _ptr(saved), _ptr(self.adj_off),
             _ptr(self.adj_ent), int(recompute), _ptr(d_verts), _ptr(d_colors), _ptr(ws), ws.numel(),
             _stream(self.device))

    def bwd_l2_raw(self, verts, colors, rgb, target, loss_weight, saved, ws, recompute, d_verts, d_colors, loss=None):
        call("gmr_render_bwd_l2", self.handle.ptr, ctypes.byref(self.batch.c), ctypes.byref(self.opts),
             _ptr(self.table), _ptr(verts), _ptr(self.faces), _ptr(colors), _ptr(rgb), _ptr(target),
             float(loss_weight), _ptr(saved), _ptr(self.adj_off), _ptr(self.adj_ent), int(recompute), _ptr(d_verts),
             _ptr(d_colors), _ptr(loss), _ptr(ws), ws.numel(), _stream(self.device))

    def bwd_recon_raw(self, verts, colors, rgb, target, color_weight, mask, sil_weight, saved, ws, recompute,
                      d_verts, d_colors, losses=None):
        call("gmr_render_bwd_recon", self.handle.ptr, ctypes.byref(self.batch.c), ctypes.byref(self.opts),
             _ptr(self.table), _ptr(verts), _ptr(self.faces), _ptr(colors), _ptr(rgb), _ptr(target),
             float(color_weight), _ptr(mask), float(sil_weight), _ptr(saved), _ptr(self.adj_off), _ptr(self.adj_ent),
             int(recompute), _ptr(d_verts), _ptr(d_colors), _ptr(losses), _ptr(ws), ws.numel(), _stream(self.device))

    # -- managed calls -------------------------------------------------------------------------------
    def _alloc_outputs(self):
        P = self.batch.num_pixels
        rgb = torch.empty((P, 3), dtype=torch.float32, device=self.device)
        alpha = torch.empty((P,), dtype=torch.float32, device=self.device)
        return rgb, alpha, self.new_saved()

    def forward(self, verts: torch.Tensor, colors: torch.Tensor, ws: torch.Tensor | None = None, check: bool | None = None):
        """Render every view.  Returns (rgb [P,3], alpha [P], saved, ws).  The instance count is
        read back (one synchronisation) on the first call and whenever check=True; on overflow the
        capacity grows and the pass is redone."""
        verts = verts.contiguous()
        colors = colors.contiguous()
        self.check_colors(colors, verts)
        rgb, alpha, saved = self._alloc_outputs()
        if check is None:
            check = not self.capacity_checked
        if ws is None or ws.numel() < self.sizes()[0]:
            ws = self.new_workspace()
        for _ in range(4):
            self.fwd_raw(verts, colors, rgb, alpha, saved, ws)
            if not check:
                break
            c = self.counters(ws)
            need = min((1 << 30) - 1, int(c.instances * self.headroom) + 1024)
            if not c.overflow and c.instances * self.headroom <= self.opts.instance_capacity:
                self.capacity_checked = True
                break
            # overflowed, or fits with too little headroom for the next calls: grow the capacity and
            # redo the pass in a workspace of the new layout (the returned one must match self.opts)
            self.opts.instance_capacity = max(need, int(self.opts.instance_capacity))
            ws = self.new_workspace()
        else:
            raise RuntimeError("instance capacity did not converge")
        return rgb, alpha, saved, ws

    def backward(self, verts, colors, d_rgb, d_alpha, saved, ws=None, recompute: bool = False):
        """dL/dverts, dL/dcolors from dL/drgb [P,3] (and dL/dalpha [P] or None).  With
        recompute=True (or no workspace) the sorted lists are rebuilt in a fresh workspace."""
        self.check_colors(colors, verts)
        if ws is None:
            ws = self.new_workspace()
            recompute = True
        dV = torch.empty_like(verts)
        dC = torch.empty_like(colors)
        self.bwd_raw(verts.contiguous(), colors.contiguous(), d_rgb.contiguous(),
                     None if d_alpha is None else d_alpha.contiguous(), saved, ws, recompute, dV, dC)
        return dV, dC

    def backward_l2(self, verts, colors, rgb, target, saved, ws=None, recompute=False, loss_weight=1.0,
                    want_loss=False):
        self.check_colors(colors, verts)
        if ws is None:
            ws = self.new_workspace()
            recompute = True
        dV = torch.empty_like(verts)
        dC = torch.empty_like(colors)
        loss = torch.empty((1,), dtype=torch.float32, device=self.device) if want_loss else None
        self.bwd_l2_raw(verts.contiguous(), colors.contiguous(), rgb, target.contiguous(), loss_weight, saved, ws,
                        recompute, dV, dC, loss)
        return (dV, dC, loss) if want_loss else (dV, dC)

    def backward_recon(self, verts, colors, rgb, target, mask, saved, ws=None, recompute=False, color_weight=1.0,
                       sil_weight=1.0):
        """Gradients of color_weight * MSE(rgb, target) + sil_weight * BCE(alpha, mask) (Sec. 3.1).
        Returns (dV, dC, losses [2] = colour, silhouette)."""
        self.check_colors(colors, verts)
        if ws is None:
            ws = self.new_workspace()
            recompute = True
        dV = torch.empty_like(verts)
        dC = torch.empty_like(colors)
        losses = torch.empty((2,), dtype=torch.float32, device=self.device)
        self.bwd_recon_raw(verts.contiguous(), colors.contiguous(), rgb, target.contiguous(), color_weight,
                           mask.contiguous(), sil_weight, saved, ws, recompute, dV, dC, losses)
        return dV, dC, losses

    def autotune(self, verts, colors, target, iters: int = 3, recompute: bool = False):
        """gmr_autotune over tile shapes and raster modes; adopts and returns the best options.
        recompute=True times the backward with the lists rebuilt (the form GraphAdamLoop and
        render(save_lists=False) run)."""
        best = gmr_options()
        ms = ctypes.c_float()
        call("gmr_autotune", self.handle.ptr, ctypes.byref(self.batch.c), ctypes.byref(self.opts), _ptr(verts),
             _ptr(self.faces), _ptr(colors), _ptr(target), _ptr(self.adj_off), _ptr(self.adj_ent), int(iters),
             int(bool(recompute)), ctypes.byref(best), ctypes.byref(ms), _stream(self.device))
        self.set_options(best)
        return best, float(ms.value)


# ------------------------------------------------------------------------------------------------
# autograd
# ------------------------------------------------------------------------------------------------

class _RenderFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, verts, colors, renderer: Renderer, save_lists: bool):
        rgb, alpha, saved, ws = renderer.forward(verts, colors)
        ctx.renderer = renderer
        ctx.ws = ws if save_lists else None
        ctx.save_for_backward(verts, colors, saved)
        ctx.mark_non_differentiable(saved)
        return rgb, alpha

    @staticmethod
    def backward(ctx, d_rgb, d_alpha):
        verts, colors, saved = ctx.saved_tensors
        r: Renderer = ctx.renderer
        if d_rgb is None:
            d_rgb = torch.zeros((r.batch.num_pixels, 3), dtype=torch.float32, device=verts.device)
        dV, dC = r.backward(verts, colors, d_rgb, d_alpha, saved, ws=ctx.ws, recompute=ctx.ws is None)
        ctx.ws = None
        return dV, dC, None, None


def render(verts: torch.Tensor, colors: torch.Tensor, renderer: Renderer, save_lists="auto"):
    """Differentiable render of every view: returns (rgb [P,3], alpha [P]).

    save_lists: True keeps the forward's sorted lists for the backward; False frees them and the
    backward rebuilds them bit-identically (the memory-light path); "auto" keeps them when the
    workspace is under a quarter of the device's free memory."""
    if save_lists == "auto":
        free, _ = torch.cuda.mem_get_info(renderer.device)
        save_lists = renderer.sizes()[0] < free // 4
    return _RenderFn.apply(verts, colors, renderer, bool(save_lists))


# ------------------------------------------------------------------------------------------------
# Adam (device step counter) and the captured optimisation step
# ------------------------------------------------------------------------------------------------

def adam_step(param, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    call("gmr_adam_step", _ptr(param), _ptr(grad), _ptr(m), _ptr(v), param.numel(), float(lr), float(beta1),
         float(beta2), float(eps), _ptr(step), _stream(param.device))


def vector_adam_step(param, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """VectorAdam on [V,3] parameters: v [V] holds one second moment per vertex."""
    if param.dim() != 2 or param.shape[1] != 3 or v.numel() != param.shape[0]:
        raise ValueError("vector_adam_step expects param/grad/m [V,3] and v [V]")
    call("gmr_vector_adam_step", _ptr(param), _ptr(grad), _ptr(m), _ptr(v), param.shape[0], float(lr), float(beta1),
         float(beta2), float(eps), _ptr(step), _stream(param.device))


class MeshGraph:
    """Unique edges and the vertex -> incident-edge CSR of a triangle mesh (built on the host once
    per topology), and the edge-length + Laplacian regularisers on it."""

    def __init__(self, faces, num_verts: int, device: int | torch.device = 0):
        f = faces.detach().cpu().numpy() if torch.is_tensor(faces) else np.asarray(faces)
        f = np.ascontiguousarray(f, dtype=np.int32)
        self.num_verts = int(num_verts)
        ne = ctypes.c_int64()
        call("gmr_mesh_graph_size", f.ctypes.data, len(f), self.num_verts, ctypes.byref(ne))
        self.num_edges = int(ne.value)
        edges = np.zeros((self.num_edges, 2), np.int32)
        off = np.zeros(self.num_verts + 1, np.int32)
        ent = np.zeros(2 * self.num_edges, np.int32)
        call("gmr_build_mesh_graph", f.ctypes.data, len(f), self.num_verts, self.num_edges, edges.ctypes.data,
             off.ctypes.data, ent.ctypes.data)
        dev = device if isinstance(device, torch.device) else torch.device("cuda", device)
        self.device = dev
        self.edges_host, self.off_host, self.ent_host = edges, off, ent
        self.edges = torch.from_numpy(edges).to(dev)
        self.off = torch.from_numpy(off).to(dev)
        self.ent = torch.from_numpy(ent).to(dev)
        nb = ctypes.c_size_t()
        call("gmr_regularizers_scratch_size", self.num_verts, self.num_edges, ctypes.byref(nb))
        self.scratch = torch.empty(max(16, nb.value), dtype=torch.uint8, device=dev)

    def regularizers_raw(self, verts, d_verts, losses, target_length=0.0, edge_weight=1.0, lap_weight=1.0):
        call("gmr_regularizers", _ptr(verts), self.num_verts, _ptr(self.edges), self.num_edges, _ptr(self.off),
             _ptr(self.ent), float(target_length), float(edge_weight), float(lap_weight), _ptr(self.scratch),
             self.scratch.numel(), _ptr(losses), _ptr(d_verts), _stream(self.device))

    def regularizers(self, verts, d_verts=None, target_length=0.0, edge_weight=1.0, lap_weight=1.0):
        """Adds the regulariser gradients to d_verts (zeros if None) and returns (d_verts, losses
        [2] = edge, Laplacian)."""
        verts = verts.contiguous()
        if d_verts is None:
            d_verts = torch.zeros_like(verts)
        losses = torch.empty((2,), dtype=torch.float32, device=self.device)
        self.regularizers_raw(verts, d_verts, losses, target_length, edge_weight, lap_weight)
        return d_verts, losses


@dataclass
class ReconWeights:
    """Weights of the reconstruction objective (Sec. 3.1, Loss Functions); the paper does not give
    its values, so every term defaults to 1 and the edge target length to 0."""
    color: float = 1.0
    silhouette: float = 1.0
    edge: float = 1.0
    laplacian: float = 1.0
    edge_length: float = 0.0


class ReconLoop:
    """The full reconstruction step of Sec. 3.1 -- forward, colour + silhouette backward (lists
    rebuilt), edge-length and Laplacian regularisers, VectorAdam on the vertices -- captured once as
    a HIP graph and replayed.  losses [4] after a step: colour, silhouette, edge, Laplacian, each
    weighted, evaluated at the vertices before that step's update."""

    def __init__(self, renderer: Renderer, verts: torch.Tensor, colors: torch.Tensor, target: torch.Tensor,
                 mask: torch.Tensor, weights: ReconWeights | None = None, lr=1e-3, betas=(0.9, 0.999), eps=1e-8,
                 recompute=True, fused=False):
        self.r = renderer
        self.fused = fused  # render the step with gmr_render_step_recon (one list build)
        dev = renderer.device
        self.w = weights or ReconWeights()
        self.verts = verts.detach().clone().contiguous()
        self.colors = colors.detach().contiguous()
        self.target = target.detach().contiguous()
        self.mask = mask.detach().to(torch.float32).contiguous()
        if self.mask.numel() != renderer.batch.num_pixels:
            raise ValueError("mask must hold one value per pixel of every view")
        self.graph_mesh = MeshGraph(renderer.faces, renderer.batch.num_verts, dev)
        self.m = torch.zeros_like(self.verts)
        self.v = torch.zeros((self.verts.shape[0],), dtype=torch.float32, device=dev)
        self.step_count = torch.zeros((1,), dtype=torch.int32, device=dev)
        self.lr, self.betas, self.eps, self.recompute = lr, betas, eps, recompute
        # eager warm-up sizes the instance capacity (with headroom) before capture; with
        # recompute the backward rebuilds the lists into the same workspace (one list buffer)
        rgb, alpha, saved, ws = renderer.forward(self.verts, self.colors, check=True)
        self.ws = ws
        self.rgb, self.alpha, self.saved = rgb, alpha, saved
        self.dV = torch.empty_like(self.verts)
        self.dC = torch.empty_like(self.colors)
        self.losses = torch.zeros((4,), dtype=torch.float32, device=dev)
        self.graph = None

    def _state(self):
        return (self.verts, self.m, self.v, self.step_count)

    def _step_body(self):
        r, w = self.r, self.w
        if self.fused:
            r.step_recon_raw(self.verts, self.colors, self.target, w.color, self.mask, w.silhouette, self.rgb,
                             self.alpha, self.saved, self.ws, self.dV, self.dC, self.losses[0:2])
        else:
            r.fwd_raw(self.verts, self.colors, self.rgb, self.alpha, self.saved, self.ws)
            r.bwd_recon_raw(self.verts, self.colors, self.rgb, self.target, w.color, self.mask, w.silhouette,
                            self.saved, self.ws, 1 if self.recompute else 0, self.dV, self.dC, self.losses[0:2])
        self.graph_mesh.regularizers_raw(self.verts, self.dV, self.losses[2:4], w.edge_length, w.edge, w.laplacian)
        vector_adam_step(self.verts, self.dV, self.m, self.v, self.step_count, self.lr, self.betas[0],
                         self.betas[1], self.eps)

    def capture(self):
        """Captures one step as a HIP graph.  An eager step runs first (on a side stream, as graph
        capture requires); the optimiser state it advanced is restored afterwards, so the first
        replay is the first step."""
        state = [t.clone() for t in self._state()]
        s = torch.cuda.Stream(self.r.device)
        s.wait_stream(torch.cuda.current_stream(self.r.device))
        with torch.cuda.stream(s):
            self._step_body()
        torch.cuda.current_stream(self.r.device).wait_stream(s)
        torch.cuda.synchronize(self.r.device)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._step_body()
        for t, saved in zip(self._state(), state):
            t.copy_(saved)
        torch.cuda.synchronize(self.r.device)
        return self

    def run(self, steps: int):
        if self.graph is None:
            self.capture()
        for _ in range(steps):
            self.graph.replay()

    def run_eager(self, steps: int):
        for _ in range(steps):
            self._step_body()

    def overflow(self) -> bool:
        """True if any list build since the previous check overflowed the instance capacity
        (synchronises; reading restarts the peak counter)."""
        c = self.r.counters(self.ws)
        return c.overflow or c.overflow_any


class GraphStep:
    """One forward + fused L2 backward (the lists reused, or rebuilt with recompute=True) captured
    once as a HIP graph and replayed: every launch of the step goes to the GPU in one submission,
    which on small batches removes the host's per-launch cost.  Outputs (rgb, alpha, dV, dC, loss)
    are this object's buffers, overwritten by each replay."""

    def __init__(self, renderer: Renderer, verts: torch.Tensor, colors: torch.Tensor, target: torch.Tensor,
                 recompute: bool = False):
        self.r = renderer
        self.verts = verts.detach().contiguous()
        self.colors = colors.detach().contiguous()
        self.target = target.detach().contiguous()
        self.recompute = bool(recompute)
        # eager warm-up sizes the instance capacity (with headroom) before capture
        self.rgb, self.alpha, self.saved, self.ws = renderer.forward(self.verts, self.colors, check=True)
        self.dV = torch.empty_like(self.verts)
        self.dC = torch.empty_like(self.colors)
        self.loss = torch.zeros((1,), dtype=torch.float32, device=renderer.device)
        self.graph = None

    def _step_body(self):
        r = self.r
        r.fwd_raw(self.verts, self.colors, self.rgb, self.alpha, self.saved, self.ws)
        r.bwd_l2_raw(self.verts, self.colors, self.rgb, self.target, 1.0, self.saved, self.ws,
                     1 if self.recompute else 0, self.dV, self.dC, self.loss)

    def capture(self):
        s = torch.cuda.Stream(self.r.device)
        s.wait_stream(torch.cuda.current_stream(self.r.device))
        with torch.cuda.stream(s):
            self._step_body()  # one eager step on a side stream before capture
        torch.cuda.current_stream(self.r.device).wait_stream(s)
        torch.cuda.synchronize(self.r.device)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._step_body()
        return self

    def replay(self):
        if self.graph is None:
            self.capture()
        self.graph.replay()

    def overflow(self) -> bool:
        """True if any list build since the previous check overflowed (synchronises)."""
        c = self.r.counters(self.ws)
        return c.overflow or c.overflow_any


class GraphAdamLoop:
    """One optimisation step -- forward, fused L2 backward with the sorted lists rebuilt, Adam on
    the vertices -- captured once as a HIP graph and replayed.  fused=True renders the step with
    gmr_render_step_l2 (one list build, compositing and adjoint in one launch)."""

    def __init__(self, renderer: Renderer, verts: torch.Tensor, colors: torch.Tensor, target: torch.Tensor,
                 lr=1e-3, betas=(0.9, 0.999), eps=1e-8, recompute=True, fused=False):
        self.fused = fused
        self.r = renderer
        dev = renderer.device
        self.verts = verts.detach().clone().contiguous()
        self.colors = colors.detach().contiguous()
        self.target = target.detach().contiguous()
        self.m = torch.zeros_like(self.verts)
        self.v = torch.zeros_like(self.verts)
        self.step_count = torch.zeros((1,), dtype=torch.int32, device=dev)
        self.lr, self.betas, self.eps, self.recompute = lr, betas, eps, recompute
        # eager warm-up sizes the instance capacity (with headroom) before capture; with
        # recompute the backward rebuilds the lists into the same workspace (one list buffer)
        rgb, alpha, saved, ws = renderer.forward(self.verts, self.colors, check=True)
        self.ws = ws
        self.rgb, self.alpha, self.saved = rgb, alpha, saved
        self.dV = torch.empty_like(self.verts)
        self.dC = torch.empty_like(self.colors)
        self.loss = torch.zeros((1,), dtype=torch.float32, device=dev)
        self.graph = None

    def _state(self):
        return (self.verts, self.m, self.v, self.step_count)

    def _step_body(self):
        r = self.r
        if self.fused:
            r.step_l2_raw(self.verts, self.colors, self.target, 1.0, self.rgb, self.alpha, self.saved, self.ws,
                          self.dV, self.dC, self.loss)
        else:
            r.fwd_raw(self.verts, self.colors, self.rgb, self.alpha, self.saved, self.ws)
            r.bwd_l2_raw(self.verts, self.colors, self.rgb, self.target, 1.0, self.saved, self.ws,
                         1 if self.recompute else 0, self.dV, self.dC, self.loss)
        adam_step(self.verts, self.dV, self.m, self.v, self.step_count, self.lr, self.betas[0], self.betas[1],
                  self.eps)

    def capture(self):
        """Captures one step as a HIP graph.  An eager step runs first (on a side stream, as graph
        capture requires); the optimiser state it advanced is restored afterwards, so the first
        replay is the first step."""
        state = [t.clone() for t in self._state()]
        s = torch.cuda.Stream(self.r.device)
        s.wait_stream(torch.cuda.current_stream(self.r.device))
        with torch.cuda.stream(s):
            self._step_body()
        torch.cuda.current_stream(self.r.device).wait_stream(s)
        torch.cuda.synchronize(self.r.device)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._step_body()
        for t, saved in zip(self._state(), state):
            t.copy_(saved)
        torch.cuda.synchronize(self.r.device)
        return self

    def run(self, steps: int):
        if self.graph is None:
            self.capture()
        for _ in range(steps):
            self.graph.replay()

    def run_eager(self, steps: int):
        for _ in range(steps):
            self._step_body()

    def overflow(self) -> bool:
        """True if any list build since the previous check overflowed the instance capacity
        (synchronises; reading restarts the peak counter)."""
        c = self.r.counters(self.ws)
        return c.overflow or c.overflow_any
