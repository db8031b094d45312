"""Shared helpers of the GPU tests: run the HIP path through the C ABI, pull the tile lists out of
a workspace, and compare against the FP64 oracle with the stated tolerances."""
from __future__ import annotations

import ctypes

import numpy as np

IMG_ATOL = 1e-5          # images: absolute, on pixels the oracle does not flag near a threshold
MASK_FRAC_MAX = 1e-3     # at most this fraction of pixels may be flagged
GRAD_REL = 1e-3          # gradients: ||d||/||g|| and per element 1e-3 |g| + 1e-5 max|g|


def to_np(t):
    return t.detach().float().cpu().numpy() if hasattr(t, "detach") else np.asarray(t)


def gpu_setup(wl, **opt_kw):
    import torch
    import paper_2602_14493_amd as gmr
    batch = gmr.Batch.from_workload(wl)
    opts = gmr.default_options(**opt_kw)
    r = gmr.Renderer(batch, wl.faces, opts)
    verts = torch.from_numpy(np.ascontiguousarray(wl.verts)).cuda()
    colors = torch.from_numpy(np.ascontiguousarray(wl.colors)).cuda()
    return r, verts, colors


def compare_images(rgb_gpu, alpha_gpu, rgb_orc, tf_orc, mask, tol=IMG_ATOL, label=""):
    rgb_gpu = to_np(rgb_gpu).reshape(-1, 3)
    alpha_gpu = to_np(alpha_gpu).reshape(-1)
    frac = float(mask.mean())
    assert frac <= MASK_FRAC_MAX, f"{label}: {frac:.2e} of pixels near a threshold"
    ok = ~mask.reshape(-1)
    e_rgb = np.abs(rgb_gpu.astype(np.float64) - rgb_orc.reshape(-1, 3))[ok].max(initial=0.0)
    e_a = np.abs(alpha_gpu.astype(np.float64) - (1.0 - tf_orc.reshape(-1)))[ok].max(initial=0.0)
    print(f"{label}: max|drgb|={e_rgb:.3e} max|dalpha|={e_a:.3e} masked={int(mask.sum())}/{mask.size}", flush=True)
    assert e_rgb <= tol, f"{label}: image error {e_rgb:.3e} > {tol}"
    assert e_a <= tol, f"{label}: alpha error {e_a:.3e} > {tol}"
    return e_rgb, e_a


def flagged_pixels_agree(rgb_gpu, alpha_gpu, rgb_orc, tf_orc, mask, tol=IMG_ATOL):
    """Whether the GPU image equals the oracle's within the image tolerance on the pixels the oracle
    flags as near a decision threshold: then both sides took the same decisions there, and a
    gradient fed from those pixels can be compared with the oracle's adjoint."""
    m = np.asarray(mask).reshape(-1)
    if not m.any():
        return True
    d_rgb = np.abs(to_np(rgb_gpu).reshape(-1, 3).astype(np.float64) - rgb_orc.reshape(-1, 3))[m].max()
    d_a = np.abs(to_np(alpha_gpu).reshape(-1).astype(np.float64) - (1.0 - tf_orc.reshape(-1)))[m].max()
    print(f"{int(m.sum())} flagged pixels: max|drgb|={d_rgb:.3e} max|dalpha|={d_a:.3e}", flush=True)
    return d_rgb <= tol and d_a <= tol


def compare_grads(g_gpu, g_ref, label="", rel=GRAD_REL):
    g = to_np(g_gpu).astype(np.float64).reshape(-1)
    r = np.asarray(g_ref, np.float64).reshape(-1)
    d = g - r
    nr = np.linalg.norm(r)
    relerr = np.linalg.norm(d) / max(nr, 1e-300)
    bound = rel * np.abs(r) + 1e-5 * np.abs(r).max()
    worst = float((np.abs(d) / np.maximum(bound, 1e-300)).max())
    print(f"{label}: ||d||/||g||={relerr:.3e} worst elem/bound={worst:.3f} ||g||={nr:.3e}", flush=True)
    assert nr > 0
    assert relerr <= rel, f"{label}: relative gradient error {relerr:.3e}"
    assert worst <= 1.0, f"{label}: an element exceeds its bound ({worst:.2f}x)"
    return relerr


def workspace_lists(r, ws):
    """Per global tile, the sorted face-view indices the forward left in workspace ws."""
    import paper_2602_14493_amd as gmr
    ro, vo, rc, bo = (ctypes.c_size_t() for _ in range(4))
    gmr._lib.call("gmr_workspace_view", ctypes.byref(r.batch.c), ctypes.byref(r.opts), ctypes.byref(ro),
                  ctypes.byref(vo), ctypes.byref(rc), ctypes.byref(bo))
    w = ws.cpu().numpy()
    ntiles = table_tiles(r)
    ranges = w[ro.value:ro.value + 8 * ntiles].view(np.uint32).reshape(-1, 2)
    cap = int(r.opts.instance_capacity)
    vals = w[vo.value:vo.value + 4 * cap].view(np.uint32)
    return ranges, vals


def blk_words(r):
    """Words per raster item of the saved composited lists: the count, then up to composited_lists
    16-bit positions, two to a word (0: none recorded)."""
    c = int(r.opts.composited_lists)
    return 1 + (c + 1) // 2 if c > 0 else 0


def blk_lists(r, saved):
    """(counts, positions, kept) of the saved composited lists: counts [items] int64 (unsigned),
    positions [items, composited_lists] int64, kept = position index < min(count, cap)."""
    import torch
    P, nw, cap = r.batch.num_pixels, blk_words(r), int(r.opts.composited_lists)
    t = saved[8 * P:].view(torch.int32).view(-1, nw)
    cnt = t[:, 0].to(torch.int64) & 0xFFFFFFFF
    pos = t[:, 1:].contiguous().view(torch.int16)[:, :cap].to(torch.int64) & 0xFFFF
    kept = torch.arange(cap, device=saved.device)[None, :] < cnt.clamp(max=cap)[:, None]
    return cnt, pos, kept


def saved_equal(r, a, b):
    """Saved states equal where they are defined: T_final and list positions per pixel, and per
    raster item the composited-list count and its first min(count, composited_lists) positions (the
    rest of an item's words is left as it was)."""
    import torch
    P = r.batch.num_pixels
    if a.numel() != b.numel() or not torch.equal(a[:8 * P], b[:8 * P]):
        return False
    if blk_words(r) == 0:
        return True
    na, pa, keep = blk_lists(r, a)
    nb, pb, _ = blk_lists(r, b)
    if not torch.equal(na, nb):
        return False
    return torch.equal(pa[keep], pb[keep])


def table_tiles(r):
    tw, th = r.opts.tile_w, r.opts.tile_h
    return int(sum(((w + tw - 1) // tw) * ((h + th - 1) // th) for w, h in r.batch.sizes))


def fv_to_face(wl):
    """Map face-view index -> (view, global face id) for a workload's view-major numbering."""
    fo = wl.face_offsets
    starts, views, face0 = [0], [], []
    for v in range(wl.num_views):
        m = int(wl.view_mesh[v])
        n = int(fo[m + 1] - fo[m])
        starts.append(starts[-1] + n)
        face0.append(int(fo[m]))
    starts = np.asarray(starts)

    def f(fv):
        fv = np.asarray(fv, np.int64)
        v = np.searchsorted(starts, fv, side="right") - 1
        return v, fv - starts[v] + np.asarray(face0)[v]
    return f
