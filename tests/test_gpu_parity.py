"""Parity of the HIP path (called through the C ABI) with the FP64 oracle, plus the GPU-side
invariants: bit-exact tile lists, determinism, recompute == saved lists, batched == per-view,
tile-shape / raster-mode independence, the capacity-overflow protocol and edge cases.

Tolerances (written here): images 1e-5 absolute on pixels the oracle does
not flag as near a decision threshold (flagged fraction <= 1e-3); gradients ||d||/||g|| <= 1e-3
and per element |d| <= 1e-3 |g| + 1e-5 max|g|; tile lists and their order bit-exact outside the
oracle's ambiguity set."""
import numpy as np
import pytest

import oracle
import workloads as wl
from gmr_testutil import (compare_grads, compare_images, fv_to_face, gpu_setup, saved_equal, to_np, workspace_lists)

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def oracle_params(**kw):
    return oracle.Params(**kw)


# ------------------------------------------------------------------------------------------------
# images and gradients vs the oracle
# ------------------------------------------------------------------------------------------------

@pytest.mark.parametrize("cov_mode", [0, 1, 2])
def test_cfg1_image_and_grads(gpu, cov_mode):
    say(f"cfg1 icosphere s2 128^2 cov_mode={cov_mode}")
    W = wl.make_workload(1)
    r, verts, colors = gpu_setup(W, cov_mode=cov_mode)
    rgb, alpha, saved, ws = r.forward(verts, colors)
    P = oracle_params(cov_mode=cov_mode)
    o_rgb, o_tf, o_nc, o_mask = oracle.render_workload(W, P)
    compare_images(rgb, alpha, o_rgb, o_tf, o_mask, label=f"cfg1 mode{cov_mode}")
    rng = np.random.default_rng(101)
    g_rgb = rng.normal(size=(W.num_pixels, 3)) * (~o_mask)[:, None]
    g_a = rng.normal(size=W.num_pixels) * (~o_mask)
    import torch
    dV, dC = r.backward(verts, colors, torch.from_numpy(g_rgb.astype(np.float32)).cuda(),
                        torch.from_numpy(g_a.astype(np.float32)).cuda(), saved, ws)
    oV, oC = oracle.adjoint_workload(W, g_rgb, g_a, P)
    compare_grads(dV, oV, f"cfg1 mode{cov_mode} dV")
    compare_grads(dC, oC, f"cfg1 mode{cov_mode} dC")


def test_cfg1_fused_l2_matches_explicit_upstream(gpu):
    """The fused L2 backward equals the explicit backward fed dL/drgb = 2 (rgb - t) / 3P; and
    with a target the oracle renders from the unjittered mesh it matches the oracle's adjoint."""
    import torch
    say("cfg1 fused L2")
    W = wl.make_workload(1)
    r, verts, colors = gpu_setup(W)
    tgt_rgb, _, _, _ = oracle.render_workload(W, verts=W.target_verts)
    target = torch.from_numpy(tgt_rgb.astype(np.float32)).cuda()
    rgb, alpha, saved, ws = r.forward(verts, colors)
    dV1, dC1, loss = r.backward_l2(verts, colors, rgb, target, saved, ws, want_loss=True)
    g = 2.0 * (rgb - target) / rgb.numel()
    dV2, dC2 = r.backward(verts, colors, g, None, saved, ws)
    compare_grads(dV1, to_np(dV2), "fused vs explicit dV", rel=1e-5)
    compare_grads(dC1, to_np(dC2), "fused vs explicit dC", rel=1e-5)
    o_rgb, o_tf, _, o_mask = oracle.render_workload(W)
    L, g_o = oracle.l2_loss(o_rgb, tgt_rgb)
    assert abs(float(loss.item()) - L) <= 1e-5 * L + 1e-9
    if not o_mask.any():
        oV, oC = oracle.adjoint_workload(W, g_o)
        compare_grads(dV1, oV, "cfg1 L2 dV vs oracle")
        compare_grads(dC1, oC, "cfg1 L2 dC vs oracle")
    else:
        g_o = g_o * (~o_mask)[:, None]
        dV3, dC3 = r.backward(verts, colors, torch.from_numpy(g_o.astype(np.float32)).cuda(), None, saved, ws)
        oV, oC = oracle.adjoint_workload(W, g_o)
        compare_grads(dV3, oV, "cfg1 L2 (masked) dV vs oracle")
        compare_grads(dC3, oC, "cfg1 L2 (masked) dC vs oracle")


def test_cfg2_images_and_crop_loss_grads(gpu):
    """Icosphere subdiv 5, 8 views 512^2: all images vs the oracle; vertex and colour gradients
    of the L2 loss restricted to the centre crop [224, 288)^2 of every view."""
    import torch
    say("cfg2 icosphere s5 8x512^2")
    W = wl.make_workload(2)
    r, verts, colors = gpu_setup(W)
    rgb, alpha, saved, ws = r.forward(verts, colors)
    o_rgb, o_tf, _, o_mask = oracle.render_workload(W)
    compare_images(rgb, alpha, o_rgb, o_tf, o_mask, label="cfg2")
    tgt, _, _, _ = oracle.render_workload(W, verts=W.target_verts)
    crop = np.zeros((W.num_views, 512, 512), bool)
    crop[:, 224:288, 224:288] = True
    crop = crop.reshape(-1) & ~o_mask
    n = 3 * int(crop.sum())
    g = np.where(crop[:, None], 2.0 * (o_rgb - tgt) / n, 0.0)
    dV, dC = r.backward(verts, colors, torch.from_numpy(g.astype(np.float32)).cuda(), None, saved, ws)
    oV, oC = oracle.adjoint_workload(W, g)
    compare_grads(dV, oV, "cfg2 crop dV")
    compare_grads(dC, oC, "cfg2 crop dC")


@pytest.mark.parametrize("cov_mode", [1, 2])
def test_other_conversions_multiview(gpu, cov_mode):
    """The literal Eq. 15 covariance (cov_mode 1, the form the paper's implementation uses) and the
    "3DGS-based" baseline conversion (cov_mode 2) through the whole path on the 8-view icosphere
    (128^2 views): images and the L2 gradients vs the oracle, and each differs from Eq. 13."""
    import torch
    say(f"cfg2 scale 0.25, cov_mode {cov_mode}")
    W = wl.make_workload(2, scale=0.25)
    r, verts, colors = gpu_setup(W, cov_mode=cov_mode)
    rgb, alpha, saved, ws = r.forward(verts, colors)
    P = oracle_params(cov_mode=cov_mode)
    o_rgb, o_tf, _, o_mask = oracle.render_workload(W, P)
    compare_images(rgb, alpha, o_rgb, o_tf, o_mask, label=f"cfg2/4 mode{cov_mode}")
    tgt, _, _, _ = oracle.render_workload(W, P, verts=W.target_verts)
    _, g = oracle.l2_loss(o_rgb, tgt)
    g = g * (~o_mask)[:, None]
    rng = np.random.default_rng(7 + cov_mode)
    g_a = rng.normal(size=W.num_pixels) * 1e-3 * (~o_mask)
    dV, dC = r.backward(verts, colors, torch.from_numpy(g.astype(np.float32)).cuda(),
                        torch.from_numpy(g_a.astype(np.float32)).cuda(), saved, ws)
    oV, oC = oracle.adjoint_workload(W, g, g_a, P)
    compare_grads(dV, oV, f"cfg2/4 mode{cov_mode} dV")
    compare_grads(dC, oC, f"cfg2/4 mode{cov_mode} dC")
    o0, _, _, _ = oracle.render_workload(W)
    assert np.abs(o0 - o_rgb).max() > 1e-2


def _sh_colours(W, deg, seed, hi=0.15):
    rng = np.random.default_rng(seed)
    K = (deg + 1) ** 2
    C = np.zeros((len(W.verts), K, 3), np.float32)
    C[:, 0] = W.colors
    C[:, 1:] = rng.normal(0, hi, size=(len(W.verts), K - 1, 3))
    return C


@pytest.mark.parametrize("deg", [1, 2, 3])
def test_view_dependent_colour_images_and_grads(gpu, deg):
    """View-dependent colour (sh_degree 1, 2 and 3) on the single view and on the 8-view icosphere
    (128^2): images, vertex gradients (through the viewing direction too) and coefficient
    gradients vs the oracle; some channels sit on the clamp at 0."""
    import torch
    for k, scale in ((1, 1.0), (2, 0.25)):
        say(f"cfg{k} scale {scale} sh_degree {deg}")
        W = wl.make_workload(k, scale=scale)
        r, verts, _ = gpu_setup(W, sh_degree=deg)
        C = _sh_colours(W, deg, 40 + deg)
        colors = torch.from_numpy(C).cuda()
        rgb, alpha, saved, ws = r.forward(verts, colors)
        P = oracle_params(sh_degree=deg)
        o_rgb, o_tf, _, o_mask = oracle.render_workload(W, P, colors=C)
        compare_images(rgb, alpha, o_rgb, o_tf, o_mask, label=f"cfg{k} sh{deg}")
        rng = np.random.default_rng(102)
        g_rgb = rng.normal(size=(W.num_pixels, 3)) * (~o_mask)[:, None]
        g_a = rng.normal(size=W.num_pixels) * (~o_mask)
        dV, dC = r.backward(verts, colors, torch.from_numpy(g_rgb.astype(np.float32)).cuda(),
                            torch.from_numpy(g_a.astype(np.float32)).cuda(), saved, ws)
        oV, oC = oracle.adjoint_workload(W, g_rgb, g_a, P, colors=C)
        assert dC.shape == colors.shape
        compare_grads(dV, oV, f"cfg{k} sh{deg} dV")
        compare_grads(dC, oC, f"cfg{k} sh{deg} dC")


def test_view_dependent_colour_reduces_to_eq16(gpu):
    """sh_degree 3 with zero higher coefficients renders the degree-0 image bit for bit, and its
    backward gives the same vertex gradients and the same coefficient-0 gradients (up to the
    order of the raster backward's float atomics)."""
    import torch
    W = wl.make_workload(2, scale=0.25)
    r0, verts, colors = gpu_setup(W)
    r3, _, _ = gpu_setup(W, sh_degree=3)
    C = np.zeros((len(W.verts), 16, 3), np.float32)
    C[:, 0] = W.colors
    c3 = torch.from_numpy(C).cuda()
    a = r0.forward(verts, colors)
    b = r3.forward(verts, c3)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    g = torch.randn_like(a[0])
    dV0, dC0 = r0.backward(verts, colors, g, None, a[2], a[3])
    dV3, dC3 = r3.backward(verts, c3, g, None, b[2], b[3])
    compare_grads(dV3, to_np(dV0), "sh3 with zero higher coefficients dV", rel=1e-5)
    compare_grads(dC3[:, 0], to_np(dC0), "sh3 with zero higher coefficients dC_0", rel=1e-5)
    assert float(dC3[:, 1:].abs().max()) > 0


def test_cfg5_view0_image_and_crop_grads_full_size(gpu):
    """2M-face torus, 32 views at 1920x1080, in the bench's launch configuration (32 x 16 tiles,
    lists rebuilt in the backward): the batched forward's first view vs the oracle, and the vertex
    and colour gradients of the L2 loss (against the noise-free torus) restricted to two 64 x 64
    crops of view 0 (a crop on the tube, one across its silhouette), vs the oracle's adjoint."""
    import torch
    say("cfg5 torus 2M, view 0 of 32 at 1920x1080, tile 32x16, recompute")
    W = wl.make_workload(5)
    r, verts, colors = gpu_setup(W, tile_w=32, tile_h=16)
    rgb, alpha, saved, ws = r.forward(verts, colors)
    Wd, Hd = 1920, 1080
    npx = Wd * Hd
    o_rgb, o_tf, _, o_mask = oracle.render_workload(W, views=[0])
    compare_images(to_np(rgb)[:npx], to_np(alpha)[:npx], o_rgb, o_tf, o_mask, label="cfg5 view0")
    # crops placed from the oracle's coverage of view 0: the 64 x 64 window (on a 32-px grid)
    # nearest the image centre that is fully covered, and one that is about half covered
    cov = (1.0 - o_tf).reshape(Hd, Wd) > 0.5
    cands = []
    for y in range(0, Hd - 64, 32):
        for x in range(0, Wd - 64, 32):
            f = cov[y:y + 64, x:x + 64].mean()
            cands.append((f, (y + 32 - Hd / 2) ** 2 + (x + 32 - Wd / 2) ** 2, y, x))
    full = min((c for c in cands if c[0] == 1.0), key=lambda c: c[1])
    half = min((c for c in cands if abs(c[2] - full[2]) >= 64 or abs(c[3] - full[3]) >= 64),
               key=lambda c: (abs(c[0] - 0.5), c[1]))
    crop = np.zeros((Hd, Wd), bool)
    for _, _, y, x in (full, half):
        crop[y:y + 64, x:x + 64] = True
    say(f"crops at {full[2:]} (covered {full[0]:.2f}) and {half[2:]} (covered {half[0]:.2f})")
    crop = crop.reshape(-1) & ~o_mask
    tgt, _, _, _ = oracle.render_workload(W, verts=W.target_verts, views=[0])
    n = 3 * int(crop.sum())
    g0 = np.where(crop[:, None], 2.0 * (o_rgb - tgt) / n, 0.0)
    g = np.zeros((W.num_pixels, 3), np.float32)
    g[:npx] = g0
    dV, dC = r.backward(verts, colors, torch.from_numpy(g).cuda(), None, saved, ws, recompute=True)
    assert not r.counters(ws).overflow
    # the oracle's adjoint of view 0 (the only view with a nonzero upstream gradient), one crop
    # window at a time (pixels are independent)
    oV, oC = np.zeros(W.verts.shape), np.zeros(W.colors.shape)
    g0 = g0.reshape(Hd, Wd, 3)
    for _, _, y, x in (full, half):
        dv, dc = oracle.adjoint_view(W.verts, W.faces, W.colors, W.cam_array()[0],
                                     np.ascontiguousarray(g0[y:y + 64, x:x + 64]), window=(x, y, x + 64, y + 64))
        oV += dv
        oC += dc
    compare_grads(dV, oV, "cfg5 view0 crops dV")
    compare_grads(dC, oC, "cfg5 view0 crops dC")


# ------------------------------------------------------------------------------------------------
# tile lists
# ------------------------------------------------------------------------------------------------

@pytest.mark.parametrize("tw,th,px", [(32, 16, 1), (16, 32, 2), (64, 64, 1)])
def test_instance_key_block_masks(gpu, tw, th, px):
    """Every sorted instance key holds its tile id in the low b = ceil(log2(tiles)) bits and, when
    the tile's raster blocks fit above them, the mask of the 8 x (8 px) blocks its record's pixel
    rectangle meets (the rasters read only the entries whose bit is set); 64 x 64 tiles (64 blocks)
    carry no mask.  The mask is recomputed here from the documented layout and the rectangles the
    projection wrote; both build paths are covered (the one-workgroup build by config 1)."""
    import ctypes
    import paper_2602_14493_amd as gmr
    for k in (2, 1):
        say(f"key block masks cfg{k} tile {tw}x{th} px {px}")
        W = wl.make_workload(k)
        r, verts, colors = gpu_setup(W, tile_w=tw, tile_h=th, px_per_lane=px)
        rgb, alpha, saved, ws = r.forward(verts, colors, check=True)
        ro, vo, rc, ko = (ctypes.c_size_t() for _ in range(4))
        gmr._lib.call("gmr_workspace_view", ctypes.byref(r.batch.c), ctypes.byref(r.opts), ctypes.byref(ro),
                      ctypes.byref(vo), ctypes.byref(rc), ctypes.byref(ko))
        w = ws.cpu().numpy()
        n = r.counters(ws).instances
        keys = w[ko.value:ko.value + 4 * n].view(np.uint32).astype(np.int64)
        vals = w[vo.value:vo.value + 4 * n].view(np.uint32).astype(np.int64)
        nfv = int(sum(W.face_offsets[int(W.view_mesh[v]) + 1] - W.face_offsets[int(W.view_mesh[v])]
                      for v in range(W.num_views)))
        rec = w[rc.value:rc.value + 48 * nfv].view(np.uint32).reshape(nfv, 12).astype(np.int64)
        # tile geometry: view-major, row-major tile numbering
        sizes = list(r.batch.sizes)
        tx_n = np.array([(a + tw - 1) // tw for a, _ in sizes])
        ty_n = np.array([(hh + th - 1) // th for _, hh in sizes])
        base = np.concatenate([[0], np.cumsum(tx_n * ty_n)])
        ntiles = int(base[-1])
        b = 0
        while (1 << b) < ntiles:
            b += 1
        sub_x, sub_y, bh = tw // 8, th // (8 * px), 8 * px
        masks_on = b <= 26 and sub_x * sub_y <= 32 - b
        tile = keys & ((1 << b) - 1)
        # the tile ids are the sorted order's: ascending, each inside the table
        assert (np.diff(tile) >= 0).all() and tile.max() < ntiles
        v = np.searchsorted(base, tile, side="right") - 1
        lt = tile - base[v]
        X0, Y0 = (lt % tx_n[v]) * tw, (lt // tx_n[v]) * th
        rx, ry = rec[vals, 7], rec[vals, 11]
        ix0, ix1, iy0, iy1 = rx & 0xffff, rx >> 16, ry & 0xffff, ry >> 16
        want = np.zeros(n, dtype=np.int64)
        for sy in range(sub_y):
            for sx in range(sub_x):
                bx0, by0 = X0 + 8 * sx, Y0 + bh * sy
                meet = (ix0 <= bx0 + 7) & (ix1 >= bx0) & (iy0 <= by0 + bh - 1) & (iy1 >= by0)
                want |= meet.astype(np.int64) << (sy * sub_x + sx)
        got = keys >> b
        say(f"  {n} instances, {ntiles} tiles, b = {b}, masks {'on' if masks_on else 'off'}")
        if masks_on:
            assert (want != 0).all(), "an instance whose rectangle meets none of its tile's blocks"
            assert np.array_equal(got, want)
        else:
            assert (got == 0).all()


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 16)])
def test_tile_lists_bit_exact(gpu, tile):
    """Every tile's list (membership and order) equals the oracle's tile list built from per-pixel
    extents and sorted by (float32 depth, id), except entries the oracle flags as ambiguous."""
    tw, th = tile
    say(f"tile lists cfg2 tile {tw}x{th}")
    W = wl.make_workload(2)
    r, verts, colors = gpu_setup(W, tile_w=tw, tile_h=th)
    rgb, alpha, saved, ws = r.forward(verts, colors)
    ranges, vals = workspace_lists(r, ws)
    conv = fv_to_face(W)
    cams = W.cam_array()
    tbase = 0
    checked = 0
    for v in range(W.num_views):
        off, ids, amb = oracle.tile_lists_view(W.verts, W.faces, W.colors, cams[v], tw, th)
        nt = len(off) - 1
        for t in range(nt):
            s, e = ranges[tbase + t]
            vv, gl = conv(vals[s:e])
            assert (vv == v).all()
            o_ids = ids[off[t]:off[t + 1]]
            o_amb = amb[off[t]:off[t + 1]]
            ambiguous = set(o_ids[o_amb != 0].tolist())
            want = [i for i, a in zip(o_ids.tolist(), o_amb.tolist()) if a == 0]
            got = [i for i in gl.tolist() if i not in ambiguous]
            assert got == want, f"view {v} tile {t}"
            assert set(gl.tolist()) <= set(o_ids.tolist())
            checked += len(want)
        tbase += nt
    say(f"checked {checked} list entries")
    assert checked > 100000


def _two_mesh_small():
    """Two small meshes, one with three views and one with a single view, interleaved in the view
    order (1,212 face-views)."""
    rng = np.random.default_rng(11)
    va, fa = wl.icosphere(2)
    vb, fb = wl.torus(14, 9, R=0.5, r=0.2)
    va = va * 0.8 + rng.normal(0, 0.01, size=va.shape)
    vb = vb + np.array([0.1, -0.05, 0.0]) + rng.normal(0, 0.01, size=vb.shape)
    verts = np.concatenate([va, vb]).astype(np.float32)
    faces = np.concatenate([fa, fb + len(va)]).astype(np.int32)
    colors = rng.uniform(size=verts.shape).astype(np.float32)
    cams = [wl.look_at_camera((0.0, 0.0, 3.0), width=96, height=80),
            wl.look_at_camera((1.5, 1.0, 1.2), width=72, height=72),
            wl.look_at_camera((-2.0, 0.5, 2.0), width=64, height=96),
            wl.look_at_camera((0.3, -2.5, 1.0), width=80, height=64)]
    return wl.Workload(name="two_mesh_small", verts=verts, faces=faces, colors=colors,
                       vert_offsets=np.array([0, len(va), len(verts)], dtype=np.int64),
                       face_offsets=np.array([0, len(fa), len(faces)], dtype=np.int64),
                       view_mesh=np.array([0, 1, 0, 0], dtype=np.int32), cams=cams)


@pytest.mark.parametrize("case", ["cfg1-8", "cfg1-16", "cfg1-32", "two-mesh"])
def test_small_build_matches_radix_build(gpu, case):
    """Small batches build their lists in one launch (an LDS bitonic sort of (tile | depth |
    face-view) keys); with a capacity above that path's limit the same batch takes the radix-sort
    path.  Both must give the same tile lists (bit for bit), the same images and saved state, and
    the same gradients (up to the order of the raster backward's float atomics); a capacity far
    too small overflows on the one-launch path and the protocol grows it."""
    import torch
    import paper_2602_14493_amd as gmr
    if case == "two-mesh":
        W, tw = _two_mesh_small(), 16
    else:
        W, tw = wl.make_workload(1), int(case.split("-")[1])
    say(f"one-launch vs radix list build: {case}")
    r_s, verts, colors = gpu_setup(W, tile_w=tw, tile_h=tw, instance_capacity=256)
    r_b, _, _ = gpu_setup(W, tile_w=tw, tile_h=tw, instance_capacity=1 << 16)
    a = r_s.forward(verts, colors, check=True)      # overflows at 256 and grows
    b = r_b.forward(verts, colors, check=True)
    cs, cb = r_s.counters(a[3]), r_b.counters(b[3])
    say(f"instances {cs.instances} (capacity {cs.capacity}) vs {cb.instances} (capacity {cb.capacity})")
    assert cs.capacity <= 8192 < cb.capacity and cs.instances == cb.instances and not cs.overflow
    ls, lb = workspace_lists(r_s, a[3]), workspace_lists(r_b, b[3])
    assert np.array_equal(ls[0], lb[0])
    n = cs.instances
    assert np.array_equal(ls[1][:n], lb[1][:n])
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and saved_equal(r_s, a[2], b[2])
    g = torch.randn_like(a[0])
    dV1, dC1 = r_s.backward(verts, colors, g, None, a[2], a[3], recompute=True)
    dV2, dC2 = r_b.backward(verts, colors, g, None, b[2], b[3], recompute=True)
    compare_grads(dV1, to_np(dV2), f"{case} dV", rel=1e-5)
    compare_grads(dC1, to_np(dC2), f"{case} dC", rel=1e-5)


def test_tile_lists_and_image_wide_depth_range(gpu):
    """A camera 0.3 units from the surface and one at radius 3: the visible depths span 0.3 .. 4,
    more than the 256 values of the high 16 key bits that let the depth sort take three passes, so
    this checks the four-pass path (lists bit-exact, image against the oracle); the narrow range of
    the other workloads checks the three-pass path."""
    W2 = wl.make_workload(2)
    cams = [wl.look_at_camera((0.0, 0.0, 1.3), width=256, height=256),
            wl.look_at_camera((1.2, 2.0, 2.0), width=256, height=256)]
    W = wl._single("icosphere_s5_near_far", W2.verts, W2.faces, W2.colors, cams)
    ca = W.cam_array()
    his = []
    for v in range(W.num_views):
        G = oracle.gaussians(W.verts, W.faces, W.colors, ca[v])
        depth = G[G[:, 0] > 0, 8].astype(np.float32)
        his.append(depth.view(np.uint32) >> 16)
    his = np.concatenate(his)
    assert int(his.max()) - int(his.min()) >= 256, "the scene must exercise the four-pass depth sort"
    say(f"wide depth range: high key bits span {int(his.max()) - int(his.min())}")
    r, verts, colors = gpu_setup(W, tile_w=16, tile_h=16)
    rgb, alpha, saved, ws = r.forward(verts, colors)
    o_rgb, o_tf, _, o_mask = oracle.render_workload(W)
    compare_images(rgb, alpha, o_rgb, o_tf, o_mask, label="wide depth")
    ranges, vals = workspace_lists(r, ws)
    conv = fv_to_face(W)
    tbase, checked = 0, 0
    for v in range(W.num_views):
        off, ids, amb = oracle.tile_lists_view(W.verts, W.faces, W.colors, ca[v], 16, 16)
        nt = len(off) - 1
        for t in range(nt):
            s, e = ranges[tbase + t]
            vv, gl = conv(vals[s:e])
            assert (vv == v).all()
            o_ids, o_amb = ids[off[t]:off[t + 1]], amb[off[t]:off[t + 1]]
            ambiguous = set(o_ids[o_amb != 0].tolist())
            want = [i for i, a in zip(o_ids.tolist(), o_amb.tolist()) if a == 0]
            assert [i for i in gl.tolist() if i not in ambiguous] == want, f"view {v} tile {t}"
            checked += len(want)
        tbase += nt
    say(f"checked {checked} list entries")
    assert checked > 10000


# ------------------------------------------------------------------------------------------------
# GPU invariants
# ------------------------------------------------------------------------------------------------

def test_determinism_and_recompute_lists(gpu):
    import torch
    say("determinism cfg2")
    W = wl.make_workload(2)
    r, verts, colors = gpu_setup(W)
    rgb1, a1, s1, ws1 = r.forward(verts, colors)
    rgb2, a2, s2, ws2 = r.forward(verts, colors)
    assert torch.equal(rgb1, rgb2) and torch.equal(a1, a2) and saved_equal(r, s1, s2)
    l1 = workspace_lists(r, ws1)
    l2 = workspace_lists(r, ws2)
    n = int(l1[0][:, 1].max())
    assert np.array_equal(l1[0], l2[0]) and np.array_equal(l1[1][:n], l2[1][:n])
    # backward with recompute rebuilds bit-identical lists in a fresh workspace
    ws3 = r.new_workspace()
    g = torch.randn_like(rgb1)
    dV3, dC3 = r.backward(verts, colors, g, None, s1, ws3, recompute=True)
    l3 = workspace_lists(r, ws3)
    assert np.array_equal(l1[0], l3[0]) and np.array_equal(l1[1][:n], l3[1][:n])
    dV1, dC1 = r.backward(verts, colors, g, None, s1, ws1, recompute=False)
    compare_grads(dV3, to_np(dV1), "recompute vs saved dV", rel=1e-5)
    compare_grads(dC3, to_np(dC1), "recompute vs saved dC", rel=1e-5)


def test_batched_equals_per_view(gpu):
    """The batched launch and one launch per view give bit-identical images; gradients agree."""
    import torch
    import paper_2602_14493_amd as gmr
    say("batched vs per-view cfg2")
    W = wl.make_workload(2)
    r, verts, colors = gpu_setup(W)
    rgb, alpha, saved, ws = r.forward(verts, colors)
    g = torch.randn_like(rgb)
    dV, dC = r.backward(verts, colors, g, None, saved, ws)
    npx = 512 * 512
    dVs = torch.zeros_like(dV)
    dCs = torch.zeros_like(dC)
    for v in range(W.num_views):
        bv = r.batch.view(v)
        rv = gmr.Renderer(bv, W.faces, gmr.copy_options(r.opts, instance_capacity=0), handle=r.handle)
        rgb_v, a_v, s_v, ws_v = rv.forward(verts, colors)
        assert torch.equal(rgb_v, rgb[v * npx:(v + 1) * npx]), v
        assert torch.equal(a_v, alpha[v * npx:(v + 1) * npx]), v
        dv, dc = rv.backward(verts, colors, g[v * npx:(v + 1) * npx], None, s_v, ws_v)
        dVs += dv
        dCs += dc
    compare_grads(dVs, to_np(dV), "per-view sum vs batched dV", rel=1e-5)
    compare_grads(dCs, to_np(dC), "per-view sum vs batched dC", rel=1e-5)


def test_tile_shape_and_raster_mode_invariance(gpu):
    import torch
    import paper_2602_14493_amd as gmr
    say("tile shape / persistent invariance cfg2")
    W = wl.make_workload(2)
    r, verts, colors = gpu_setup(W)
    base, base_a, _, _ = r.forward(verts, colors)
    for tw, th, mode in [(8, 8, 0), (32, 16, 0), (16, 16, 1), (64, 64, 1), (8, 24, 1)]:
        r2 = gmr.Renderer(r.batch, W.faces, gmr.default_options(tile_w=tw, tile_h=th, raster_mode=mode),
                          handle=r.handle)
        rgb, a, _, _ = r2.forward(verts, colors)
        assert torch.equal(rgb, base), (tw, th, mode)
        assert torch.equal(a, base_a), (tw, th, mode)


def test_overflow_protocol(gpu):
    """A workspace too small for the instances sets the overflow counter (writes are clamped);
    the managed forward then grows the capacity and reproduces the full-capacity image."""
    import torch
    import paper_2602_14493_amd as gmr
    say("overflow cfg1")
    W = wl.make_workload(1)
    r, verts, colors = gpu_setup(W, instance_capacity=64)
    rgb, alpha, saved = r._alloc_outputs()
    ws = r.new_workspace()
    r.fwd_raw(verts, colors, rgb, alpha, saved, ws)
    c = r.counters(ws)
    assert c.overflow and c.instances > 64 and c.capacity == 64
    r2, _, _ = gpu_setup(W, instance_capacity=1 << 20)
    ref, _, _, _ = r2.forward(verts, colors)
    out, _, _, ws_b = r.forward(verts, colors, check=True)
    assert not r.counters(ws_b).overflow and r.opts.instance_capacity > 64
    assert torch.equal(out, ref)


def test_overflow_radix_lists_are_valid(gpu):
    """Overflow on the radix path with two tile passes and a 512-bin first tile digit (8 views of
    1024 x 1024, 8 x 8 tiles: 17 tile bits): what the build writes within the capacity is a valid
    tile-sorted list of real instances with consistent ranges, i.e. the later passes sort exactly
    the instances the emission placed and nothing lands past the capacity."""
    import ctypes
    import paper_2602_14493_amd as gmr
    say("overflow on the radix path, cfg2 at 1024^2, 8x8 tiles")
    W = wl.make_workload(2, scale=2.0)
    r_full, verts, colors = gpu_setup(W, tile_w=8, tile_h=8)
    _, _, _, ws_full = r_full.forward(verts, colors, check=True)
    N = r_full.counters(ws_full).instances
    C = N // 3
    r, _, _ = gpu_setup(W, tile_w=8, tile_h=8, instance_capacity=C)
    rgb, alpha, saved = r._alloc_outputs()
    ws = r.new_workspace()
    r.fwd_raw(verts, colors, rgb, alpha, saved, ws)
    c = r.counters(ws)
    say(f"  {N} instances, capacity {C}")
    assert c.overflow and c.instances == N and c.capacity == C
    ranges, vals = workspace_lists(r, ws)
    nz = ranges[:, 1] > ranges[:, 0]
    tiles = np.nonzero(nz)[0]
    starts, ends = ranges[nz, 0].astype(np.int64), ranges[nz, 1].astype(np.int64)
    # the non-empty ranges tile [0, C) in tile order
    assert starts[0] == 0 and ends[-1] == C and np.array_equal(starts[1:], ends[:-1])
    # every (tile, face-view) pair is an instance: the face-view's pixel rectangle meets the tile,
    # in the tile's view; no pair twice
    key = np.repeat(tiles, ends - starts).astype(np.int64)
    fv = vals[:C].astype(np.int64)
    assert fv.max() < W.num_views * len(W.faces)
    ro, vo, rc, bo = (ctypes.c_size_t() for _ in range(4))
    gmr._lib.call("gmr_workspace_view", ctypes.byref(r.batch.c), ctypes.byref(r.opts), ctypes.byref(ro),
                  ctypes.byref(vo), ctypes.byref(rc), ctypes.byref(bo))
    w = ws.cpu().numpy()
    rec = w[rc.value:rc.value + 48 * W.num_views * len(W.faces)].view(np.uint32).reshape(-1, 12)
    xr, yr = rec[fv, 7].astype(np.int64), rec[fv, 11].astype(np.int64)
    per_view = 128 * 128
    view_of_tile, local = key // per_view, key % per_view
    ty, tx = local // 128, local % 128
    v_fv, _ = fv_to_face(W)(fv)
    assert np.array_equal(v_fv, view_of_tile)
    assert np.all((xr & 0xFFFF) <= 8 * tx + 7) and np.all((xr >> 16) >= 8 * tx)
    assert np.all((yr & 0xFFFF) <= 8 * ty + 7) and np.all((yr >> 16) >= 8 * ty)
    assert len(np.unique(key * (1 << 32) + fv)) == C


def test_edge_cases(gpu):
    """Camera looking away (no instances), odd image sizes, 1x1 image, a degenerate face (zero
    gradient), a mesh partly behind the camera."""
    import torch
    import paper_2602_14493_amd as gmr
    say("edge cases")
    rng = np.random.default_rng(7)
    V, F = wl.random_mesh(rng, 30, spread=0.4, size=0.12)
    V = V.astype(np.float32)
    V[3:6] = V[3]  # face 1 collapsed to a point: culled
    C = rng.uniform(size=V.shape).astype(np.float32)
    cams = [wl.look_at_camera((0.2, 0.1, 2.0), width=37, height=23),
            wl.look_at_camera((0.0, 0.0, 2.0), target=(0.0, 0.0, 5.0), width=16, height=16),  # looks away
            wl.look_at_camera((0.1, 0.0, 2.2), width=1, height=1),
            wl.look_at_camera((0.0, 0.0, 0.05), width=40, height=40)]  # inside the cloud
    for k, cam in enumerate(cams):
        say(f"edge view {k} {cam.width}x{cam.height}")
        Wk = wl._single("edge", V, F, C, [cam])
        r, verts, colors = gpu_setup(Wk)
        rgb, alpha, saved, ws = r.forward(verts, colors)
        o_rgb, o_tf, _, o_mask = oracle.render_workload(Wk)
        if o_mask.mean() <= 1e-3:
            compare_images(rgb, alpha, o_rgb, o_tf, o_mask, label=f"edge{k}")
        g = rng.normal(size=(Wk.num_pixels, 3)) * (~o_mask)[:, None]
        dV, dC = r.backward(verts, colors, torch.from_numpy(g.astype(np.float32)).cuda(), None, saved, ws)
        d = to_np(dV)
        assert np.isfinite(d).all()
        assert (d[3:6] == 0).all() or k == 1
        if k == 1:
            assert (to_np(rgb) == 0).all() and (d == 0).all()
        oV, oC = oracle.adjoint_workload(Wk, g)
        if np.abs(oV).max() > 0:
            compare_grads(dV, oV, f"edge{k} dV")
    # the four views in one batch: a face's views are then split over 8 lanes in the face backward
    # (a small batch with several views per mesh), the degenerate face included
    say("edge cases, all views in one batch")
    Wa = wl._single("edge_all", V, F, C, cams)
    r, verts, colors = gpu_setup(Wa)
    rgb, alpha, saved, ws = r.forward(verts, colors)
    o_rgb, o_tf, _, o_mask = oracle.render_workload(Wa)
    g = rng.normal(size=(Wa.num_pixels, 3)) * (~o_mask)[:, None]
    dV, dC = r.backward(verts, colors, torch.from_numpy(g.astype(np.float32)).cuda(), None, saved, ws)
    d = to_np(dV)
    assert np.isfinite(d).all() and (d[3:6] == 0).all()
    oV, oC = oracle.adjoint_workload(Wa, g)
    compare_grads(dV, oV, "edge all views dV")
    compare_grads(dC, oC, "edge all views dC")


def test_small_two_mesh_batch_images_and_grads(gpu):
    """Two small meshes, one with three views and one with a single view, interleaved in the view
    order: the face backward splits each face's views over 8 lanes (a mesh with fewer views leaves
    lanes idle); images and gradients against the oracle."""
    import torch
    say("small two-mesh batch")
    rng = np.random.default_rng(11)
    va, fa = wl.icosphere(2)
    vb, fb = wl.torus(14, 9, R=0.5, r=0.2)
    va = va * 0.8 + rng.normal(0, 0.01, size=va.shape)
    vb = vb + np.array([0.1, -0.05, 0.0]) + rng.normal(0, 0.01, size=vb.shape)
    verts = np.concatenate([va, vb]).astype(np.float32)
    faces = np.concatenate([fa, fb + len(va)]).astype(np.int32)
    colors = rng.uniform(size=verts.shape).astype(np.float32)
    cams = [wl.look_at_camera((0.0, 0.0, 3.0), width=96, height=80),
            wl.look_at_camera((1.5, 1.0, 1.2), width=72, height=72),
            wl.look_at_camera((-2.0, 0.5, 2.0), width=64, height=96),
            wl.look_at_camera((0.3, -2.5, 1.0), width=80, height=64)]
    W = wl.Workload(name="two_mesh_small", verts=verts, faces=faces, colors=colors,
                    vert_offsets=np.array([0, len(va), len(verts)], dtype=np.int64),
                    face_offsets=np.array([0, len(fa), len(faces)], dtype=np.int64),
                    view_mesh=np.array([0, 1, 0, 0], dtype=np.int32), cams=cams)
    r, v_d, c_d = gpu_setup(W)
    rgb, alpha, saved, ws = r.forward(v_d, c_d)
    o_rgb, o_tf, _, o_mask = oracle.render_workload(W)
    compare_images(rgb, alpha, o_rgb, o_tf, o_mask, label="two-mesh")
    g = rng.normal(size=(W.num_pixels, 3)) * (~o_mask)[:, None] / W.num_pixels
    dV, dC = r.backward(v_d, c_d, torch.from_numpy(g.astype(np.float32)).cuda(), None, saved, ws)
    oV, oC = oracle.adjoint_workload(W, g)
    compare_grads(dV, oV, "two-mesh dV")
    compare_grads(dC, oC, "two-mesh dC")


@pytest.mark.parametrize("cfg,kw", [(2, {}), (2, {"lane_lists": 0}), (2, {"px_per_lane": 2, "tile_w": 16, "tile_h": 16}),
                                    (2, {"px_per_lane": 4, "tile_w": 32, "tile_h": 32}), (2, {"raster_mode": 1}),
                                    (2, {"px_per_lane": 2, "tile_w": 16, "tile_h": 16, "lane_lists": 0}),
                                    (2, {"composited_lists": 7}), (3, {"tile_w": 32, "tile_h": 16})])
def test_backward_composited_lists_equal_full_walk(gpu, cfg, kw):
    """The backward walks, per 8 x 8 block, only the Gaussians the forward recorded as composited by
    one of its pixels (the saved buffer's per-item lists); with every list marked as not fitting it
    walks the tile's whole list instead.  Both give the same pair count and the same gradients (up to
    the order of the float atomics), lists saved or rebuilt; the lists hold ascending positions below
    each block's furthest stop, at most composited_lists of them."""
    import torch
    from gmr_testutil import blk_lists, blk_words
    say(f"composited lists vs full walk: cfg{cfg} {kw}")
    W = wl.make_workload(cfg, scale=0.25 if cfg == 3 else 1.0)
    r, verts, colors = gpu_setup(W, **kw)
    rgb, alpha, saved, ws = r.forward(verts, colors, check=True)
    P = W.num_pixels
    cap = int(r.opts.composited_lists)
    cnt, ent, keep = blk_lists(r, saved)
    say(f"  {cnt.shape[0]} items, counts mean {float(cnt.float().mean()):.1f} max {int(cnt.max())}, "
        f"{int((cnt > cap).sum())} over the capacity")
    fit = cnt <= cap
    asc = (ent[:, 1:] > ent[:, :-1]) | ~keep[:, 1:]
    assert bool(asc[fit].all()), "positions not ascending"
    g = torch.randn_like(rgb)
    for recompute in (False, True):
        dV, dC = r.backward(verts, colors, g, None, saved, ws, recompute=recompute)
        pairs = r.counters(ws).pairs_bwd
        s2 = saved.clone()
        b2 = s2[8 * P:].view(torch.int32).view(-1, blk_words(r))
        b2[:, 0] = -1  # 0xffffffff: no list
        dV2, dC2 = r.backward(verts, colors, g, None, s2, ws, recompute=recompute)
        assert r.counters(ws).pairs_bwd == pairs
        compare_grads(dV2, to_np(dV), f"cfg{cfg} lists vs full walk dV", rel=1e-5)
        compare_grads(dC2, to_np(dC), f"cfg{cfg} lists vs full walk dC", rel=1e-5)


def test_composited_lists_off_equals_default(gpu):
    """composited_lists = 0 records no lists (the saved state is the 8 bytes per pixel) and the
    backward walks every tile's whole list: images, per-pixel saved state, pair counts and
    gradients (up to atomic order) equal those of the default options."""
    import torch
    say("composited lists off vs default: cfg2")
    W = wl.make_workload(2)
    outs = []
    for kw in ({}, {"composited_lists": 0}):
        r, verts, colors = gpu_setup(W, **kw)
        rgb, alpha, saved, ws = r.forward(verts, colors, check=True)
        g = torch.randn(rgb.shape, device="cuda", generator=torch.Generator("cuda").manual_seed(5))
        dV, dC = r.backward(verts, colors, g, None, saved, ws)
        c = r.counters(ws)
        outs.append((rgb, alpha, saved, dV, dC, c.pairs_fwd, c.pairs_bwd))
    a, b = outs
    P = W.num_pixels
    assert b[2].numel() == 8 * P
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and torch.equal(a[2][:8 * P], b[2])
    assert a[5:] == b[5:]
    compare_grads(b[3], to_np(a[3]), "lists off dV", rel=1e-5)
    compare_grads(b[4], to_np(a[4]), "lists off dC", rel=1e-5)


def test_composited_lists_long_tile_lists(gpu):
    """A tile list longer than 16-bit positions reach records no composited list (count
    0xffffffff) and its blocks walk the whole list: the uv sphere's 400,000 faces in 64 x 64 views
    of one 64 x 64 tile each.  Images, per-pixel saved state, pair counts and gradients equal those
    with the lists off."""
    import torch
    from gmr_testutil import blk_lists
    say("composited lists, tile lists over 65536 entries: uvsphere 4 x 64^2, one tile per view")
    W = wl.make_workload(3, scale=1 / 16)
    outs = []
    for kw in ({}, {"composited_lists": 0}):
        r, verts, colors = gpu_setup(W, tile_w=64, tile_h=64, **kw)
        rgb, alpha, saved, ws = r.forward(verts, colors, check=True)
        if kw == {}:
            cnt, _, _ = blk_lists(r, saved)
            say(f"  {r.counters(ws).instances} instances over {W.num_views} tiles")
            assert r.counters(ws).instances > 65536 * W.num_views
            assert bool((cnt == 0xFFFFFFFF).all())
        g = torch.randn(rgb.shape, device="cuda", generator=torch.Generator("cuda").manual_seed(9))
        dV, dC = r.backward(verts, colors, g, None, saved, ws)
        c = r.counters(ws)
        outs.append((rgb, alpha, saved, dV, dC, c.pairs_fwd, c.pairs_bwd))
    a, b = outs
    P = W.num_pixels
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and torch.equal(a[2][:8 * P], b[2])
    assert a[5:] == b[5:]
    compare_grads(b[3], to_np(a[3]), "long lists dV", rel=1e-5)
    compare_grads(b[4], to_np(a[4]), "long lists dC", rel=1e-5)


def test_autograd_recompute_equals_saved(gpu):
    import torch
    import paper_2602_14493_amd as gmr
    say("autograd save vs recompute cfg2")
    W = wl.make_workload(2)
    r, verts, colors = gpu_setup(W)
    tgt = torch.rand((W.num_pixels, 3), device="cuda", generator=torch.Generator("cuda").manual_seed(3))
    grads = []
    for save in (True, False):
        v = verts.clone().requires_grad_(True)
        c = colors.clone().requires_grad_(True)
        rgb, alpha = gmr.render(v, c, r, save_lists=save)
        loss = ((rgb - tgt) ** 2).mean() + 0.1 * alpha.mean()
        loss.backward()
        grads.append((v.grad.clone(), c.grad.clone()))
    compare_grads(grads[1][0], to_np(grads[0][0]), "autograd recompute vs saved dV", rel=1e-5)
    compare_grads(grads[1][1], to_np(grads[0][1]), "autograd recompute vs saved dC", rel=1e-5)


@pytest.mark.parametrize("recompute", [False, True])
def test_graph_step_replays_match_eager(gpu, recompute):
    """The captured forward + fused L2 backward (the bench's step on the smaller workloads),
    replayed three times with eager work and synchronisations in between: every replay gives the
    eager step's image bit for bit, its loss, and its gradients up to the order of the raster
    backward's float atomics."""
    import torch
    import paper_2602_14493_amd as gmr
    say(f"graph step cfg2 scale 0.25, recompute={recompute}")
    W = wl.make_workload(2, scale=0.25)
    r, verts, colors = gpu_setup(W)
    tgt_rgb, _, _, _ = oracle.render_workload(W, verts=W.target_verts)
    target = torch.from_numpy(tgt_rgb.astype(np.float32)).cuda()
    eager = gmr.GraphStep(r, verts, colors, target, recompute=recompute)
    graph = gmr.GraphStep(r, verts, colors, target, recompute=recompute).capture()
    for k in range(3):
        eager._step_body()
        torch.cuda.synchronize()
        graph.graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(graph.rgb, eager.rgb) and torch.equal(graph.alpha, eager.alpha), k
        assert abs(graph.loss.item() - eager.loss.item()) <= 1e-6 * eager.loss.item(), k
        compare_grads(graph.dV, to_np(eager.dV), f"replay {k} dV", rel=1e-5)
        compare_grads(graph.dC, to_np(eager.dC), f"replay {k} dC", rel=1e-5)
        graph.rgb.fill_(float("nan"))      # the next replay must write every pixel again
    assert not graph.overflow()


def test_graph_adam_replays_match_eager(gpu):
    """The captured step (forward, fused L2 backward with recomputed lists, Adam) replayed several
    times tracks the same steps run eagerly; every replay is checked."""
    import torch
    import paper_2602_14493_amd as gmr
    say("graph adam cfg1")
    W = wl.make_workload(1)
    r, verts, colors = gpu_setup(W)
    tgt_rgb, _, _, _ = oracle.render_workload(W, verts=W.target_verts)
    target = torch.from_numpy(tgt_rgb.astype(np.float32)).cuda()
    eager = gmr.GraphAdamLoop(r, verts, colors, target, lr=1e-3)
    graph = gmr.GraphAdamLoop(r, verts, colors, target, lr=1e-3)
    graph.capture()
    assert torch.equal(graph.verts, verts) and int(graph.step_count.item()) == 0   # capture keeps the state
    for k in range(5):
        eager.run_eager(1)
        graph.graph.replay()
        torch.cuda.synchronize()
        d = (eager.verts - graph.verts).abs().max().item()
        say(f"replay {k}: max |dverts| = {d:.3e}  loss eager {eager.loss.item():.6e} graph {graph.loss.item():.6e}")
        assert d <= 1e-5
        assert abs(eager.loss.item() - graph.loss.item()) <= 1e-4 * eager.loss.item()
    assert int(graph.step_count.item()) == 5
    assert not graph.overflow()
    moved = (graph.verts - verts).abs().max().item()
    assert 1e-4 < moved < 1e-2
