"""GPU checks at the full sizes of the larger workloads, plus the rasteriser's block-shape
invariance and the autotuner.

  * UV sphere (399k faces, 4 views 1024^2): gradients through the torch.autograd.Function with the
    sorted lists rebuilt in the backward, against FP64 central differences of the oracle's loss on
    32 seeded random vertices and one pole vertex (whose fan faces fall under Eq. 12's epsilon
    clamp).  Each difference re-renders only the pixel window the vertex's faces cover, with the
    faces whose extents meet that window -- every other pixel's value is unchanged by the move.
  * 16-mesh batch (64 views of 256/512/800 px): one batched launch set equals the per-view
    launches bit for bit; sampled views match the oracle.
"""
import numpy as np
import pytest

import oracle
import workloads as wl
from gmr_testutil import compare_grads, compare_images, gpu_setup, saved_equal, to_np

pytestmark = pytest.mark.gpu
f32 = np.float32


def say(*a):
    print(*a, flush=True)


def test_block_shape_invariance(gpu):
    """1, 2 or 4 pixels per lane (8x8, 8x16, 8x32 blocks per wavefront), either raster schedule and
    either forward list walk (block-uniform or per-lane lists) give bit-identical images and saved
    transmittances; gradients agree to float rounding (atomic order)."""
    import torch
    import paper_2602_14493_amd as gmr
    say("pixels-per-lane invariance cfg2")
    W = wl.make_workload(2)
    r, verts, colors = gpu_setup(W)
    base, base_a, s0, ws0 = r.forward(verts, colors)
    g = torch.randn_like(base)
    dV0, dC0 = r.backward(verts, colors, g, None, s0, ws0)
    pairs_bwd0 = r.counters(ws0).pairs_bwd
    assert r.opts.lane_lists == 1
    for tw, th, px, mode, ll in [(16, 16, 2, 0, 0), (32, 32, 4, 0, 0), (8, 32, 4, 1, 0), (16, 16, 2, 1, 0),
                                 (64, 32, 4, 0, 0), (16, 16, 1, 0, 0), (8, 8, 1, 1, 1), (32, 32, 2, 0, 1),
                                 (32, 32, 4, 1, 1), (64, 32, 4, 0, 1)]:
        cfg = (tw, th, px, mode, ll)
        say("  tile %dx%d px %d mode %d lane lists %d" % cfg)
        r2 = gmr.Renderer(r.batch, W.faces, gmr.default_options(tile_w=tw, tile_h=th, px_per_lane=px,
                                                                raster_mode=mode, lane_lists=ll), handle=r.handle)
        rgb, a, s2, ws2 = r2.forward(verts, colors)
        assert torch.equal(rgb, base), cfg
        assert torch.equal(a, base_a), cfg
        # saved transmittance always; the saved list positions are relative to the tile's list, and
        # the composited lists belong to the raster items (blocks of 8 x 8 px pixels)
        nT = 4 * W.num_pixels
        assert torch.equal(s2[:nT], s0[:nT]), cfg
        if (tw, th) == (r.opts.tile_w, r.opts.tile_h):
            assert torch.equal(s2[:2 * nT], s0[:2 * nT]), cfg
            if px == r.opts.px_per_lane:
                assert saved_equal(r, s2, s0), cfg
        assert r2.counters(ws2).pairs_fwd == r.counters(ws0).pairs_fwd, cfg
        dV, dC = r2.backward(verts, colors, g, None, s2, ws2)
        assert r2.counters(ws2).pairs_bwd == pairs_bwd0, cfg
        compare_grads(dV, to_np(dV0), f"px{px} {tw}x{th} m{mode} l{ll} dV", rel=1e-5)
        compare_grads(dC, to_np(dC0), f"px{px} {tw}x{th} m{mode} l{ll} dC", rel=1e-5)


def test_autotune(gpu):
    """The autotuner returns a valid configuration whose image equals the default's bit for bit."""
    import torch
    say("autotune cfg2")
    W = wl.make_workload(2)
    r, verts, colors = gpu_setup(W)
    base, _, _, _ = r.forward(verts, colors)
    target = torch.zeros_like(base)
    best, ms = r.autotune(verts, colors, target, iters=2)
    say(f"best tile {best.tile_w}x{best.tile_h} px {best.px_per_lane} mode {best.raster_mode}: {ms:.3f} ms")
    assert ms > 0 and best.instance_capacity > 0
    rgb, _, _, ws = r.forward(verts, colors, check=True)
    assert torch.equal(rgb, base)
    best2, ms2 = r.autotune(verts, colors, target, iters=2)  # cached
    assert (best2.tile_w, best2.tile_h, best2.px_per_lane, best2.raster_mode) == \
           (best.tile_w, best.tile_h, best.px_per_lane, best.raster_mode)
    # timed with the lists rebuilt in the backward: its own cache entry, a valid configuration whose
    # recompute backward equals the saved-lists backward of the default configuration
    r3, _, _ = gpu_setup(W)
    g = torch.randn_like(base)
    _, _, s0, ws0 = r3.forward(verts, colors)
    dV0, dC0 = r3.backward(verts, colors, g, None, s0, ws0)
    best3, ms3 = r3.autotune(verts, colors, target, iters=1, recompute=True)
    say(f"recompute: best tile {best3.tile_w}x{best3.tile_h} px {best3.px_per_lane}: {ms3:.3f} ms")
    assert ms3 > 0 and best3.instance_capacity > 0
    rgb3, _, s3, ws3 = r3.forward(verts, colors, check=True)
    assert torch.equal(rgb3, base)
    dV3, dC3 = r3.backward(verts, colors, g, None, s3, r3.new_workspace(), recompute=True)
    compare_grads(dV3, to_np(dV0), "autotuned recompute dV", rel=1e-5)
    compare_grads(dC3, to_np(dC0), "autotuned recompute dC", rel=1e-5)


def test_autotune_view_dependent_colour(gpu):
    """The autotuner with sh_degree 2 (colour gradients of 9 x 3 floats per vertex in its own
    scratch) on the same handle as a degree-0 tuning: each keeps its colour model, and the tuned
    degree-2 image equals the untuned one bit for bit."""
    import torch
    import paper_2602_14493_amd as gmr
    say("autotune sh_degree 2 cfg1")
    W = wl.make_workload(1)
    r0, verts, colors = gpu_setup(W)
    base0, _, _, _ = r0.forward(verts, colors)
    r0.autotune(verts, colors, torch.zeros_like(base0), iters=1)
    r2 = gmr.Renderer(gmr.Batch.from_workload(W), W.faces, gmr.default_options(sh_degree=2), handle=r0.handle)
    C = np.zeros((len(W.verts), 9, 3), np.float32)
    C[:, 0] = W.colors
    C[:, 1:] = np.random.default_rng(3).normal(0, 0.1, size=(len(W.verts), 8, 3))
    c2 = torch.from_numpy(C).cuda()
    base2, _, _, _ = r2.forward(verts, c2)
    best, ms = r2.autotune(verts, c2, torch.zeros_like(base2), iters=1)
    assert best.sh_degree == 2 and r0.opts.sh_degree == 0 and ms > 0
    rgb, _, _, _ = r2.forward(verts, c2, check=True)
    assert torch.equal(rgb, base2)


def _window_submesh(G, faces_of, W, H, margin=2.0):
    """Pixel window covered by the faces in faces_of (from per-face screen records G) and the faces
    whose extents meet it."""
    ok = G[faces_of, 0] > 0
    if not ok.any():
        return None, None
    f = np.asarray(faces_of)[ok]
    u, v, rx, ry = G[f, 1], G[f, 2], G[f, 6], G[f, 7]
    x0 = int(np.floor((u - rx).min() - margin)); x1 = int(np.ceil((u + rx).max() + margin)) + 1
    y0 = int(np.floor((v - ry).min() - margin)); y1 = int(np.ceil((v + ry).max() + margin)) + 1
    x0, y0, x1, y1 = max(0, x0), max(0, y0), min(W, x1), min(H, y1)
    if x0 >= x1 or y0 >= y1:
        return None, None
    allok = G[:, 0] > 0
    meet = allok & (G[:, 1] + G[:, 6] + margin >= x0) & (G[:, 1] - G[:, 6] - margin <= x1) & \
        (G[:, 2] + G[:, 7] + margin >= y0) & (G[:, 2] - G[:, 7] - margin <= y1)
    return (x0, y0, x1, y1), np.nonzero(meet)[0]


def test_cfg3_autograd_recompute_vs_finite_differences(gpu):
    import torch
    import paper_2602_14493_amd as gmr
    say("cfg3 UV sphere 399k faces, 4x1024^2: autograd (recompute lists) vs FP64 FD")
    W = wl.make_workload(3)
    r, verts, colors = gpu_setup(W)
    P = W.num_pixels
    cams = W.cam_array()
    tgt, _, _, _ = oracle.render_workload(W, verts=W.target_verts)
    o_rgb, o_tf, _, o_mask = oracle.render_workload(W)
    say(f"oracle masked fraction {o_mask.mean():.2e}")
    weight = (~o_mask).astype(np.float64)
    target = torch.from_numpy(tgt.astype(f32)).cuda()
    wt = torch.from_numpy(weight.astype(f32)).cuda()
    v = verts.clone().requires_grad_(True)
    c = colors.clone().requires_grad_(True)
    rgb, alpha = gmr.render(v, c, r, save_lists=False)
    compare_images(rgb.detach(), alpha.detach(), o_rgb, o_tf, o_mask, label="cfg3")
    loss = (((rgb - target) ** 2) * wt[:, None]).sum() / (3 * P)
    loss.backward()
    dV = to_np(v.grad).astype(np.float64)
    scale = np.abs(dV).max()
    rng = np.random.default_rng(33)
    faces = W.faces
    vids = list(rng.choice(len(W.verts), 32, replace=False)) + [1]   # vertex 1: first ring, pole fan
    inc = {int(vid): np.nonzero((faces == vid).any(1))[0] for vid in vids}
    pole_faces = inc[1]
    areas = 0.5 * np.linalg.norm(np.cross(W.verts[faces[pole_faces, 1]].astype(float) - W.verts[faces[pole_faces, 0]],
                                          W.verts[faces[pole_faces, 2]].astype(float) - W.verts[faces[pole_faces, 0]]), axis=1)
    assert (areas < 1.0392e-6).any(), "the pole vertex should touch clamped faces"
    Gs = [oracle.gaussians(W.verts, faces, W.colors, cams[k]) for k in range(W.num_views)]
    po = W.pixel_offsets()
    checked, worst = 0, 0.0
    for vid in vids:
        vid = int(vid)
        views = []
        for k in range(W.num_views):
            win, sub = _window_submesh(Gs[k], inc[vid], W.cams[k].width, W.cams[k].height)
            if win is not None:
                views.append((k, win, sub))
        if not views:
            continue

        def local(k, win, sub, Vx):
            x0, y0, x1, y1 = win
            Wk = W.cams[k].width
            idx = (po[k] + (np.arange(y0, y1)[:, None] * Wk + np.arange(x0, x1)[None, :])).reshape(-1)
            return idx

        def loss_fn(Vx):
            tot = 0.0
            for k, win, sub in views:
                rgbw, _, _, _ = oracle.render_view(Vx, faces[sub], W.colors, cams[k], window=win)
                idx = local(k, win, sub, Vx)
                d = rgbw.reshape(-1, 3) - tgt[idx]
                tot += float((weight[idx][:, None] * d * d).sum())
            return tot / (3 * P)

        def decisions(Vx):
            return b"".join(oracle.render_view(Vx, faces[sub], W.colors, cams[k], window=win, want_hash=True)[4].tobytes()
                            for k, win, sub in views)

        fd = oracle.fd_vertex_grad(loss_fn, W.verts, vid, h=1e-6, decision_fn=decisions)
        for a in range(3):
            if fd[a] is None:
                continue
            err = abs(dV[vid, a] - fd[a])
            bound = 1e-3 * abs(fd[a]) + 1e-5 * scale
            worst = max(worst, err / bound)
            checked += 1
            assert err <= bound, (vid, a, dV[vid, a], fd[a])
    say(f"checked {checked} coordinates, worst err/bound {worst:.3f}")
    assert checked >= 60


def test_cfg4_batched_equals_per_view_and_oracle(gpu):
    import torch
    import paper_2602_14493_amd as gmr
    say("cfg4 16 meshes / 64 views: batched vs per-view")
    W = wl.make_workload(4)
    r, verts, colors = gpu_setup(W)
    rgb, alpha, saved, ws = r.forward(verts, colors)
    po = W.pixel_offsets()
    for v in range(W.num_views):
        bv = r.batch.view(v)
        v0, v1, f0, f1 = bv.mesh_range
        rv = gmr.Renderer(bv, W.faces[f0:f1] - v0, gmr.copy_options(r.opts, instance_capacity=0),
                          handle=r.handle)
        rgb_v, a_v, _, _ = rv.forward(verts[v0:v1].contiguous(), colors[v0:v1].contiguous())
        assert torch.equal(rgb_v, rgb[po[v]:po[v + 1]]), v
        assert torch.equal(a_v, alpha[po[v]:po[v + 1]]), v
    cams = W.cam_array()
    for v in [0, 17, 40, W.num_views - 1]:
        m = int(W.view_mesh[v])
        mv, mf, mc = W.mesh(m)
        o_rgb, o_tf, _, o_mask = oracle.render_view(mv, mf, mc, cams[v], gid_base=int(W.face_offsets[m]))
        compare_images(to_np(rgb)[po[v]:po[v + 1]], to_np(alpha)[po[v]:po[v + 1]], o_rgb.reshape(-1, 3),
                       o_tf.reshape(-1), o_mask.reshape(-1), label=f"cfg4 view {v}")


def test_cfg4_batched_grads_two_meshes(gpu):
    """16-mesh batch (64 views) in one launch set, bench tiling (32 x 16): vertex and colour
    gradients of a random upstream gradient (colour and alpha) on a 64 x 64 crop of one view of the
    smallest mesh and one of the largest, vs the oracle's adjoint of those views.  The batch's
    vertices are global indices into one CSR gather: every other mesh's gradient must be zero."""
    import torch
    say("cfg4 16 meshes / 64 views: batched gradients of two meshes")
    W = wl.make_workload(4)
    r, verts, colors = gpu_setup(W, tile_w=32, tile_h=16)
    rgb, alpha, saved, ws = r.forward(verts, colors)
    F = np.diff(W.face_offsets)
    ms = sorted(set(int(m) for m in W.view_mesh))
    m_small, m_large = min(ms, key=lambda m: F[m]), max(ms, key=lambda m: F[m])
    views = [int(np.flatnonzero(W.view_mesh == m_small)[0]), int(np.flatnonzero(W.view_mesh == m_large)[-1])]
    po = W.pixel_offsets()
    cams = W.cam_array()
    rng = np.random.default_rng(44)
    g = np.zeros((W.num_pixels, 3), np.float32)
    ga = np.zeros(W.num_pixels, np.float32)
    oV, oC = np.zeros(W.verts.shape), np.zeros(W.colors.shape)
    for v in views:
        m = int(W.view_mesh[v])
        mv, mf, mc = W.mesh(m)
        v0, v1, f0 = int(W.vert_offsets[m]), int(W.vert_offsets[m + 1]), int(W.face_offsets[m])
        Wv, Hv = W.cams[v].width, W.cams[v].height
        o_rgb, o_tf, _, o_mask = oracle.render_view(mv, mf, mc, cams[v], gid_base=f0)
        cov = (1.0 - o_tf) > 0.5
        # the 64 x 64 window (16-px grid) nearest the centre whose coverage is closest to 3/4
        best = min(((abs(cov[y:y + 64, x:x + 64].mean() - 0.75), (y - Hv / 2) ** 2 + (x - Wv / 2) ** 2, y, x)
                    for y in range(0, Hv - 63, 16) for x in range(0, Wv - 63, 16)))
        _, _, y, x = best
        keep = ~o_mask[y:y + 64, x:x + 64]
        gr = (rng.normal(size=(64, 64, 3)) * keep[..., None]).astype(np.float32)
        gal = (0.1 * rng.normal(size=(64, 64)) * keep).astype(np.float32)
        say(f"view {v} (mesh {m}, {F[m]} faces, {Wv}x{Hv}): crop at ({x}, {y}), "
            f"coverage {cov[y:y + 64, x:x + 64].mean():.2f}")
        rows = po[v] + (np.arange(y, y + 64)[:, None] * Wv + np.arange(x, x + 64)[None, :]).reshape(-1)
        g[rows] = gr.reshape(-1, 3)
        ga[rows] = gal.reshape(-1)
        dv, dc = oracle.adjoint_view(mv, mf, mc, cams[v], gr.astype(np.float64), gal.astype(np.float64),
                                     gid_base=f0, window=(x, y, x + 64, y + 64))
        oV[v0:v1] += dv
        oC[v0:v1] += dc
    dV, dC = r.backward(verts, colors, torch.from_numpy(g).cuda(), torch.from_numpy(ga).cuda(), saved, ws)
    for m in (m_small, m_large):
        v0, v1 = int(W.vert_offsets[m]), int(W.vert_offsets[m + 1])
        compare_grads(dV[v0:v1], oV[v0:v1], f"cfg4 mesh {m} dV")
        compare_grads(dC[v0:v1], oC[v0:v1], f"cfg4 mesh {m} dC")
    others = np.ones(len(W.verts), bool)
    for m in (m_small, m_large):
        others[int(W.vert_offsets[m]):int(W.vert_offsets[m + 1])] = False
    assert float(dV[torch.from_numpy(others).cuda()].abs().max()) == 0.0
    assert float(dC[torch.from_numpy(others).cuda()].abs().max()) == 0.0


@pytest.mark.parametrize("cfg", [3, 4])
def test_tile_lists_bit_exact_large_inputs(gpu, cfg):
    """Every tile list of the UV sphere (1.6M face-views) and of the 16-mesh batch (64 views)
    against the oracle's, at full size in the bench's default tiling.  These inputs take the
    large-input paths the 8-view icosphere does not: 4096-face-view blocks of the one-pass
    scan + emission (look-back over hundreds of blocks), 4096-element onesweep partitions for the
    depth and tile digits."""
    from gmr_testutil import fv_to_face, workspace_lists
    W = wl.make_workload(cfg)
    r, verts, colors = gpu_setup(W, tile_w=16, tile_h=16)
    rgb, alpha, saved, ws = r.forward(verts, colors)
    cnt = r.counters(ws)
    fv = sum(int(W.face_offsets[m + 1] - W.face_offsets[m]) for m in W.view_mesh)
    say(f"cfg{cfg}: {fv} face-views, {cnt.instances} instances")
    assert not cnt.overflow
    assert fv >= (1 << 20) and cnt.instances >= (1 << 18), "the workload must take the large-input paths"
    ranges, vals = workspace_lists(r, ws)
    vv_all, gl_all = fv_to_face(W)(vals[:cnt.instances])
    cams = W.cam_array()
    tbase, checked = 0, 0
    for v in range(W.num_views):
        m = int(W.view_mesh[v])
        mv, mf, mc = W.mesh(m)
        f0 = int(W.face_offsets[m])
        off, ids, amb = oracle.tile_lists_view(mv, mf, mc, cams[v], 16, 16, gid_base=f0)
        nt = len(off) - 1
        rv = ranges[tbase:tbase + nt].astype(np.int64)
        ne = rv[:, 1] > rv[:, 0]
        if ne.any():  # tile ids are view-major: view v's instances are one run
            assert (vv_all[rv[ne, 0].min():rv[ne, 1].max()] == v).all(), f"view {v}"
        for t in range(nt):
            s, e = rv[t]
            gl = gl_all[s:e]
            o_ids, o_amb = ids[off[t]:off[t + 1]], amb[off[t]:off[t + 1]]
            if not o_amb.any():  # no entry near an extent margin: the lists must be identical
                assert np.array_equal(gl, o_ids), f"view {v} tile {t}"
                checked += len(o_ids)
                continue
            ambiguous = set(o_ids[o_amb != 0].tolist())
            want = [i for i, a in zip(o_ids.tolist(), o_amb.tolist()) if a == 0]
            assert [i for i in gl.tolist() if i not in ambiguous] == want, f"view {v} tile {t}"
            assert set(gl.tolist()) <= set(o_ids.tolist()), f"view {v} tile {t}"
            checked += len(want)
        tbase += nt
    say(f"checked {checked} list entries")
    assert checked >= cnt.instances // 2


def test_bench_json_contract(gpu):
    """bench.py prints one JSON line with the fields its contract names, on a small run."""
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    cmd = [sys.executable, os.path.join(root, "bench.py"), "--config", "1", "--steps", "3", "--warmup", "1",
           "--no-per-view", "--cpu-seconds", "0.5"]
    say("bench contract: " + " ".join(cmd[1:]))
    out = subprocess.run(cmd, capture_output=True, text=True, timeout=110)
    assert out.returncode == 0, out.stderr[-2000:]
    lines = [l for l in out.stdout.splitlines() if l.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 3 and d["warmup"] == 1 and d["value"] > 0
    assert d["config"]["workload"] == "icosphere_s2_1x128"
    rf = d["roofline"]
    assert rf["bound"] in ("hbm", "alu") and rf["peak"] > 0
    assert rf["frac"] == pytest.approx(rf["achieved"] / rf["peak"], rel=2e-2, abs=1e-6)
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["cores"] >= 1
