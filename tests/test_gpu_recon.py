"""Parity of the reconstruction step around the renderer (Sec. 3.1: colour MSE + silhouette BCE
backward, edge-length and Laplacian regularisers, VectorAdam) with the FP64 oracle, through the C
ABI, and the captured step against the same step run eagerly.

Tolerances: losses 1e-5 relative where the arithmetic is a float32 sum of P terms checked against
the same terms in FP64 (1e-4 for the regularisers, whose per-vertex Laplacian is a float32
difference of nearby coordinates); gradients as the renderer's parity tests (||d||/||g|| <= 1e-3,
per element 1e-3 |g| + 1e-5 max|g|); VectorAdam parameters 1e-6 absolute after five steps."""
import numpy as np
import pytest

import oracle
import workloads as wl
from gmr_testutil import compare_grads, gpu_setup, to_np
from oracle import recon

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def _silhouette(W):
    """Binary target mask: the oracle's alpha of the target mesh above one half."""
    _, tf, _, _ = oracle.render_workload(W, verts=W.target_verts)
    return (1.0 - tf > 0.5).astype(np.float64)


@pytest.mark.parametrize("k,scale", [(1, 1.0), (2, 0.25)])
def test_recon_backward_vs_oracle(gpu, k, scale):
    import torch
    say(f"recon backward cfg{k} scale {scale}")
    W = wl.make_workload(k, scale=scale)
    r, verts, colors = gpu_setup(W)
    tgt, _, _, _ = oracle.render_workload(W, verts=W.target_verts)
    sil = _silhouette(W)
    target = torch.from_numpy(tgt.astype(np.float32)).cuda()
    mask = torch.from_numpy(sil.astype(np.float32)).cuda()
    cw, sw = 0.7, 0.4
    rgb, alpha, saved, ws = r.forward(verts, colors)
    dV, dC, losses = r.backward_recon(verts, colors, rgb, target, mask, saved, ws, color_weight=cw, sil_weight=sw)
    c = r.counters(ws)
    losses = to_np(losses).astype(np.float64)
    assert c.loss == pytest.approx(losses[0], rel=1e-7) and c.loss_sil == pytest.approx(losses[1], rel=1e-7)

    # the fused terms against the same terms in FP64 from the GPU's own image; alpha is taken as
    # 1 - T_final from the saved state (the float32 alpha output rounds away T's low bits, which
    # the BCE derivative 1 / (alpha (1 - alpha)) magnifies near opaque pixels)
    T = saved.view(torch.float32)[:W.num_pixels]
    g_rgb_np, g_a_np = to_np(rgb).astype(np.float64), 1.0 - to_np(T).astype(np.float64)
    Lc_g, gr_g = oracle.l2_loss(g_rgb_np, tgt)
    Ls_g, ga_g = recon.silhouette_bce(g_a_np, sil, weight=sw)
    say(f"losses gpu {losses} fp64-of-gpu-image {cw * Lc_g:.8e} {Ls_g:.8e}")
    assert losses[0] == pytest.approx(cw * Lc_g, rel=1e-5)
    assert losses[1] == pytest.approx(Ls_g, rel=1e-5)
    dV2, dC2 = r.backward(verts, colors, torch.from_numpy((cw * gr_g).astype(np.float32)).cuda(),
                          torch.from_numpy(ga_g.astype(np.float32)).cuda(), saved, ws)
    compare_grads(dV, to_np(dV2), "fused recon vs explicit dV", rel=1e-5)
    compare_grads(dC, to_np(dC2), "fused recon vs explicit dC", rel=1e-5)

    # against the oracle's image and adjoint
    o_rgb, o_tf, _, o_mask = oracle.render_workload(W)
    Lc, g_rgb = oracle.l2_loss(o_rgb, tgt)
    Ls, g_a = recon.silhouette_bce(1.0 - o_tf, sil, weight=sw)
    g_rgb = cw * g_rgb
    if not o_mask.any():
        assert losses[0] == pytest.approx(cw * Lc, rel=1e-5)
        assert losses[1] == pytest.approx(Ls, rel=1e-5)
        oV, oC = oracle.adjoint_workload(W, g_rgb, g_a)
        compare_grads(dV, oV, f"cfg{k} recon dV vs oracle")
        compare_grads(dC, oC, f"cfg{k} recon dC vs oracle")
    else:
        keep = ~o_mask
        g_rgb = g_rgb * keep[:, None]
        g_a = g_a * keep
        dV3, dC3 = r.backward(verts, colors, torch.from_numpy(g_rgb.astype(np.float32)).cuda(),
                              torch.from_numpy(g_a.astype(np.float32)).cuda(), saved, ws)
        oV, oC = oracle.adjoint_workload(W, g_rgb, g_a)
        compare_grads(dV3, oV, f"cfg{k} recon (masked) dV vs oracle")
        compare_grads(dC3, oC, f"cfg{k} recon (masked) dC vs oracle")


def test_recon_silhouette_only_and_clamp(gpu):
    """Colour weight 0 leaves the silhouette gradient alone; an all-background view (every pixel at
    alpha = 0, inside the clamp) gives the closed-form loss -log(1 - 1e-6) or -log(1e-6) per pixel
    and a zero gradient."""
    import torch
    W = wl.make_workload(1)
    r, verts, colors = gpu_setup(W)
    P = W.num_pixels
    far = verts + torch.tensor([0.0, 0.0, 100.0], device=verts.device)   # behind the camera: culled
    rgb, alpha, saved, ws = r.forward(far, colors)
    assert float(alpha.abs().max()) == 0.0
    for s_val, want in [(0.0, -np.log1p(-1e-6)), (1.0, -np.log(1e-6))]:
        mask = torch.full((P,), s_val, dtype=torch.float32, device=verts.device)
        dV, dC, losses = r.backward_recon(far, colors, rgb, rgb, mask, saved, ws, color_weight=0.0,
                                          sil_weight=1.0)
        l = to_np(losses)
        say(f"empty view, mask {s_val}: losses {l}")
        assert l[0] == 0.0
        assert l[1] == pytest.approx(want, rel=1e-4)
        assert float(dV.abs().max()) == 0.0 and float(dC.abs().max()) == 0.0
    sil = _silhouette(W)
    mask = torch.from_numpy(sil.astype(np.float32)).cuda()
    rgb, alpha, saved, ws = r.forward(verts, colors)
    dV, dC, losses = r.backward_recon(verts, colors, rgb, rgb, mask, saved, ws, color_weight=0.0, sil_weight=1.0)
    T = saved.view(torch.float32)[:P]
    _, ga = recon.silhouette_bce(1.0 - to_np(T).astype(np.float64), sil)
    dV2, dC2 = r.backward(verts, colors, torch.zeros_like(rgb), torch.from_numpy(ga.astype(np.float32)).cuda(),
                          saved, ws)
    compare_grads(dV, to_np(dV2), "silhouette-only dV", rel=1e-5)
    assert float(to_np(losses)[0]) == 0.0


def _graph(faces, nv):
    import paper_2602_14493_amd as gmr
    return gmr.MeshGraph(faces, nv, 0)


def _reg_mesh(name):
    rng = np.random.default_rng(3)
    if name == "icosphere3":
        v, f = wl.icosphere(3)
    elif name == "uv_sphere":                          # pole vertices of degree 40
        v, f = wl.uv_sphere(40, 30)
    else:                                              # two meshes back to back, as in a batch
        v1, f1 = wl.torus(30, 20)
        v2, f2 = wl.icosphere(2)
        v, f = np.concatenate([v1, v2 + 3.0]), np.concatenate([f1, f2 + len(v1)]).astype(np.int32)
    return v + rng.normal(0.0, 0.01, v.shape), f


@pytest.mark.parametrize("name", ["icosphere3", "uv_sphere", "torus+icosphere"])
def test_regularizers_vs_oracle(gpu, name):
    import torch
    verts, faces = _reg_mesh(name)
    say(f"regularisers on {name}: V={len(verts)} F={len(faces)}")
    g = _graph(faces, len(verts))
    edges = recon.mesh_edges(faces)
    nb = recon.neighbours(len(verts), edges)
    v = torch.from_numpy(verts.astype(np.float32)).cuda()
    v64 = verts.astype(np.float32).astype(np.float64)
    for l0, we, wlap in [(0.0, 1.0, 1.0), (0.05, 2.5, 0.0), (0.0, 0.0, 0.3)]:
        # a small incoming gradient, so that d - base carries no rounding of note
        base = 1e-3 * torch.randn(v.shape, device=v.device, generator=torch.Generator(device="cuda").manual_seed(7))
        d, losses = g.regularizers(v, base.clone(), l0, we, wlap)
        Le, ge = recon.edge_length(v64, edges, l0=l0, weight=we)
        Ll, gl = recon.laplacian_smoothing(v64, nb, weight=wlap)
        l = to_np(losses).astype(np.float64)
        say(f"l0={l0} we={we} wl={wlap}: gpu {l} fp64 {Le:.8e} {Ll:.8e}")
        assert l[0] == pytest.approx(Le, rel=1e-4, abs=1e-30)
        assert l[1] == pytest.approx(Ll, rel=1e-4, abs=1e-30)
        compare_grads(d - base, ge + gl, f"{name} regulariser grad l0={l0} we={we} wl={wlap}")
    # determinism: no float atomics on the gradient
    d1, _ = g.regularizers(v)
    d2, _ = g.regularizers(v)
    assert torch.equal(d1, d2)


def test_vector_adam_vs_oracle(gpu):
    import torch
    import paper_2602_14493_amd as gmr
    rng = np.random.default_rng(11)
    V = 1000
    p = rng.normal(size=(V, 3)).astype(np.float32)
    gs = [rng.normal(size=(V, 3)).astype(np.float32) for _ in range(5)]
    for gg in gs:
        gg[17] = 0.0                                   # a vertex that never receives a gradient
    pt = torch.from_numpy(p).cuda()
    m = torch.zeros_like(pt)
    vv = torch.zeros((V,), dtype=torch.float32, device=pt.device)
    step = torch.zeros((1,), dtype=torch.int32, device=pt.device)
    po, mo, vo = p.astype(np.float64), np.zeros((V, 3)), np.zeros(V)
    for t, gg in enumerate(gs, start=1):
        gmr.vector_adam_step(pt, torch.from_numpy(gg).cuda(), m, vv, step, lr=1e-2)
        # the kernel receives the hyper-parameters as float32: give the oracle the same values
        po, mo, vo = recon.vector_adam_step(po, gg.astype(np.float64), mo, vo, t, lr=float(np.float32(1e-2)),
                                            b1=float(np.float32(0.9)), b2=float(np.float32(0.999)),
                                            eps=float(np.float32(1e-8)))
        err = np.abs(to_np(pt).astype(np.float64) - po).max()
        say(f"vector adam step {t}: max |dp| = {err:.3e}")
        assert err <= 1e-6
    assert int(step.item()) == 5
    np.testing.assert_allclose(to_np(vv), vo, rtol=1e-5)
    assert np.array_equal(to_np(pt)[17], p[17])


def test_recon_loop_graph_matches_eager_and_descends(gpu):
    """The captured reconstruction step replayed tracks the eager step (every replay checked), and
    from the jittered sphere towards the target the weighted objective goes down."""
    import torch
    import paper_2602_14493_amd as gmr
    say("recon loop cfg1")
    W = wl.make_workload(1)
    r, verts, colors = gpu_setup(W)
    tgt, _, _, _ = oracle.render_workload(W, verts=W.target_verts)
    target = torch.from_numpy(tgt.astype(np.float32)).cuda()
    mask = torch.from_numpy(_silhouette(W).astype(np.float32)).cuda()
    w = gmr.ReconWeights(color=1.0, silhouette=0.1, edge=0.01, laplacian=0.01)
    eager = gmr.ReconLoop(r, verts, colors, target, mask, w, lr=1e-3)
    graph = gmr.ReconLoop(r, verts, colors, target, mask, w, lr=1e-3)
    graph.capture()
    assert torch.equal(graph.verts, verts) and int(graph.step_count.item()) == 0   # capture keeps the state
    for k in range(5):
        eager.run_eager(1)
        graph.graph.replay()
        torch.cuda.synchronize()
        d = (eager.verts - graph.verts).abs().max().item()
        le, lg = to_np(eager.losses), to_np(graph.losses)
        say(f"replay {k}: max |dverts| = {d:.3e} losses eager {le} graph {lg}")
        assert d <= 1e-5
        np.testing.assert_allclose(lg, le, rtol=1e-4)
    assert int(graph.step_count.item()) == 5
    first = to_np(graph.losses).sum()
    graph.run(60)
    torch.cuda.synchronize()
    last = to_np(graph.losses).sum()
    say(f"objective after 5 steps {first:.6e}, after 65 {last:.6e}")
    assert np.isfinite(last) and last < first
    assert not graph.overflow()


def _vector_adam_update_tolerance(p, g, m, v, t, hp, rel):
    """How far VectorAdam's new vertices can move when each gradient element moves within the
    gradient tolerance: the largest deviation over the 8 sign patterns of that bound per vertex."""
    bound = np.where(g == 0.0, 0.0, rel * np.abs(g) + 1e-5 * np.abs(g).max())
    base, _, _ = recon.vector_adam_step(p, g, m, v, t, **hp)
    tol = np.zeros_like(p)
    for sx in (-1, 1):
        for sy in (-1, 1):
            for sz in (-1, 1):
                q, _, _ = recon.vector_adam_step(p, g + bound * np.array([sx, sy, sz]), m, v, t, **hp)
                tol = np.maximum(tol, np.abs(q - base))
    return base, tol


def test_recon_loop_steps_vs_oracle_chain(gpu):
    """Icosphere subdiv 2 at 128^2: three replays of the captured reconstruction step (colour MSE
    1, silhouette BCE 0.1, edge length 0.01, Laplacian 0.01; VectorAdam lr 1e-3).  Before each
    replay the GPU state is read; the oracle takes the same step from it: render -> both image
    losses and their adjoint -> + the regulariser gradients -> VectorAdam.  Checked per step: the
    four losses, the gradient the step applied (the loop's dV buffer), the update given the GPU's
    gradient (tight) and the update given the oracle's (within what the gradient tolerance
    allows)."""
    import torch
    import paper_2602_14493_amd as gmr
    from gmr_testutil import GRAD_REL, flagged_pixels_agree
    say("recon loop vs oracle chain, cfg1")
    W = wl.make_workload(1)
    r, verts, colors = gpu_setup(W)
    tgt, _, _, _ = oracle.render_workload(W, verts=W.target_verts)
    sil = _silhouette(W)
    target = torch.from_numpy(tgt.astype(np.float32)).cuda()
    mask = torch.from_numpy(sil.astype(np.float32)).cuda()
    w = gmr.ReconWeights(color=1.0, silhouette=0.1, edge=0.01, laplacian=0.01)
    lr = 1e-3
    hp = dict(lr=float(np.float32(lr)), b1=float(np.float32(0.9)), b2=float(np.float32(0.999)),
              eps=float(np.float32(1e-8)))
    loop = gmr.ReconLoop(r, verts, colors, target, mask, w, lr=lr)
    loop.capture()
    edges = recon.mesh_edges(W.faces)
    nb = recon.neighbours(len(W.verts), edges)
    loose_total, compared = 0, 0
    for t in range(1, 4):
        p0 = to_np(loop.verts).astype(np.float64)
        m0 = to_np(loop.m).astype(np.float64)
        v0 = to_np(loop.v).astype(np.float64)
        loop.graph.replay()
        torch.cuda.synchronize()
        assert int(loop.step_count.item()) == t and not loop.overflow()
        dV = to_np(loop.dV).astype(np.float64)
        pg, mg, vg = recon.vector_adam_step(p0, dV, m0, v0, t, **hp)
        p1 = to_np(loop.verts).astype(np.float64)
        e = np.abs(p1 - pg).max()
        say(f"  step {t}: |p - vector_adam(p0, dV_gpu)| max {e:.3e}")
        assert e <= 1e-6
        np.testing.assert_allclose(to_np(loop.m), mg, rtol=1e-5, atol=1e-6 * np.abs(mg).max())
        np.testing.assert_allclose(to_np(loop.v), vg, rtol=1e-5, atol=1e-6 * np.abs(vg).max())
        o_rgb, o_tf, _, o_mask = oracle.render_workload(W, verts=p0.astype(np.float32))
        # a pixel near a decision threshold counts only where both sides took the same decisions
        # (its image value); else the oracle comparison of this step is skipped
        if not flagged_pixels_agree(loop.rgb, loop.alpha, o_rgb, o_tf, o_mask):
            say(f"  step {t}: flagged pixels disagree, oracle comparison skipped")
            continue
        compared += 1
        Lc, g_rgb = oracle.l2_loss(o_rgb, tgt)
        Ls, g_a = recon.silhouette_bce(1.0 - o_tf, sil, weight=w.silhouette)
        Le, ge = recon.edge_length(p0, edges, l0=w.edge_length, weight=w.edge)
        Ll, gl = recon.laplacian_smoothing(p0, nb, weight=w.laplacian)
        lg = to_np(loop.losses).astype(np.float64)
        say(f"  step {t}: losses gpu {lg} oracle {[w.color * Lc, Ls, Le, Ll]}")
        assert lg[0] == pytest.approx(w.color * Lc, rel=1e-5)
        assert lg[1] == pytest.approx(Ls, rel=1e-5)
        assert lg[2] == pytest.approx(Le, rel=1e-4)
        assert lg[3] == pytest.approx(Ll, rel=1e-4)
        oV, _ = oracle.adjoint_workload(W, w.color * g_rgb, g_a, verts=p0.astype(np.float32))
        oV = oV + ge + gl
        compare_grads(dV, oV, f"step {t} dV (renderer + regularisers)")
        po, tol = _vector_adam_update_tolerance(p0, oV, m0, v0, t, hp, GRAD_REL)
        d = np.abs(p1 - po)
        assert (d <= tol + 1e-6).all(), np.argwhere(d > tol + 1e-6)[:5]
        loose = (tol > 0.1 * lr).any(axis=1)
        loose_total += int(loose.sum())
        say(f"  step {t}: |p - vector_adam(p0, dV_oracle)| max {d.max():.3e}; {int(loose.sum())} vertices "
            f"whose gradient is within its tolerance of zero")
    assert compared >= 2, "the oracle comparison ran on fewer than two of the three steps"
    assert loose_total <= 0.05 * 3 * len(W.verts)


def test_synthetic_reconstruction_converges(gpu):
    """A small version of the synthetic-target experiment (Sec. 3.1): a 2,880-face sphere fitted to
    the 'blob' target from 32 hemisphere views at 96^2, 4 views per iteration.  The chamfer distance
    must fall by 10x and the normal consistency rise; every step goes through the C ABI."""
    from paper_2602_14493_amd import experiments as ex
    cfg = ex.ReconConfig(target="blob", target_freq=10, init_freq=12, views=32, size=96, batch=4, iters=600,
                         samples=4000, log_every=200)
    res = ex.run(cfg, verbose=True)
    say(f"CD {res['cd_init']:.3e} -> {res['cd']:.3e}, NC {res['nc_init']:.4f} -> {res['nc']:.4f}, "
        f"{res['iters_per_s']:.0f} it/s")
    assert res["cd"] < 0.1 * res["cd_init"]
    assert res["nc"] > res["nc_init"]
    assert res["overflow_events"] == 0


def test_recon_backward_with_recompute_and_options(gpu):
    """The reconstruction backward rebuilding its lists equals the one reusing the forward's, with
    view-dependent colour and with the baseline conversion (options compose with the loss)."""
    import torch
    W = wl.make_workload(2, scale=0.25)
    tgt, _, _, _ = oracle.render_workload(W, verts=W.target_verts)
    target = torch.from_numpy(tgt.astype(np.float32)).cuda()
    mask = torch.from_numpy(_silhouette(W).astype(np.float32)).cuda()
    for kw in ({"sh_degree": 2}, {"cov_mode": 2}):
        say(f"recon backward, recompute vs saved lists, {kw}")
        r, verts, colors = gpu_setup(W, **kw)
        if "sh_degree" in kw:
            C = np.zeros((len(W.verts), 9, 3), np.float32)
            C[:, 0] = W.colors
            C[:, 1:] = np.random.default_rng(5).normal(0, 0.1, size=(len(W.verts), 8, 3))
            colors = torch.from_numpy(C).cuda()
        rgb, alpha, saved, ws = r.forward(verts, colors)
        dV0, dC0, l0 = r.backward_recon(verts, colors, rgb, target, mask, saved, ws, sil_weight=0.5)
        dV1, dC1, l1 = r.backward_recon(verts, colors, rgb, target, mask, saved, None, sil_weight=0.5)
        compare_grads(dV1, to_np(dV0), f"recompute vs saved dV {kw}", rel=1e-5)
        compare_grads(dC1, to_np(dC0), f"recompute vs saved dC {kw}", rel=1e-5)
        np.testing.assert_allclose(to_np(l1), to_np(l0), rtol=1e-6)


def test_autograd_with_view_dependent_colour(gpu):
    """torch.autograd through render() with sh_degree 1: the coefficient and vertex gradients equal
    the explicit backward's, with the lists kept and rebuilt."""
    import torch
    import paper_2602_14493_amd as gmr
    W = wl.make_workload(1)
    r, verts, _ = gpu_setup(W, sh_degree=1)
    C = np.zeros((len(W.verts), 4, 3), np.float32)
    C[:, 0] = W.colors
    C[:, 1:] = np.random.default_rng(6).normal(0, 0.2, size=(len(W.verts), 3, 3))
    grads = []
    for save in (True, False):
        v = verts.clone().requires_grad_()
        c = torch.from_numpy(C).cuda().requires_grad_()
        rgb, alpha = gmr.render(v, c, r, save_lists=save)
        (rgb.square().mean() + 0.3 * alpha.mean()).backward()
        grads.append((v.grad.clone(), c.grad.clone()))
    assert grads[0][1].shape == (len(W.verts), 4, 3)
    compare_grads(grads[1][0], to_np(grads[0][0]), "autograd sh1 recompute vs saved dV", rel=1e-5)
    compare_grads(grads[1][1], to_np(grads[0][1]), "autograd sh1 recompute vs saved dC", rel=1e-5)
    rgb, alpha, saved, ws = r.forward(verts, torch.from_numpy(C).cuda())
    g = 2.0 * rgb / rgb.numel()
    ga = torch.full_like(alpha, 0.3 / alpha.numel())
    dV, dC = r.backward(verts, torch.from_numpy(C).cuda(), g, ga, saved, ws)
    compare_grads(grads[0][0], to_np(dV), "autograd sh1 vs explicit dV", rel=1e-5)
    compare_grads(grads[0][1], to_np(dC), "autograd sh1 vs explicit dC", rel=1e-5)


def test_input_layout_checked_before_launch(gpu):
    """Colours in the wrong layout for the colour model, or vertices of the wrong size, are refused
    on the host before any kernel sees them."""
    import torch
    W = wl.make_workload(1)
    r, verts, colors = gpu_setup(W, sh_degree=2)
    with pytest.raises(ValueError):
        r.forward(verts, colors)                           # [V,3] where [V,9,3] is expected
    C = torch.zeros((len(W.verts), 9, 3), device=verts.device)
    with pytest.raises(ValueError):
        r.forward(verts[:-1], C)
    rgb, alpha, saved, ws = r.forward(verts, C)
    with pytest.raises(ValueError):
        r.backward(verts, colors, torch.zeros_like(rgb), None, saved, ws)


def test_recon_and_view_dependent_colour_full_size(gpu):
    """The 8-view 512^2 icosphere at full size, in the launch configuration the bench times: the
    reconstruction backward (colour + silhouette) and, separately, sh_degree 3 colour against the
    oracle's image and adjoint (pixels the oracle flags near a threshold are left out of the
    upstream gradients)."""
    import torch
    W = wl.make_workload(2)
    tgt, _, _, _ = oracle.render_workload(W, verts=W.target_verts)
    sil = _silhouette(W)
    # reconstruction backward
    r, verts, colors = gpu_setup(W)
    target = torch.from_numpy(tgt.astype(np.float32)).cuda()
    mask = torch.from_numpy(sil.astype(np.float32)).cuda()
    rgb, alpha, saved, ws = r.forward(verts, colors)
    o_rgb, o_tf, _, o_mask = oracle.render_workload(W)
    from gmr_testutil import compare_images
    compare_images(rgb, alpha, o_rgb, o_tf, o_mask, label="cfg2 full")
    keep = ~o_mask
    _, g_rgb = oracle.l2_loss(o_rgb, tgt)
    _, g_a = recon.silhouette_bce(1.0 - o_tf, sil, weight=0.5)
    g_rgb, g_a = g_rgb * keep[:, None], g_a * keep
    dV, dC = r.backward(verts, colors, torch.from_numpy(g_rgb.astype(np.float32)).cuda(),
                        torch.from_numpy(g_a.astype(np.float32)).cuda(), saved, ws)
    oV, oC = oracle.adjoint_workload(W, g_rgb, g_a)
    compare_grads(dV, oV, "cfg2 full recon upstream dV")
    compare_grads(dC, oC, "cfg2 full recon upstream dC")
    dVf, dCf, losses = r.backward_recon(verts, colors, rgb, target, mask, saved, ws, sil_weight=0.5)
    if not o_mask.any():
        compare_grads(dVf, oV, "cfg2 full fused recon dV")
    # view-dependent colour, degree 3
    rs, _, _ = gpu_setup(W, sh_degree=3)
    rng = np.random.default_rng(44)
    C = np.zeros((len(W.verts), 16, 3), np.float32)
    C[:, 0] = W.colors
    C[:, 1:] = rng.normal(0, 0.15, size=(len(W.verts), 15, 3))
    c3 = torch.from_numpy(C).cuda()
    rgb, alpha, saved, ws = rs.forward(verts, c3)
    P = oracle.Params(sh_degree=3)
    o_rgb, o_tf, _, o_mask = oracle.render_workload(W, P, colors=C)
    compare_images(rgb, alpha, o_rgb, o_tf, o_mask, label="cfg2 full sh3")
    g = rng.normal(size=(W.num_pixels, 3)) * (~o_mask)[:, None] / W.num_pixels
    dV, dC = rs.backward(verts, c3, torch.from_numpy(g.astype(np.float32)).cuda(), None, saved, ws)
    oV, oC = oracle.adjoint_workload(W, g, None, P, colors=C)
    compare_grads(dV, oV, "cfg2 full sh3 dV")
    compare_grads(dC, oC, "cfg2 full sh3 dC")
