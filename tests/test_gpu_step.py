"""gmr_render_step_l2 -- the forward and the fused L2 backward from one list build, the compositing
and its adjoint in one launch -- against gmr_render_fwd followed by gmr_render_bwd_l2: the image,
alpha and saved state bit for bit, the loss equal, and the vertex and colour gradients equal up to
the order of the float atomics that sum each face-view's gradient.  Both paths are checked against
the oracle elsewhere (images, the L2 adjoint); this pins the fused one to them."""
import numpy as np
import pytest

import workloads as wl
from gmr_testutil import compare_grads, gpu_setup, saved_equal, to_np

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


CASES = {
    "cfg1": (1, 1.0, {}),
    "cfg2-half": (2, 0.5, {}),
    "cfg2-half-block-uniform": (2, 0.5, {"lane_lists": 0}),
    "cfg2-half-px2": (2, 0.5, {"px_per_lane": 2, "tile_w": 16, "tile_h": 16}),
    "cfg2-half-lists-off": (2, 0.5, {"composited_lists": 0}),
    "cfg2-half-lists-7": (2, 0.5, {"composited_lists": 7}),
    "cfg3-quarter": (3, 0.25, {"tile_w": 16, "tile_h": 16}),
}


def _setup(name):
    import torch
    k, scale, kw = CASES[name]
    W = wl.make_workload(k, scale=scale)
    r, verts, colors = gpu_setup(W, **kw)
    tv = torch.from_numpy(np.ascontiguousarray(W.target_verts, dtype=np.float32)).cuda()
    target, _, _, _ = r.forward(tv, colors, check=True)
    return W, r, verts, colors, target.clone()


@pytest.mark.parametrize("name", list(CASES))
def test_step_l2_matches_fwd_then_bwd_l2(gpu, name):
    import torch
    say(f"fused step vs forward + L2 backward: {name}")
    W, r, verts, colors, target = _setup(name)
    rgb, alpha, saved, ws = r.forward(verts, colors, check=True)
    dV, dC, loss = r.backward_l2(verts, colors, rgb, target, saved, ws, want_loss=True)
    rgb2, alpha2, saved2 = r._alloc_outputs()
    ws2 = r.new_workspace()
    dV2, dC2 = torch.empty_like(dV), torch.empty_like(dC)
    loss2 = torch.zeros((1,), dtype=torch.float32, device="cuda")
    r.step_l2_raw(verts, colors, target, 1.0, rgb2, alpha2, saved2, ws2, dV2, dC2, loss2)
    torch.cuda.synchronize()
    c = r.counters(ws2)
    say(f"  {c.instances} instances, loss {float(loss):.6e} / {float(loss2):.6e}, pairs {c.pairs_fwd} {c.pairs_bwd}")
    assert not c.overflow
    assert torch.equal(rgb2, rgb) and torch.equal(alpha2, alpha) and saved_equal(r, saved2, saved)
    assert abs(float(loss2) - float(loss)) <= 1e-6 * abs(float(loss))
    c_ref = r.counters(ws)
    assert c.pairs_fwd == c_ref.pairs_fwd and c.pairs_bwd == c_ref.pairs_bwd
    compare_grads(dV2, to_np(dV), f"{name} step dV", rel=1e-5)
    compare_grads(dC2, to_np(dC), f"{name} step dC", rel=1e-5)


def test_graph_adam_fused_step_matches_two_call_step(gpu):
    """The captured Adam loop rendered with the fused step against the one rendered with
    gmr_render_fwd + gmr_render_bwd_l2 (lists rebuilt): one replay each from the same state gives
    the same loss and gradients (atomic order aside), and the same update where the gradient is
    not near zero (Adam's first step moves a coordinate by lr times the sign of its gradient)."""
    import torch
    import paper_2602_14493_amd as gmr
    say("captured Adam step, fused vs two calls, cfg1")
    W, r, verts, colors, target = _setup("cfg1")
    loops = [gmr.GraphAdamLoop(r, verts, colors, target, lr=1e-3, recompute=True, fused=f).capture()
             for f in (False, True)]
    for lp in loops:
        lp.graph.replay()
    torch.cuda.synchronize()
    a, b = loops
    assert abs(float(a.loss) - float(b.loss)) <= 1e-6 * abs(float(a.loss))
    compare_grads(b.dV, to_np(a.dV), "graph step dV", rel=1e-5)
    g = to_np(a.dV).reshape(-1)
    big = np.abs(g) > 1e-3 * np.abs(g).max()
    va, vb = to_np(a.verts).reshape(-1), to_np(b.verts).reshape(-1)
    assert np.allclose(vb[big], va[big], rtol=0, atol=1e-6)
    assert int(a.step_count) == int(b.step_count) == 1


@pytest.mark.parametrize("name", ["cfg1", "cfg2-half", "cfg2-half-px2"])
def test_step_recon_matches_fwd_then_bwd_recon(gpu, name):
    """gmr_render_step_recon (colour + silhouette terms of Sec. 3.1) against gmr_render_fwd
    followed by gmr_render_bwd_recon: outputs bit for bit, both losses, gradients up to atomic
    order."""
    import torch
    say(f"fused reconstruction step vs forward + reconstruction backward: {name}")
    W, r, verts, colors, target = _setup(name)
    tv = torch.from_numpy(np.ascontiguousarray(W.target_verts, dtype=np.float32)).cuda()
    _, t_alpha, _, _ = r.forward(tv, colors, check=True)
    mask = (t_alpha > 0.5).to(torch.float32)
    rgb, alpha, saved, ws = r.forward(verts, colors, check=True)
    dV, dC, losses = r.backward_recon(verts, colors, rgb, target, mask, saved, ws, color_weight=1.0, sil_weight=0.1)
    rgb2, alpha2, saved2 = r._alloc_outputs()
    ws2 = r.new_workspace()
    dV2, dC2 = torch.empty_like(dV), torch.empty_like(dC)
    losses2 = torch.zeros((2,), dtype=torch.float32, device="cuda")
    r.step_recon_raw(verts, colors, target, 1.0, mask, 0.1, rgb2, alpha2, saved2, ws2, dV2, dC2, losses2)
    torch.cuda.synchronize()
    assert not r.counters(ws2).overflow
    assert torch.equal(rgb2, rgb) and torch.equal(alpha2, alpha) and saved_equal(r, saved2, saved)
    l1, l2 = to_np(losses).astype(np.float64), to_np(losses2).astype(np.float64)
    say(f"  losses {l1} / {l2}")
    assert np.all(np.abs(l2 - l1) <= 1e-6 * np.abs(l1))
    compare_grads(dV2, to_np(dV), f"{name} recon step dV", rel=1e-5)
    compare_grads(dC2, to_np(dC), f"{name} recon step dC", rel=1e-5)
