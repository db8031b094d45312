"""The forward entry point that allocates nothing (gmr_render_fwd_noalloc): its workspace is the
library's static device array.  Checked through the C ABI against gmr_render_fwd, which runs the
same kernels in a caller workspace: images, alpha and the saved per-pixel state must be
bit-identical and the instance count it reports equal, on two calls in a row, the second with a
smaller input; a batch whose workspace exceeds the static array is refused before anything is
enqueued, and the next call still works."""
import ctypes

import numpy as np
import pytest

import workloads as wl
from gmr_testutil import gpu_setup, saved_equal

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def _noalloc(r, verts, colors, counters=None):
    import torch
    from paper_2602_14493_amd import _lib
    from paper_2602_14493_amd.render import _ptr, _stream
    P = r.batch.num_pixels
    # outputs prefilled with values no call writes, so a pixel left unwritten shows
    rgb = torch.full((P, 3), float("nan"), dtype=torch.float32, device=r.device)
    alpha = torch.full((P,), float("nan"), dtype=torch.float32, device=r.device)
    saved = torch.full((r.sizes()[1],), 0xAB, dtype=torch.uint8, device=r.device)
    _lib.call("gmr_render_fwd_noalloc", r.handle.ptr, ctypes.byref(r.batch.c), ctypes.byref(r.opts), _ptr(r.table),
              _ptr(verts), _ptr(r.faces), _ptr(colors), _ptr(rgb), _ptr(alpha), _ptr(saved), _ptr(counters),
              _stream(r.device))
    return rgb, alpha, saved


def test_noalloc_forward_matches_workspace_forward(gpu):
    import torch
    from paper_2602_14493_amd import _lib
    # the 8-view icosphere at 256^2, then the single-view icosphere at 64^2 (the smaller input)
    for k, scale in ((2, 0.5), (1, 0.5)):
        W = wl.make_workload(k, scale=scale)
        r, verts, colors = gpu_setup(W)
        ref_rgb, ref_alpha, ref_saved, ws = r.forward(verts, colors, check=True)
        c_ref = r.counters(ws)
        need = r.sizes()[0]
        assert need <= _lib.NOALLOC_WORKSPACE_BYTES and not c_ref.overflow
        cnt = torch.full((2,), 7, dtype=torch.int32, device="cuda")
        rgb, alpha, saved = _noalloc(r, verts, colors, cnt)
        torch.cuda.synchronize()
        say(f"cfg{k} scale {scale}: {W.num_pixels} px, workspace {need} B, {c_ref.instances} instances, "
            f"no-alloc counters {cnt.tolist()}")
        assert torch.equal(rgb, ref_rgb) and torch.equal(alpha, ref_alpha) and saved_equal(r, saved, ref_saved)
        assert int(cnt[0]) == c_ref.instances and int(cnt[1]) == 0
        # the saved state drives the backward like the caller-workspace forward's (lists rebuilt)
        g = torch.randn_like(rgb)
        dV1, dC1 = r.backward(verts, colors, g, None, ref_saved, r.new_workspace(), recompute=True)
        dV2, dC2 = r.backward(verts, colors, g, None, saved, r.new_workspace(), recompute=True)
        assert float((dV1 - dV2).abs().max()) <= 1e-6 * float(dV1.abs().max())
        assert float((dC1 - dC2).abs().max()) <= 1e-6 * float(dC1.abs().max())


def test_noalloc_forward_refuses_oversized_workspace(gpu):
    import torch
    import paper_2602_14493_amd as gmr
    from paper_2602_14493_amd import _lib
    W = wl.make_workload(1)
    r, verts, colors = gpu_setup(W)
    r.forward(verts, colors, check=True)
    ok_opts = gmr.copy_options(r.opts)
    r.opts.instance_capacity = 1 << 24                # 16M instances: far beyond the static array
    assert r.sizes()[0] > _lib.NOALLOC_WORKSPACE_BYTES
    with pytest.raises(gmr.GMRError) as e:
        _noalloc(r, verts, colors)
    assert e.value.status == _lib.GMR_ERR_WORKSPACE
    say(f"refused: {e.value}")
    r.opts = ok_opts                                    # a fitting call afterwards still works
    ref_rgb, _, _, _ = r.forward(verts, colors, check=False)
    rgb, _, _ = _noalloc(r, verts, colors)
    torch.cuda.synchronize()
    assert torch.equal(rgb, ref_rgb)
