"""Parity of the configuration's optimiser step with the FP64 oracle, through the C ABI: the plain
Adam kernel alone (several steps, a resumed step counter, a ragged length), and the captured
optimisation step (forward, fused L2 backward with the lists rebuilt, Adam) checked step by step
against the oracle's render -> L2 adjoint -> Adam chain.

Tolerances: parameters 1e-6 absolute and moments 1e-5 relative plus 1e-6 of the largest moment
(the first moment's update can cancel) when both sides take the same gradient (the kernel works in float32 with float32 hyper-parameters, which the oracle is given);
the renderer's gradients as its own parity tests (||d||/||g|| <= 1e-3, per element
1e-3 |g| + 1e-5 max|g|); an update computed from the oracle's gradient may differ from the kernel's
by what Adam makes of that per-element gradient tolerance (the spread of the oracle's own update
over the tolerance interval), plus float32 rounding of the parameter."""
import numpy as np
import pytest

import oracle
import workloads as wl
from gmr_testutil import GRAD_REL, compare_grads, flagged_pixels_agree, gpu_setup, to_np
from oracle import recon

pytestmark = pytest.mark.gpu

F32 = np.float32


def say(*a):
    print(*a, flush=True)


def _hyper(lr, b1=0.9, b2=0.999, eps=1e-8):
    """The hyper-parameters as the kernel receives them (rounded to float32), for the oracle."""
    return dict(lr=float(F32(lr)), b1=float(F32(b1)), b2=float(F32(b2)), eps=float(F32(eps)))


@pytest.mark.parametrize("n,step0", [(3001, 0), (1, 0), (777, 7)])
def test_adam_kernel_vs_oracle(gpu, n, step0):
    """gmr_adam_step over five steps against the oracle's Adam (Kingma & Ba with bias correction):
    parameters, both moments and the device step counter.  step0 > 0 resumes a run, so the bias
    correction must use the counter's value, not the number of calls."""
    import torch
    say(f"adam kernel n={n} step0={step0}")
    rng = np.random.default_rng(100 + n)
    p = rng.normal(size=n).astype(F32)
    m0 = (0.1 * rng.normal(size=n)).astype(F32) if step0 else np.zeros(n, F32)
    v0 = (0.01 * rng.random(n)).astype(F32) if step0 else np.zeros(n, F32)
    gs = [rng.normal(size=n).astype(F32) * F32(10.0 ** rng.uniform(-3, 1)) for _ in range(5)]
    for g in gs:
        g[n // 2] = 0.0                       # a coordinate that never receives a gradient
    pt = torch.from_numpy(p.copy()).cuda()
    mt = torch.from_numpy(m0.copy()).cuda()
    vt = torch.from_numpy(v0.copy()).cuda()
    step = torch.full((1,), step0, dtype=torch.int32, device="cuda")
    hp = _hyper(1e-2)
    po, mo, vo = p.astype(np.float64), m0.astype(np.float64), v0.astype(np.float64)
    for k, g in enumerate(gs):
        gpu.adam_step(pt, torch.from_numpy(g).cuda(), mt, vt, step, lr=1e-2)
        po, mo, vo = recon.adam_step(po, g.astype(np.float64), mo, vo, step0 + k + 1, **hp)
        torch.cuda.synchronize()
        ep = np.abs(to_np(pt).astype(np.float64) - po).max()
        say(f"  step {step0 + k + 1}: max |dp| = {ep:.3e}")
        assert ep <= 1e-6
        # m = b1 m + (1 - b1) g can cancel: its float32 rounding is relative to the terms, so the
        # absolute part of the bound scales with the largest moment
        np.testing.assert_allclose(to_np(mt), mo, rtol=1e-5, atol=1e-6 * np.abs(mo).max())
        np.testing.assert_allclose(to_np(vt), vo, rtol=1e-5, atol=1e-6 * np.abs(vo).max())
    assert int(step.item()) == step0 + 5
    if not step0:
        assert to_np(pt)[n // 2] == p[n // 2]


def test_adam_kernel_empty_and_invalid(gpu):
    """n = 0 launches nothing and still advances the counter; bad hyper-parameters are refused on
    the host before anything is enqueued."""
    import torch
    from paper_2602_14493_amd._lib import GMRError
    p = torch.ones(4, device="cuda")
    z = torch.zeros(4, device="cuda")
    step = torch.zeros((1,), dtype=torch.int32, device="cuda")
    gpu._lib.call("gmr_adam_step", p.data_ptr(), z.data_ptr(), z.data_ptr(), z.data_ptr(), 0, 1e-3, 0.9, 0.999,
                  1e-8, step.data_ptr(), None)
    torch.cuda.synchronize()
    assert int(step.item()) == 1 and bool((p == 1).all())
    for bad in (dict(beta1=1.0), dict(beta2=-0.1), dict(eps=0.0), dict(lr=float("nan"))):
        with pytest.raises(GMRError):
            gpu.adam_step(p, z, z, z, step, **bad)
    torch.cuda.synchronize()
    assert int(step.item()) == 1


def _adam_update_tolerance(p, g, m, v, t, hp):
    """How far Adam's new parameters can move when each gradient element moves within the
    renderer's gradient tolerance: the larger deviation of the update at g -/+ that bound."""
    bound = np.where(g == 0.0, 0.0, GRAD_REL * np.abs(g) + 1e-5 * np.abs(g).max())
    base, _, _ = recon.adam_step(p, g, m, v, t, **hp)
    lo, _, _ = recon.adam_step(p, g - bound, m, v, t, **hp)
    hi, _, _ = recon.adam_step(p, g + bound, m, v, t, **hp)
    return base, np.maximum(np.abs(lo - base), np.abs(hi - base))


@pytest.mark.parametrize("recompute", [True, False])
def test_graph_adam_steps_vs_oracle_chain(gpu, recompute):
    """Icosphere subdiv 2 at 128^2: three replays of the captured step.  Before each replay the GPU
    state (vertices, moments) is read; the oracle renders those vertices, takes the L2 loss against
    the target and its adjoint, and applies Adam.  Checked per step: the loss, the renderer's vertex
    gradient (the graph's own dV buffer), the update given the GPU's gradient (tight) and the update
    given the oracle's gradient (within what the gradient tolerance allows)."""
    import torch
    say(f"graph adam vs oracle chain, cfg1, recompute={recompute}")
    W = wl.make_workload(1)
    r, verts, colors = gpu_setup(W)
    tgt_rgb, _, _, _ = oracle.render_workload(W, verts=W.target_verts)
    target = torch.from_numpy(tgt_rgb.astype(F32)).cuda()
    lr = 1e-3
    hp = _hyper(lr)
    loop = gpu.GraphAdamLoop(r, verts, colors, target, lr=lr, recompute=recompute)
    loop.capture()
    # capture() leaves the state as it found it
    assert torch.equal(loop.verts, verts) and int(loop.step_count.item()) == 0
    assert float(loop.m.abs().max()) == 0.0 and float(loop.v.abs().max()) == 0.0
    loose_total, compared = 0, 0
    for t in range(1, 4):
        p0 = to_np(loop.verts).astype(np.float64)
        m0 = to_np(loop.m).astype(np.float64)
        v0 = to_np(loop.v).astype(np.float64)
        loop.graph.replay()
        torch.cuda.synchronize()
        assert int(loop.step_count.item()) == t
        assert not loop.overflow()
        dV = to_np(loop.dV).astype(np.float64)
        # the fused backward against the explicit one fed the GPU's own image (tight)
        g_gpu = 2.0 * (loop.rgb - target) / loop.rgb.numel()
        dVx, _ = r.backward(loop.verts.new_tensor(p0.astype(F32)), colors, g_gpu, None, loop.saved, loop.ws,
                            recompute=True)
        compare_grads(dV, to_np(dVx), f"step {t} fused vs explicit dV", rel=1e-5)
        # the update from the GPU's own gradient: the Adam kernel alone
        pg, mg, vg = recon.adam_step(p0, dV, m0, v0, t, **hp)
        p1 = to_np(loop.verts).astype(np.float64)
        e = np.abs(p1 - pg).max()
        say(f"  step {t}: |p - adam(p0, dV_gpu)| max {e:.3e}")
        assert e <= 1e-6
        np.testing.assert_allclose(to_np(loop.m), mg, rtol=1e-5, atol=1e-6 * np.abs(mg).max())
        np.testing.assert_allclose(to_np(loop.v), vg, rtol=1e-5, atol=1e-6 * np.abs(vg).max())
        # oracle at the vertices the GPU step started from
        o_rgb, o_tf, _, o_mask = oracle.render_workload(W, verts=p0.astype(F32))
        L, g_img = oracle.l2_loss(o_rgb, tgt_rgb)
        say(f"  step {t}: loss gpu {loop.loss.item():.8e} oracle {L:.8e}, flagged px {int(o_mask.sum())}")
        assert abs(float(loop.loss.item()) - L) <= 1e-5 * L
        # a pixel near a decision threshold counts only where both sides took the same decisions
        # (checked on its image value); else this step's gradient is checked through the explicit
        # backward above and the oracle comparison of the update is skipped
        if not flagged_pixels_agree(loop.rgb, loop.alpha, o_rgb, o_tf, o_mask):
            say(f"  step {t}: flagged pixels disagree, oracle gradient comparison skipped")
            continue
        compared += 1
        oV, _ = oracle.adjoint_workload(W, g_img, verts=p0.astype(F32))
        compare_grads(dV, oV, f"step {t} dV")
        # a coordinate no composited pixel depends on has an exactly zero gradient on both sides
        assert np.array_equal(dV == 0.0, oV == 0.0)
        # the update from the oracle's gradient
        po, tol = _adam_update_tolerance(p0, oV, m0, v0, t, hp)
        d = np.abs(p1 - po)
        ok = d <= tol + 1e-6
        loose = tol > 0.1 * lr
        loose_total += int(loose.sum())
        say(f"  step {t}: |p - adam(p0, dV_oracle)| max {d.max():.3e}; {int(loose.sum())} of {d.size} "
            f"coordinates whose gradient is within its tolerance of zero")
        assert ok.all(), np.argwhere(~ok)[:5]
    # the comparison pins the update: only a few coordinates sit where the sign of their gradient
    # is not decided by the tolerance (visible vertices whose gradient is ~0; about 2 % here)
    assert compared >= 2, "the oracle comparison ran on fewer than two of the three steps"
    assert loose_total <= 0.05 * 3 * W.verts.size
