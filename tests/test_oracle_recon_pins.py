"""Pins of the reconstruction-step oracle (silhouette BCE, edge-length and Laplacian regularisers,
VectorAdam) against closed forms, invariances and central differences -- not against its own
formulas.  CPU only."""
import math

import numpy as np
import pytest

from oracle import recon
import workloads as wl


def _fd(fun, x, h=1e-6):
    x = np.asarray(x, np.float64)
    g = np.zeros_like(x)
    it = np.nditer(x, flags=["multi_index"])
    for _ in it:
        i = it.multi_index
        xp = x.copy(); xm = x.copy()
        xp[i] += h; xm[i] -= h
        g[i] = (fun(xp) - fun(xm)) / (2 * h)
    return g


def _tetra(a=1.0):
    v = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], np.float64) * (a / math.sqrt(8.0))
    f = np.array([[0, 1, 2], [0, 3, 1], [0, 2, 3], [1, 3, 2]], np.int32)
    return v, f


def _hex_fan():
    ang = np.arange(6) * np.pi / 3
    ring = np.stack([np.cos(ang), np.sin(ang), np.zeros(6)], axis=1)
    v = np.concatenate([[[0.0, 0.0, 0.0]], ring])
    f = np.array([[0, 1 + i, 1 + (i + 1) % 6] for i in range(6)], np.int32)
    return v, f


# ---- silhouette BCE ---------------------------------------------------------------------------

def test_bce_closed_form_values():
    loss, g = recon.silhouette_bce([0.5, 0.9], [1.0, 0.0])
    assert loss == pytest.approx((math.log(2.0) - math.log(0.1)) / 2, rel=1e-12)
    # d/da -(log a) = -1/a at a = 0.5; d/da -(log(1 - a)) = 1/(1 - a) at a = 0.9; mean over 2
    assert g == pytest.approx([-2.0 / 2, 10.0 / 2], rel=1e-9)


def test_bce_clamp_and_symmetry():
    loss, g = recon.silhouette_bce([0.0, 1.0], [1.0, 0.0])
    assert loss == pytest.approx(-math.log(1e-6), rel=1e-9)      # both pixels hit the clamp
    assert np.all(g == 0.0)
    rng = np.random.default_rng(1)
    a = rng.uniform(0.01, 0.99, 50); s = (rng.random(50) < 0.5).astype(float)
    assert recon.silhouette_bce(a, s)[0] == pytest.approx(recon.silhouette_bce(1 - a, 1 - s)[0], rel=1e-12)


def test_bce_gradient_matches_central_differences():
    rng = np.random.default_rng(2)
    a = rng.uniform(0.02, 0.98, 20); s = (rng.random(20) < 0.5).astype(float)
    _, g = recon.silhouette_bce(a, s, weight=0.7)
    fd = _fd(lambda x: recon.silhouette_bce(x, s, weight=0.7)[0], a)
    assert np.allclose(g, fd, rtol=1e-6, atol=1e-9)


# ---- edges and neighbours -----------------------------------------------------------------------

def test_mesh_edges_and_neighbours():
    v, f = _tetra()
    e = recon.mesh_edges(f)
    assert len(e) == 6 and set(map(tuple, e.tolist())) == {(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)}
    nb = recon.neighbours(4, e)
    assert all(sorted(nb[i].tolist()) == [j for j in range(4) if j != i] for i in range(4))
    vi, fi = wl.icosphere(3)
    assert len(recon.mesh_edges(fi)) == 3 * len(fi) // 2          # closed 2-manifold: E = 3F/2


# ---- edge length --------------------------------------------------------------------------------

def test_edge_length_regular_tetrahedron():
    a = 0.37
    v, f = _tetra(a)
    e = recon.mesh_edges(f)
    loss, g = recon.edge_length(v, e)
    assert loss == pytest.approx(a * a, rel=1e-12)                  # every edge has length a
    loss, g = recon.edge_length(v, e, l0=a)
    assert loss == pytest.approx(0.0, abs=1e-24) and np.allclose(g, 0.0, atol=1e-12)
    # with l0 = 0 the gradient pulls every vertex towards the centroid: dL/dv = (2/E) sum (v - v_j)
    _, g = recon.edge_length(v, e)
    assert np.allclose(g, 2.0 / 6.0 * (3 * v - (v.sum(0) - v)), atol=1e-12)


def test_edge_length_gradient_fd_and_translation():
    rng = np.random.default_rng(3)
    v, f = wl.icosphere(1)
    v = v + rng.normal(0, 0.05, v.shape)
    e = recon.mesh_edges(f)
    _, g = recon.edge_length(v, e, l0=0.3, weight=2.0)
    fd = _fd(lambda x: recon.edge_length(x.reshape(-1, 3), e, l0=0.3, weight=2.0)[0], v)
    assert np.allclose(g, fd, rtol=1e-5, atol=1e-9)
    assert np.allclose(g.sum(0), 0.0, atol=1e-12)


# ---- Laplacian ----------------------------------------------------------------------------------

def test_laplacian_hexagon_fan_closed_form():
    v, f = _hex_fan()
    nb = recon.neighbours(7, recon.mesh_edges(f))
    loss, g = recon.laplacian_smoothing(v, nb)
    # centre: mean of the unit ring = 0; ring vertex: (centre + two neighbours)/3 - r = -2/3 r
    assert loss == pytest.approx(6 * (2.0 / 3.0) / 7, rel=1e-12)


def test_laplacian_gradient_fd_translation_and_scale():
    rng = np.random.default_rng(4)
    v, f = wl.icosphere(1)
    v = v + rng.normal(0, 0.05, v.shape)
    nb = recon.neighbours(len(v), recon.mesh_edges(f))
    loss, g = recon.laplacian_smoothing(v, nb, weight=1.5)
    fd = _fd(lambda x: recon.laplacian_smoothing(x.reshape(-1, 3), nb, weight=1.5)[0], v)
    assert np.allclose(g, fd, rtol=1e-5, atol=1e-9)
    assert np.allclose(g.sum(0), 0.0, atol=1e-12)
    assert recon.laplacian_smoothing(2.5 * v + 7.0, nb, weight=1.5)[0] == pytest.approx(2.5 * loss, rel=1e-12)


# ---- VectorAdam ---------------------------------------------------------------------------------

def test_vector_adam_first_step_closed_form():
    rng = np.random.default_rng(5)
    p = rng.normal(size=(10, 3)); g = rng.normal(size=(10, 3))
    p1, m1, v1 = recon.vector_adam_step(p, g, np.zeros((10, 3)), np.zeros(10), 1, lr=0.01)
    # bias-corrected moments of the first step are g and |g|^2
    assert np.allclose(p1, p - 0.01 * g / (np.linalg.norm(g, axis=1, keepdims=True) + 1e-8), atol=1e-15)


def test_vector_adam_rotation_equivariance():
    rng = np.random.default_rng(6)
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    gs = [rng.normal(size=(8, 3)) for _ in range(5)]
    pa = np.zeros((8, 3)); ma = np.zeros((8, 3)); va = np.zeros(8)
    pb = np.zeros((8, 3)); mb = np.zeros((8, 3)); vb = np.zeros(8)
    for t, g in enumerate(gs, start=1):
        pa, ma, va = recon.vector_adam_step(pa, g, ma, va, t, lr=0.1)
        pb, mb, vb = recon.vector_adam_step(pb, g @ q.T, mb, vb, t, lr=0.1)
    assert np.allclose(pb, pa @ q.T, atol=1e-12)                     # rotated gradients, rotated path


# ---- Adam (the torus workload's optimiser) ------------------------------------------------------

def test_adam_first_step_closed_form():
    """Bias correction makes the first step's moments g and g^2: p moves by lr g / (|g| + eps)."""
    rng = np.random.default_rng(7)
    p = rng.normal(size=(12, 3)); g = rng.normal(size=(12, 3))
    p1, m1, v1 = recon.adam_step(p, g, np.zeros_like(p), np.zeros_like(p), 1, lr=0.01)
    assert np.allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), atol=1e-15)
    assert np.allclose(m1, 0.1 * g, atol=1e-16) and np.allclose(v1, 0.001 * g * g, atol=1e-16)


def test_adam_two_steps_hand_computed():
    """g = 1 then g = -2 from p = 0 with lr 0.1, betas (0.9, 0.999), eps 0.  By hand: m1 = 0.1,
    v1 = 0.001, step 1 moves by -lr (m1 / 0.1) / sqrt(v1 / 0.001) = -0.1; m2 = 0.09 - 0.2 = -0.11,
    v2 = 0.000999 + 0.004 = 0.004999, m2 / (1 - 0.81) = -11/19, v2 / (1 - 0.998001) = 4999/1999, so
    p2 = -0.1 + (11/190) sqrt(1999/4999) = -0.0633896472964154434717... (40-digit decimal)."""
    p, m, v = np.zeros(1), np.zeros(1), np.zeros(1)
    p, m, v = recon.adam_step(p, [1.0], m, v, 1, lr=0.1, eps=0.0)
    assert p[0] == pytest.approx(-0.1, abs=1e-15)
    p, m, v = recon.adam_step(p, [-2.0], m, v, 2, lr=0.1, eps=0.0)
    assert m[0] == pytest.approx(-0.11, abs=1e-15) and v[0] == pytest.approx(0.004999, abs=1e-17)
    assert p[0] == pytest.approx(-0.06338964729641544347, abs=1e-15)


def test_adam_zero_gradient_and_constant_gradient():
    """A coordinate that never receives a gradient never moves (eps > 0 keeps 0 / 0 away); a
    constant gradient moves its coordinate by exactly lr sign(g) on every step when eps = 0, since
    both bias-corrected moments are then exact (m_hat = g, v_hat = g^2 for every t)."""
    g = np.array([0.0, 3.0, -0.25, 1e-3])
    p0 = np.array([0.5, -1.0, 2.0, 0.0])
    p, m, v = p0.copy(), np.zeros(4), np.zeros(4)
    q = p0[1:].copy(); mq, vq = np.zeros(3), np.zeros(3)
    for t in range(1, 8):
        p, m, v = recon.adam_step(p, g, m, v, t, lr=0.05)
        assert p[0] == p0[0] and m[0] == 0.0 and v[0] == 0.0
        q, mq, vq = recon.adam_step(q, g[1:], mq, vq, t, lr=0.05, eps=0.0)
        assert np.allclose(q, p0[1:] - 0.05 * t * np.sign(g[1:]), atol=1e-13)


def test_adam_scale_and_sign_invariance():
    """With eps = 0 the update is invariant to a positive scale of every gradient and odd under a
    sign flip of every gradient; with eps > 0 a scale of 1e6 changes it by a negligible amount."""
    rng = np.random.default_rng(8)
    gs = [rng.normal(size=20) for _ in range(6)]
    runs = {}
    for key, c, eps in (("one", 1.0, 0.0), ("big", 1e6, 0.0), ("neg", -1.0, 0.0), ("eps", 1e6, 1e-8)):
        p, m, v = np.zeros(20), np.zeros(20), np.zeros(20)
        for t, g in enumerate(gs, start=1):
            p, m, v = recon.adam_step(p, c * g, m, v, t, lr=0.02, eps=eps)
        runs[key] = p
    assert np.allclose(runs["big"], runs["one"], rtol=1e-12, atol=1e-15)
    assert np.allclose(runs["neg"], -runs["one"], rtol=1e-12, atol=1e-15)
    assert np.allclose(runs["eps"], runs["one"], rtol=1e-9, atol=1e-12)


def test_adam_equals_vector_adam_on_one_axis():
    """VectorAdam's second moment is |g|^2 per vertex; with gradients on the x axis only, that is
    g_x^2 and the two optimisers take the same steps (a cross-check of two independent forms)."""
    rng = np.random.default_rng(9)
    gs = [np.stack([rng.normal(size=6), np.zeros(6), np.zeros(6)], axis=1) for _ in range(4)]
    pa, ma, va = np.zeros((6, 3)), np.zeros((6, 3)), np.zeros((6, 3))
    pb, mb, vb = np.zeros((6, 3)), np.zeros((6, 3)), np.zeros(6)
    for t, g in enumerate(gs, start=1):
        pa, ma, va = recon.adam_step(pa, g, ma, va, t, lr=0.03)
        pb, mb, vb = recon.vector_adam_step(pb, g, mb, vb, t, lr=0.03)
    assert np.allclose(pa, pb, atol=1e-15)
    assert np.allclose(va[:, 0], vb, atol=1e-18)


def test_adam_rejects_step_zero():
    with pytest.raises(ValueError):
        recon.adam_step(np.zeros(2), np.ones(2), np.zeros(2), np.zeros(2), 0, lr=0.1)
