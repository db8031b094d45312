"""Pins of the FP64 oracle against facts the paper and the mathematics fix, independent of the
oracle's own code (CPU only).

Conversion (Sec. 2.2): hand-derived worked examples (tests/golden), brute-force integration of the
uniform triangle, Monte Carlo, numpy eigh, the covariance identity, PSD (after Eq. 9), the
area-matching invariant (Eq. 12), Eq. 14's frame relation, permutation and rigid-motion
invariance, the epsilon clamp, degenerate faces.
Projection + compositing (Sec. 2.1's 3DGS rasteriser as read in the design notes): a single
triangle facing the camera (closed form), two-triangle occlusion including the stop at the
double-opaque core, face-reordering invariance, partition of unity, linearity in colours, rigid
motion of camera and mesh together, tile lists vs per-pixel brute force.
Adjoint: FP64 central differences on tiny meshes (both covariance forms, the clamped branch), and
exact colour gradients by linearity.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads as wl

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "conversion_examples.json")))
f32 = np.float32
KAPPA0 = 6.0 * math.sqrt(3.0) / math.pi


def rand_tris(rng, n, scale=1.0):
    return rng.normal(0, scale, size=(n, 3, 3))


# ------------------------------------------------------------------------------------------------
# conversion
# ------------------------------------------------------------------------------------------------

def test_right_triangle_worked_example():
    g = GOLD["right_triangle"]
    s = oracle.face_steps(*np.array(g["vertices"], float))
    for k in ["xj", "xk", "yk", "mux", "muy", "Exx", "Exy", "Eyy", "l1", "l2", "area", "kappa"]:
        assert s[k] == pytest.approx(g[k], rel=1e-14, abs=1e-15), k
    np.testing.assert_allclose(s["S2"], g["S2"], rtol=1e-14)
    np.testing.assert_allclose(np.abs(s["u1"]), g["u1_abs"], rtol=1e-14)
    assert s["u1"][0] * s["u1"][1] < 0  # principal direction (1,-1)/sqrt2


def test_equilateral_isotropic():
    g = GOLD["equilateral"]
    a = g["side"]
    v = np.array([[0, 0, 0], [a, 0, 0], [a / 2, a * math.sqrt(3) / 2, 0]], float)
    s = oracle.face_steps(*v)
    np.testing.assert_allclose(s["S2"], g["S2"], atol=1e-15)
    assert s["area"] == pytest.approx(g["area"], rel=1e-14)
    assert s["kappa"] == pytest.approx(g["kappa"], rel=1e-14)
    assert s["l1"] == pytest.approx(s["l2"], rel=1e-13)


def test_clamped_kappa():
    g = GOLD["clamped_small_triangle"]
    s = oracle.face_steps(*np.array(g["vertices"], float))
    assert s["area"] == pytest.approx(g["area"], rel=1e-12)
    assert s["l1"] * s["l2"] < 1e-14
    assert s["kappa"] == pytest.approx(g["kappa"], rel=1e-12)


def brute_force_moments(p, n=600):
    """Second moments of the uniform triangle p[3][2] by midpoint quadrature over an n x n
    subdivision of the barycentric square folded onto the triangle (independent of Eq. 6-8)."""
    t = (np.arange(n) + 0.5) / n
    a, b = np.meshgrid(t, t, indexing="ij")
    a, b = a.ravel(), b.ravel()
    keep = a + b <= 1.0
    # exact quadrature weights on the boundary cells are not needed: the midpoint rule's error is
    # O(1/n), tolerance is set accordingly
    a, b = a[keep], b[keep]
    x = p[0, 0] + a * (p[1, 0] - p[0, 0]) + b * (p[2, 0] - p[0, 0])
    y = p[0, 1] + a * (p[1, 1] - p[0, 1]) + b * (p[2, 1] - p[0, 1])
    return np.mean(x * x), np.mean(x * y), np.mean(y * y), np.mean(x), np.mean(y)


def test_moments_vs_quadrature_and_monte_carlo():
    rng = np.random.default_rng(11)
    for _ in range(5):
        v = rand_tris(rng, 1)[0]
        s = oracle.face_steps(*v)
        p2 = np.array([[0, 0], [s["xj"], 0], [s["xk"], s["yk"]]])
        exx, exy, eyy, mx, my = brute_force_moments(p2)
        scale = max(s["xj"], abs(s["xk"]), s["yk"]) ** 2
        assert abs(s["Exx"] - exx) < 5e-3 * scale
        assert abs(s["Exy"] - exy) < 5e-3 * scale
        assert abs(s["Eyy"] - eyy) < 5e-3 * scale
        # Monte Carlo over the 3D triangle: the covariance must equal R_f blockdiag(S2, 0) R_f^T
        u = rng.uniform(size=(400000, 2))
        flip = u.sum(1) > 1
        u[flip] = 1 - u[flip]
        pts = v[0] + u[:, :1] * (v[1] - v[0]) + u[:, 1:] * (v[2] - v[0])
        cov = np.cov(pts.T, bias=True)
        E = np.stack([s["x_axis"], s["y_axis"]], 1)
        S2 = np.array([[s["S2"][0], s["S2"][1]], [s["S2"][1], s["S2"][2]]])
        assert np.abs(cov - E @ S2 @ E.T).max() < 1e-2 * np.abs(cov).max()
        np.testing.assert_allclose(pts.mean(0), s["mu"], atol=5e-3 * np.abs(v).max())


def test_covariance_identity_and_eigh():
    """Sigma2D embedded in 3D equals (1/12) sum (q - mu)(q - mu)^T; eigenvalues match numpy."""
    rng = np.random.default_rng(12)
    for v in rand_tris(rng, 50):
        s = oracle.face_steps(*v)
        m = v.mean(0)
        ident = sum(np.outer(q - m, q - m) for q in v) / 12.0
        E = np.stack([s["x_axis"], s["y_axis"]], 1)
        S2 = np.array([[s["S2"][0], s["S2"][1]], [s["S2"][1], s["S2"][2]]])
        np.testing.assert_allclose(E @ S2 @ E.T, ident, rtol=1e-12, atol=1e-14 * np.abs(ident).max())
        w = np.linalg.eigh(S2)[0]
        assert s["l1"] == pytest.approx(w[1], rel=1e-12)
        assert s["l2"] == pytest.approx(w[0], rel=1e-10, abs=1e-15 * w[1])
        np.testing.assert_allclose(s["mu"], m, atol=1e-14 * np.abs(v).max())


def test_psd_area_match_and_kappa():
    """PSD for non-collinear vertices (after Eq. 9); det = |A|^2/108; the 1-sigma ellipse area of
    kappa*Sigma2D equals |A| (Eq. 12's design rule)."""
    rng = np.random.default_rng(13)
    for v in rand_tris(rng, 200, scale=rng.uniform(0.1, 3.0)):
        s = oracle.face_steps(*v)
        assert s["l2"] > 0
        area = 0.5 * np.linalg.norm(np.cross(v[1] - v[0], v[2] - v[0]))
        assert s["area"] == pytest.approx(area, rel=1e-12)
        assert s["l1"] * s["l2"] == pytest.approx(area * area / 108.0, rel=1e-10)
        assert s["kappa"] == pytest.approx(KAPPA0, rel=1e-10)
        assert math.pi * math.sqrt(s["kappa"] ** 2 * s["l1"] * s["l2"]) == pytest.approx(area, rel=1e-10)
        w = np.linalg.eigvalsh(s["S"])
        assert w[0] > -1e-12 * w[2]
        # Eq. 13: eigenvalues of Sigma3D are kappa*l1, kappa*l2, s_z^2 with n_f for s_z^2
        np.testing.assert_allclose(sorted(w), sorted([s["kappa"] * s["l1"], s["kappa"] * s["l2"], 1e-12]),
                                   rtol=1e-9, atol=1e-13 * w[2])
        np.testing.assert_allclose(s["S"] @ s["n_f"], 1e-12 * s["n_f"], atol=1e-12 * w[2])


def test_eq14_frame_relation():
    """R_local = R_f blockdiag(U, 1) and both are orthonormal (Eq. 14)."""
    rng = np.random.default_rng(14)
    for v in rand_tris(rng, 30):
        s = oracle.face_steps(*v)
        Rf = np.stack([s["x_axis"], s["y_axis"], s["n_f"]], 1)
        U = np.stack([s["u1"], s["u2"]], 1)
        B = np.eye(3); B[:2, :2] = U
        Rl = np.stack([s["xp"], s["yp"], s["n_f"]], 1)
        np.testing.assert_allclose(Rl, Rf @ B, atol=1e-14)
        np.testing.assert_allclose(Rf.T @ Rf, np.eye(3), atol=1e-14)
        np.testing.assert_allclose(Rl.T @ Rl, np.eye(3), atol=1e-14)
        # n_f is the facet normal
        n = np.cross(v[1] - v[0], v[2] - v[0]); n /= np.linalg.norm(n)
        np.testing.assert_allclose(s["n_f"], n, atol=1e-13)


def test_literal_equals_closed_form_both_modes():
    """Eq. 13 computed through the eigen route equals kappa/12 sum qq^T + s_z^2 nn^T, and Eq. 15
    equals (1/12) sum qq^T, to 1e-12 relative (float32 inputs)."""
    rng = np.random.default_rng(15)
    V = rng.normal(size=(300, 3)).astype(f32)
    Fc = rng.integers(0, 300, size=(400, 3)).astype(np.int32)
    Fc = Fc[(Fc[:, 0] != Fc[:, 1]) & (Fc[:, 1] != Fc[:, 2]) & (Fc[:, 0] != Fc[:, 2])]
    C = rng.uniform(size=(300, 3)).astype(f32)
    for mode in (0, 1, 2):
        mu, S, col, ok = oracle.convert(V, Fc, C, mode)
        mu2, S2, ok2 = oracle.convert_closed(V, Fc, mode)
        assert ok.all() and ok2.all()
        np.testing.assert_allclose(mu, mu2, rtol=1e-13, atol=1e-15)
        scale = np.abs(S).reshape(len(S), -1).max(1)[:, None, None]
        assert np.abs(S - S2).max() <= 1e-12 * scale.max()
        assert (np.abs(S - S2) <= 1e-12 * scale).all()
        # Eq. 16 colours
        np.testing.assert_allclose(col, C.astype(float)[Fc].mean(1), rtol=1e-15)
        if mode == 1:
            # Eq. 15: strictly planar, kappa not applied
            m = V.astype(float)[Fc].mean(1)
            q = V.astype(float)[Fc] - m[:, None, :]
            np.testing.assert_allclose(S, np.einsum("fki,fkj->fij", q, q) / 12.0, rtol=1e-12, atol=1e-15)


# ---- the "3DGS-based" baseline conversion (Sec. 3.1, Baselines): frame from the normal and the
# ---- first edge; scales read as the area-matched variances along those axes ------------------

def test_baseline_right_triangle_worked_example():
    """Right triangle in the xy plane, first edge along x: the frame is the world frame, so the
    baseline keeps the diagonal of kappa Sigma2D (hand-derived values) and drops its -1/36."""
    g = GOLD["right_triangle"]
    s = oracle.face_steps(*np.array(g["vertices"], float), cov_mode=2)
    k = g["kappa"]
    want = np.diag([k * g["S2"][0], k * g["S2"][2], 1e-12])
    np.testing.assert_allclose(s["S"], want, rtol=1e-13, atol=1e-16)
    s0 = oracle.face_steps(*np.array(g["vertices"], float), cov_mode=0)
    assert s0["S"][0, 1] == pytest.approx(k * g["S2"][1], rel=1e-13)      # what the baseline drops


def test_baseline_equals_eq13_when_first_edge_is_principal():
    """Isosceles triangle with its base as the first edge: by symmetry the base direction is a
    principal axis of the triangle's covariance, so the edge frame is Eq. 14's frame."""
    rng = np.random.default_rng(30)
    for h in (0.3, 0.7, 2.5):
        v = np.array([[-1.0, 0, 0], [1.0, 0, 0], [0, h, 0]])
        q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        v = v @ q.T + rng.normal(size=3)
        s0, s2 = oracle.face_steps(*v, cov_mode=0), oracle.face_steps(*v, cov_mode=2)
        np.testing.assert_allclose(s2["S"], s0["S"], atol=1e-13 * np.abs(s0["S"]).max())


def test_baseline_frame_and_invariants():
    """For any triangle: the first edge and the normal are eigenvectors of the baseline's
    covariance; its variance along the first edge and its in-plane trace are those of Eq. 13; it
    moves rigidly with the triangle; unlike Eq. 13 it depends on which edge comes first."""
    rng = np.random.default_rng(31)
    changed = 0
    for v in rand_tris(rng, 20):
        s0, s2 = oracle.face_steps(*v, cov_mode=0), oracle.face_steps(*v, cov_mode=2)
        S0, S2 = s0["S"], s2["S"]
        tol = 1e-12 * np.abs(S0).max()
        x = (v[1] - v[0]) / np.linalg.norm(v[1] - v[0])
        n = np.cross(v[1] - v[0], v[2] - v[0]); n /= np.linalg.norm(n)
        y = np.cross(n, x)
        np.testing.assert_allclose(S2 @ x, (x @ S2 @ x) * x, atol=tol)
        np.testing.assert_allclose(S2 @ n, 1e-12 * n, atol=tol)
        assert x @ S2 @ x == pytest.approx(x @ S0 @ x, abs=tol)
        assert np.trace(S2) == pytest.approx(np.trace(S0), abs=tol)
        assert abs(x @ S2 @ y) <= tol
        Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        t = rng.normal(size=3)
        sr = oracle.face_steps(*(v @ Q.T + t), cov_mode=2)
        np.testing.assert_allclose(sr["S"], Q @ S2 @ Q.T, atol=1e-13 * np.abs(S2).max())
        sc = oracle.face_steps(*v[[1, 2, 0]], cov_mode=2)
        changed += np.abs(sc["S"] - S2).max() > 1e-6 * np.abs(S2).max()
    assert changed >= 18


def test_permutation_and_rigid_invariance():
    rng = np.random.default_rng(16)
    import itertools
    for v in rand_tris(rng, 10):
        s0 = oracle.face_steps(*v)
        for perm in itertools.permutations(range(3)):
            s = oracle.face_steps(*v[list(perm)])
            np.testing.assert_allclose(s["S"], s0["S"], atol=1e-13 * np.abs(s0["S"]).max())
            np.testing.assert_allclose(s["mu"], s0["mu"], atol=1e-14)
        q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        t = rng.normal(size=3)
        s = oracle.face_steps(*(v @ q.T + t))
        np.testing.assert_allclose(s["S"], q @ s0["S"] @ q.T, atol=1e-13 * np.abs(s0["S"]).max())
        np.testing.assert_allclose(s["mu"], q @ s0["mu"] + t, atol=1e-13)


def test_degenerate_faces_culled():
    assert oracle.face_steps([0, 0, 0], [1, 1, 1], [2, 2, 2]) is None
    assert oracle.face_steps([0, 0, 0], [0, 0, 0], [1, 0, 0]) is None
    V = np.array([[0, 0, 0], [1, 0, 0], [2, 0, 0], [0, 1, 0]], f32)
    Fc = np.array([[0, 1, 2], [0, 1, 3], [0, 0, 3]], np.int32)
    _, _, _, ok = oracle.convert(V, Fc, np.ones((4, 3), f32))
    assert ok.tolist() == [False, True, False]


# ------------------------------------------------------------------------------------------------
# projection + compositing
# ------------------------------------------------------------------------------------------------

def frontal_camera(W=96, H=96, f=120.0, z=3.0):
    c = wl.look_at_camera((0.0, 0.0, z), width=W, height=H)
    arr = c.as_array()
    arr[12] = arr[13] = f
    return arr


def equilateral(side, z=0.0, center=(0.0, 0.0)):
    R = side / math.sqrt(3.0)
    ang = np.radians([90.0, 210.0, 330.0])
    return np.stack([center[0] + R * np.cos(ang), center[1] + R * np.sin(ang), np.full(3, z)], 1)


def test_single_triangle_closed_form():
    """A camera-facing equilateral triangle on the optical axis: Sigma' = (f/z)^2 kappa a^2/24 I +
    0.3 I, so rgb(p) = c * min(0.99, exp(-r^2 / (2 s'^2))) inside the 3-sigma box when alpha >=
    1/255, else background."""
    side, f, z = 0.4, 120.0, 3.0
    cam = frontal_camera(f=f, z=z)
    v = equilateral(side).astype(f32)
    col = np.array([[0.2, 0.5, 0.9]] * 3, f32)
    P = oracle.Params()
    rgb, Tf, nc, mask = oracle.render_view(v, np.array([[0, 1, 2]], np.int32), col, cam, P)
    vv = v.astype(float)
    a = np.linalg.norm(vv[1] - vv[0])
    s2 = (f / z) ** 2 * KAPPA0 * a * a / 24.0 + P.dilation
    cx = cy = 48.0
    mu = vv.mean(0)
    u = f * mu[0] / (z - 0.0) * 1.0 + cx   # camera looks down -z: x maps to +x
    v_ = f * (-mu[1]) / z + cy              # world +y maps to image -y
    r = 3.0 * math.sqrt(s2)
    ii, jj = np.meshgrid(np.arange(96) + 0.5, np.arange(96) + 0.5, indexing="xy")
    dx, dy = u - ii, v_ - jj
    alpha = np.minimum(P.alpha_max, np.exp(-(dx * dx + dy * dy) / (2 * s2)))
    inside = (np.abs(dx) <= r) & (np.abs(dy) <= r) & (alpha >= P.alpha_min)
    expect = np.where(inside[..., None], alpha[..., None] * col[0].astype(float), 0.0)
    assert not mask.any()
    # float32 vertices make the triangle equilateral only to ~1e-7 relative
    np.testing.assert_allclose(rgb, expect, rtol=2e-6, atol=1e-9)
    np.testing.assert_allclose(1 - Tf, np.where(inside, alpha, 0.0), rtol=2e-6, atol=1e-9)
    assert nc.max() == 1


def test_two_triangle_occlusion_and_double_core_stop():
    """Front triangle at z=0.5 (closer), back one at z=0: rgb = a1 c1 + (1-a1) a2 c2 while
    T stays above the stop; at the shared centre both alphas clamp at 0.99 and
    T(1-a2) = (1-0.99)^2 falls below 1e-4 in float32 constants, so the back one is not composited
    and rgb = 0.99 c1."""
    f, z = 120.0, 3.0
    cam = frontal_camera(f=f, z=z)
    front = equilateral(0.5, z=0.5)
    back = equilateral(0.5, z=0.0)
    v = np.concatenate([back, front]).astype(f32)
    Fc = np.array([[0, 1, 2], [3, 4, 5]], np.int32)
    c_back, c_front = np.array([0.1, 0.8, 0.3]), np.array([0.9, 0.2, 0.6])
    col = np.array([c_back] * 3 + [c_front] * 3, f32)
    P = oracle.Params()
    rgb, Tf, nc, mask = oracle.render_view(v, Fc, col, cam, P)
    vv = v.astype(float)
    a = np.linalg.norm(vv[1] - vv[0])
    s_in = KAPPA0 * a * a / 24.0
    s_front = (f / (z - 0.5)) ** 2 * s_in + P.dilation
    s_back = (f / z) ** 2 * s_in + P.dilation
    ii, jj = np.meshgrid(np.arange(96) + 0.5, np.arange(96) + 0.5, indexing="xy")
    m_back, m_front = vv[:3].mean(0), vv[3:].mean(0)
    ub, vb = f * m_back[0] / z + 48, -f * m_back[1] / z + 48
    uf, vf = f * m_front[0] / (z - 0.5) + 48, -f * m_front[1] / (z - 0.5) + 48

    def alpha_of(u, v_, s2):
        dx, dy = u - ii, v_ - jj
        a_ = np.minimum(P.alpha_max, np.exp(-(dx * dx + dy * dy) / (2 * s2)))
        ins = (np.abs(dx) <= 3 * math.sqrt(s2)) & (np.abs(dy) <= 3 * math.sqrt(s2)) & (a_ >= P.alpha_min)
        return np.where(ins, a_, 0.0)

    a1 = alpha_of(uf, vf, s_front)
    a2 = alpha_of(ub, vb, s_back)
    stop = (1 - a1) * (1 - a2) < P.t_eps
    expect = a1[..., None] * c_front + np.where(stop, 0.0, (1 - a1) * a2)[..., None] * c_back
    ok = ~mask
    np.testing.assert_allclose(rgb.astype(float)[ok], expect.astype(np.float64)[ok] * 1.0, atol=2e-7)
    # the centre pixel region: both clamped -> stop, the back colour is absent
    both = (a1 == P.alpha_max) & (a2 == P.alpha_max)
    assert both.any() and stop[both].all()
    np.testing.assert_allclose(rgb[both & ok], np.broadcast_to(P.alpha_max * c_front, rgb[both & ok].shape), atol=3e-7)
    # the documented float32-constant decision: (1 - fl32(0.99))^2 < fl32(1e-4)
    assert (1 - P.alpha_max) ** 2 < P.t_eps


def test_projection_mean_geometry():
    """Pinhole geometry: the look-at target lands on the principal point; a world offset x along
    the camera's right axis at depth z lands fx*x/z pixels right of it (OpenCV axes: +y down)."""
    cam = wl.look_at_camera((0.0, 0.0, 3.0), width=100, height=80)
    arr = cam.as_array()
    S = np.eye(3) * 1e-4
    p = oracle.project_one([0, 0, 0], S, arr)
    assert (p["u"], p["v"], p["depth"]) == pytest.approx((50.0, 40.0, 3.0), abs=1e-12)
    p = oracle.project_one([0.3, 0.0, 0.0], S, arr)  # camera looks down -z: world +x is image right
    assert p["u"] == pytest.approx(50.0 + cam.fx * 0.3 / 3.0, abs=1e-10)
    p = oracle.project_one([0.0, 0.2, 1.0], S, arr)  # world +y is image up; depth 2
    assert (p["v"], p["depth"]) == pytest.approx((40.0 - cam.fy * 0.2 / 2.0, 2.0), abs=1e-10)


def test_projection_covariance_first_order():
    """EWA: the screen covariance (conic^-1 minus the dilation) is the pinhole map's Jacobian,
    taken numerically here, applied to Sigma; and it matches the covariance of projected samples
    of a small Gaussian."""
    rng = np.random.default_rng(21)
    cam = wl.look_at_camera((1.0, 0.8, 2.5), width=200, height=150)
    arr = cam.as_array()
    R, t = cam.R.astype(float), cam.t.astype(float)

    def pix(x):
        pc = R @ x + t
        return np.array([cam.fx * pc[0] / pc[2] + cam.cx, cam.fy * pc[1] / pc[2] + cam.cy])

    for _ in range(5):
        mu = rng.normal(0, 0.4, 3)
        A = rng.normal(0, 1e-3, (3, 3))
        S = A @ A.T
        p = oracle.project_one(mu, S, arr, dilation=0.3)
        a, b, c = p["conic"]
        Sp = np.linalg.inv(np.array([[a, b], [b, c]])) - 0.3 * np.eye(2)
        h = 1e-6
        Jn = np.stack([(pix(mu + h * e) - pix(mu - h * e)) / (2 * h) for e in np.eye(3)], 1)
        np.testing.assert_allclose(Sp, Jn @ S @ Jn.T, rtol=1e-6, atol=1e-9 * np.abs(Sp).max())
        x = rng.multivariate_normal(mu, S, size=200000)
        pc = x @ R.T + t
        uv = np.stack([cam.fx * pc[:, 0] / pc[:, 2] + cam.cx, cam.fy * pc[:, 1] / pc[:, 2] + cam.cy], 1)
        np.testing.assert_allclose(np.cov(uv.T), Sp, rtol=3e-2, atol=3e-2 * np.abs(Sp).max())
        assert p["rx"] == pytest.approx(3 * math.sqrt(Sp[0, 0] + 0.3), rel=1e-9)


def small_scene(seed=0, n_faces=40, W=64, H=48):
    rng = np.random.default_rng(seed)
    V, Fc = wl.random_mesh(rng, n_faces, spread=0.5, size=0.15)
    C = rng.uniform(size=V.shape)
    cam = wl.look_at_camera((0.3, 0.2, 2.5), width=W, height=H).as_array()
    return V.astype(f32), Fc, C.astype(f32), cam


def test_face_reordering_invariance():
    V, Fc, C, cam = small_scene(1, 80)
    rgb0, Tf0, _, m0 = oracle.render_view(V, Fc, C, cam)
    perm = np.random.default_rng(2).permutation(len(Fc))
    rgb1, Tf1, _, m1 = oracle.render_view(V, Fc[perm], C, cam)
    ok = ~(m0 | m1)
    np.testing.assert_allclose(rgb1[ok], rgb0[ok], atol=1e-13)
    np.testing.assert_allclose(Tf1[ok], Tf0[ok], atol=1e-13)


def test_partition_of_unity_and_transmittance_bounds():
    V, Fc, C, cam = small_scene(3, 120)
    P = oracle.Params(bg=(1.0, 1.0, 1.0))
    rgb, Tf, nc, mask = oracle.render_view(V, Fc, np.ones_like(C), cam, P)
    np.testing.assert_allclose(rgb, 1.0, atol=1e-12)
    assert (Tf <= 1.0).all() and (Tf >= P.t_eps).all()
    assert nc.max() > 3  # composite of several Gaussians happened


def test_linearity_in_colours():
    V, Fc, C, cam = small_scene(4, 60)
    rng = np.random.default_rng(5)
    C1 = rng.uniform(size=C.shape).astype(f32)
    C2 = rng.uniform(size=C.shape).astype(f32)
    r1 = oracle.render_view(V, Fc, C1, cam)[0]
    r2 = oracle.render_view(V, Fc, C2, cam)[0]
    r12 = oracle.render_view(V, Fc, (C1.astype(float) + C2.astype(float)).astype(f32), cam)[0]
    # C1 + C2 is rounded to float32; compare against the sum with that rounding folded back in
    np.testing.assert_allclose(r12, r1 + r2, atol=1e-6)


def test_rigid_motion_of_camera_and_mesh():
    V, Fc, C, cam = small_scene(6, 60)
    q, _ = np.linalg.qr(np.random.default_rng(7).normal(size=(3, 3)))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    t = np.array([0.3, -0.2, 0.5])
    V2 = (V.astype(float) @ q.T + t).astype(f32)
    R = cam[:9].reshape(3, 3)
    cam2 = cam.copy()
    R2 = R @ q.T
    cam2[:9] = R2.reshape(-1)
    cam2[9:12] = cam[9:12] - R2 @ t
    rgb0, _, _, m0 = oracle.render_view(V, Fc, C, cam)
    rgb1, _, _, m1 = oracle.render_view(V2, Fc, C, cam2)
    ok = ~(m0 | m1)
    # float32 rounding of the moved vertices perturbs positions by ~1e-7
    np.testing.assert_allclose(rgb1[ok], rgb0[ok], atol=1e-4)
    assert np.abs(rgb1[ok] - rgb0[ok]).mean() < 1e-6


def test_tile_lists_match_per_pixel_brute_force():
    V, Fc, C, cam = small_scene(8, 50, W=40, H=24)
    G = oracle.gaussians(V, Fc, C, cam)
    W, H, tw, th = 40, 24, 8, 8
    off, ids, amb = oracle.tile_lists_view(V, Fc, C, cam, tw, th)
    ntx = W // tw
    for t in range(len(off) - 1):
        tx, ty = t % ntx, t // ntx
        brute = set()
        for j in range(ty * th, (ty + 1) * th):
            for i in range(tx * tw, (tx + 1) * tw):
                for f in range(len(Fc)):
                    g = G[f]
                    if g[0] and abs(i + 0.5 - g[1]) <= g[6] and abs(j + 0.5 - g[2]) <= g[7]:
                        brute.add(f)
        lst = ids[off[t]:off[t + 1]]
        a = amb[off[t]:off[t + 1]]
        assert set(lst[a != 2].tolist()) == brute
        keys = [(float(f32(G[f][8])), f) for f in lst]
        assert keys == sorted(keys)


# ------------------------------------------------------------------------------------------------
# adjoint
# ------------------------------------------------------------------------------------------------

def _fd_check(V, Fc, C, cam, P, vids, seed=0, rtol=1e-5, linear=True):
    rng = np.random.default_rng(seed)
    H, W = int(cam[17]), int(cam[16])
    g_rgb = rng.normal(size=(H, W, 3))
    g_alpha = rng.normal(size=(H, W))

    def loss(Vx):
        rgb, Tf, _, _ = oracle.render_view(Vx, Fc, C, cam, P)
        return float((g_rgb * rgb).sum() + (g_alpha * (1 - Tf)).sum())

    def decisions(Vx):
        return oracle.render_view(Vx, Fc, C, cam, P, want_hash=True)[4].tobytes()

    dV, dC = oracle.adjoint_view(V, Fc, C, cam, g_rgb, g_alpha, P)
    scale = np.abs(dV).max()
    rgb0, Tf0, nc0, _ = oracle.render_view(V, Fc, C, cam, P)
    assert (nc0 > 0).mean() > 0.05 and scale > 0  # the scene is on screen; the check is not vacuous
    checked = 0
    for vid in vids:
        fd = oracle.fd_vertex_grad(loss, V, vid, h=2e-6, decision_fn=decisions)
        for k in range(3):
            if fd[k] is None:
                continue
            checked += 1 if dV[vid, k] != 0.0 else 0
            assert abs(fd[k] - dV[vid, k]) <= rtol * scale + 1e-4 * abs(dV[vid, k]), (vid, k, fd[k], dV[vid, k])
    assert checked >= 2 * len(vids)
    if not linear:
        return dV, dC
    # colour gradients are exact by linearity: L(C) - L(0) = sum dC . C
    l_c = loss(V)
    rgb0, Tf0, _, _ = oracle.render_view(V, Fc, np.zeros_like(C), cam, P)
    l_0 = float((g_rgb * rgb0).sum() + (g_alpha * (1 - Tf0)).sum())
    assert l_c - l_0 == pytest.approx(float((dC * C.astype(float)).sum()), rel=1e-10, abs=1e-10)
    return dV, dC


@pytest.mark.parametrize("cov_mode", [0, 1, 2])
def test_adjoint_vs_finite_differences(cov_mode):
    V, Fc, C, cam = small_scene(9, 12, W=48, H=40)
    P = oracle.Params(cov_mode=cov_mode, bg=(0.2, 0.3, 0.1))
    _fd_check(V, Fc, C, cam, P, vids=range(0, len(V), 3))


def test_adjoint_vs_fd_icosphere_mesh():
    v0, f = wl.icosphere(1)
    rng = np.random.default_rng(10)
    V = (v0 * 0.8 + rng.normal(0, 0.01, v0.shape)).astype(f32)
    C = rng.uniform(size=v0.shape).astype(f32)
    cam = wl.look_at_camera((0.4, 0.6, 2.6), width=48, height=48).as_array()
    _fd_check(V, f, C, cam, oracle.Params(), vids=range(0, len(V), 4))


def test_adjoint_vs_fd_clamped_kappa_branch():
    """Triangles under the epsilon clamp of Eq. 12 (|A| < 1.04e-6) seen from close by, so their
    covariance dominates the screen footprint."""
    rng = np.random.default_rng(17)
    tris = []
    for k in range(4):
        c = np.array([rng.uniform(-4e-4, 4e-4), rng.uniform(-4e-4, 4e-4), 0.0])
        tris.append(c + rng.normal(0, 5e-4, size=(3, 3)) * [1, 1, 0.2])
    V = np.concatenate(tris).astype(f32)
    Fc = np.arange(len(V), dtype=np.int32).reshape(-1, 3)
    _, _, _, ok = oracle.convert(V, Fc, np.ones_like(V), 0)
    areas = [0.5 * np.linalg.norm(np.cross(t[1] - t[0], t[2] - t[0])) for t in V.astype(float).reshape(-1, 3, 3)]
    assert ok.all() and max(areas) < 1.03e-6
    C = rng.uniform(size=V.shape).astype(f32)
    cam = wl.look_at_camera((0.0, 0.0, 0.05), width=48, height=48).as_array()
    cam[12] = cam[13] = 2500.0
    _fd_check(V, Fc, C, cam, oracle.Params(), vids=range(len(V)))


def test_l2_loss_gradient():
    rng = np.random.default_rng(18)
    a, b = rng.normal(size=(10, 3)), rng.normal(size=(10, 3))
    L, g = oracle.l2_loss(a, b)
    assert L == pytest.approx(((a - b) ** 2).mean())
    h = 1e-6
    a2 = a.copy(); a2[3, 1] += h
    assert (oracle.l2_loss(a2, b)[0] - L) / h == pytest.approx(g[3, 1], rel=1e-4)
