"""Pins of the oracle's view-dependent colour (the extension named with the colour assignment of
Sec. 2.2; real spherical harmonics of degree 1-3 in the 3DGS sign convention, coefficient 0 = the
colour itself).  Independent of the oracle's code: orthonormality under a quadrature exact for
these polynomials, harmonicity and homogeneity of each basis polynomial, the sign convention at
the axes, reduction to Eq. 16 when the higher coefficients vanish, the per-face colour against the
basis at the viewing direction, FD of the vertex gradient through the viewing direction (with and
without active clamps) and exact coefficient gradients by linearity.  CPU only."""
import numpy as np
import pytest

import oracle
import workloads as wl
from test_oracle_pins import _fd_check, small_scene

f32 = np.float32


def _sphere_quadrature(nz=10, nphi=24):
    """Gauss-Legendre in z times the trapezoid rule in phi: exact for polynomials in (x, y, z) of
    degree <= 2 nz - 1 in z and < nphi in phi.  Returns unit directions and weights summing to 4 pi."""
    z, wz = np.polynomial.legendre.leggauss(nz)
    phi = 2 * np.pi * np.arange(nphi) / nphi
    Z, PH = np.meshgrid(z, phi, indexing="ij")
    r = np.sqrt(1 - Z ** 2)
    d = np.stack([r * np.cos(PH), r * np.sin(PH), Z], -1).reshape(-1, 3)
    w = (wz[:, None] * np.full(nphi, 2 * np.pi / nphi)[None, :]).reshape(-1)
    return d, w


def test_basis_orthonormal():
    d, w = _sphere_quadrature()
    Y = oracle.sh_basis(3, d)
    G = (Y * w[:, None]).T @ Y                       # integral of Y_i Y_j over the sphere
    want = np.eye(16)
    want[0, 0] = 4 * np.pi                           # Y_0 = 1: the colour itself, not Y_00
    np.testing.assert_allclose(G, want, atol=1e-12)


def test_basis_polynomials_harmonic_and_homogeneous():
    rng = np.random.default_rng(0)
    p = rng.normal(size=(50, 3))
    h = 1e-3
    lap = -6 * oracle.sh_basis(3, p)
    for a in range(3):
        e = np.zeros(3); e[a] = h
        lap += oracle.sh_basis(3, p + e) + oracle.sh_basis(3, p - e)
    lap /= h * h
    np.testing.assert_allclose(lap[:, 1:], 0.0, atol=1e-6)      # each band-l polynomial is harmonic
    band = np.array([0, 1, 1, 1, 2, 2, 2, 2, 2, 3, 3, 3, 3, 3, 3, 3])
    s = 1.7
    np.testing.assert_allclose(oracle.sh_basis(3, s * p), oracle.sh_basis(3, p) * s ** band, rtol=1e-12)


def test_basis_sign_convention():
    def Y(v):
        v = np.asarray(v, float)
        return oracle.sh_basis(3, v / np.linalg.norm(v))[0]
    c1 = np.sqrt(3 / (4 * np.pi))
    assert Y([0, 1, 0])[1] == pytest.approx(-c1) and Y([0, 0, 1])[2] == pytest.approx(c1)
    assert Y([1, 0, 0])[3] == pytest.approx(-c1)
    assert Y([1, 1, 0])[4] > 0 and Y([0, 1, 1])[5] < 0 and Y([0, 0, 1])[6] > 0 and Y([1, 0, 1])[7] < 0
    assert Y([1, 0, 0])[8] > 0
    assert Y([0, 1, 0])[9] > 0 and Y([1, 1, 1])[10] > 0 and Y([0, 1, 0])[11] > 0 and Y([0, 0, 1])[12] > 0
    assert Y([1, 0, 0])[13] > 0 and Y([1, 0, 1])[14] > 0 and Y([1, 0, 0])[15] < 0


def _coefs(rng, nv, degree, dc=(0.4, 1.0), hi=0.02):
    K = (degree + 1) ** 2
    C = np.empty((nv, K, 3))
    C[:, 0] = rng.uniform(*dc, size=(nv, 3))
    C[:, 1:] = rng.normal(0, hi, size=(nv, K - 1, 3))
    return C.astype(f32)


def test_zero_higher_coefficients_is_eq16():
    V, Fc, C, cam = small_scene(21, 60)
    for deg in (1, 2, 3):
        K = (deg + 1) ** 2
        Csh = np.zeros((len(V), K, 3), f32)
        Csh[:, 0] = C
        a = oracle.render_view(V, Fc, C, cam)
        b = oracle.render_view(V, Fc, Csh, cam, oracle.Params(sh_degree=deg))
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y)


def test_face_colour_is_basis_at_viewing_direction():
    rng = np.random.default_rng(22)
    V, Fc, _, _ = small_scene(22, 40)
    eye = np.array([0.7, -0.4, 2.2])
    cam = wl.look_at_camera(eye, width=64, height=48).as_array()
    for deg in (1, 3):
        C = _coefs(rng, len(V), deg, dc=(0.0, 0.4), hi=0.4)
        P = oracle.Params(sh_degree=deg)
        G = oracle.gaussians(V, Fc, C, cam, P)
        ok = G[:, 0] > 0
        assert ok.sum() > 10
        mu = V.astype(float)[Fc].mean(1)
        d = (mu - eye) / np.linalg.norm(mu - eye, axis=1, keepdims=True)
        Y = oracle.sh_basis(deg, d)
        coef = C.astype(float)[Fc].mean(1)                       # [F, K, 3]
        want = np.maximum(0.0, np.einsum("fk,fkc->fc", Y, coef))
        np.testing.assert_allclose(G[ok, 9:12], want[ok], atol=1e-6)   # eye is float32-rounded in R, t
        assert (want[ok] == 0).any() and (want[ok] > 0).any()           # some channels clamp at 0


@pytest.mark.parametrize("deg", [1, 3])
def test_adjoint_vs_fd_view_dependent_colour(deg):
    V, Fc, _, cam = small_scene(9, 12, W=48, H=40)
    C = _coefs(np.random.default_rng(23), len(V), deg, hi=0.05)
    P = oracle.Params(sh_degree=deg, bg=(0.2, 0.3, 0.1))
    dV, dC = _fd_check(V, Fc, C, cam, P, vids=range(0, len(V), 3))
    assert dC.shape == C.shape and np.abs(dC[:, 1:]).max() > 0


def test_adjoint_vs_fd_with_active_clamps():
    V, Fc, _, cam = small_scene(9, 12, W=48, H=40)
    C = _coefs(np.random.default_rng(24), len(V), 2, dc=(0.0, 0.4), hi=0.4)
    P = oracle.Params(sh_degree=2)
    G = oracle.gaussians(V, Fc, C, cam, P)
    assert (G[G[:, 0] > 0, 9:12] == 0).any()                             # the clamp is active somewhere
    _fd_check(V, Fc, C, cam, P, vids=range(0, len(V), 3), linear=False)
