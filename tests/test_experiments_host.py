"""Host-side pieces of the synthetic-target reconstruction experiments: the geodesic sphere, the
hemisphere views, the diameter normalisation, the surface sampler and the CD / NC metrics.
CPU only."""
import numpy as np
import pytest

import workloads as wl
from oracle import recon


@pytest.mark.parametrize("freq", [1, 3, 8])
def test_geodesic_sphere_is_a_closed_unit_sphere(freq):
    v, f = wl.geodesic_sphere(freq)
    assert len(f) == 20 * freq * freq and len(v) == 10 * freq * freq + 2
    assert len(recon.mesh_edges(f)) == 3 * len(f) // 2                 # closed 2-manifold
    np.testing.assert_allclose(np.linalg.norm(v, axis=1), 1.0, atol=1e-12)
    n = np.cross(v[f[:, 1]] - v[f[:, 0]], v[f[:, 2]] - v[f[:, 0]])
    assert (np.einsum("ij,ij->i", n, v[f].mean(1)) > 0).all()           # outward orientation
    if freq == 1:
        v0, f0 = wl.icosphere(0)
        assert len(v) == len(v0)


def test_hemisphere_dirs():
    d = wl.hemisphere_dirs(253)
    np.testing.assert_allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-12)
    assert (d[:, 1] > 0).all()
    # uniform over the hemisphere: mean height 1/2, mean horizontal direction ~ 0
    assert d[:, 1].mean() == pytest.approx(0.5, abs=1e-3)
    assert np.abs(d[:, [0, 2]].mean(0)).max() < 0.02


def test_normalise_and_metrics():
    pytest.importorskip("torch")
    from paper_2602_14493_amd import experiments as ex
    rng = np.random.default_rng(0)
    v, f = ex.target_mesh("ellipsoid", freq=6)
    assert np.linalg.norm(v, axis=1).max() == pytest.approx(1.0, rel=1e-12)
    p, n = ex.surface_samples(v, f, 4000, rng)
    # samples lie on the faces: inside the unit ball, on the ellipsoid's scale
    assert np.linalg.norm(p, axis=1).max() <= 1.0 + 1e-9 and np.abs(np.linalg.norm(n, axis=1) - 1).max() < 1e-12
    cd, nc = ex.chamfer_nc(p, n, p, n, "cpu")
    assert cd < 1e-12 and nc == pytest.approx(1.0)
    # shifted by |t| = 5 (diameter 2): every nearest neighbour lies between |t| - 2 and |t| away
    cd2, _ = ex.chamfer_nc(p + [5.0, 0, 0], n, p, n, "cpu")
    assert 2 * 3.0 ** 2 < cd2 < 2 * 5.0 ** 2
