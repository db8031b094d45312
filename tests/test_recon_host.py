"""Host side of the reconstruction step: the mesh-graph builder of the C ABI against the oracle's
edge list and neighbour sets, and the argument checks of the regulariser and VectorAdam entry
points (each rejected before any device work).  CPU only."""
import ctypes

import numpy as np
import pytest

import workloads as wl
from oracle import recon


def _graph(f, nv):
    from paper_2602_14493_amd import _lib
    ne = ctypes.c_int64()
    _lib.call("gmr_mesh_graph_size", f.ctypes.data, len(f), nv, ctypes.byref(ne))
    E = ne.value
    edges = np.zeros((E, 2), np.int32)
    off = np.zeros(nv + 1, np.int32)
    ent = np.zeros(2 * E, np.int32)
    _lib.call("gmr_build_mesh_graph", f.ctypes.data, len(f), nv, E, edges.ctypes.data, off.ctypes.data,
              ent.ctypes.data)
    return edges, off, ent


@pytest.mark.parametrize("level", [0, 2])
def test_mesh_graph_matches_oracle(level):
    v, f = wl.icosphere(level)
    edges, off, ent = _graph(f, len(v))
    np.testing.assert_array_equal(edges, recon.mesh_edges(f))
    nb = recon.neighbours(len(v), edges)
    for i in range(len(v)):
        row = ent[off[i]:off[i + 1]]
        assert np.all(np.diff(row >> 1) > 0)                        # ascending edge index
        other = edges[row >> 1, 1 - (row & 1)]
        assert np.all(edges[row >> 1, row & 1] == i)                  # side names this vertex's end
        np.testing.assert_array_equal(np.sort(other), nb[i])


def test_mesh_graph_skips_degenerate_corners_and_isolated_vertices():
    f = np.array([[0, 1, 2], [2, 2, 3], [1, 0, 2]], np.int32)       # one degenerate face, one repeat
    edges, off, ent = _graph(f, 5)                                    # vertex 4 is isolated
    np.testing.assert_array_equal(edges, recon.mesh_edges(f))
    assert edges.tolist() == [[0, 1], [0, 2], [1, 2], [2, 3]]
    assert off[4] == off[5]


def test_mesh_graph_rejects_bad_input():
    from paper_2602_14493_amd import _lib
    L = _lib.load()
    v, f = wl.icosphere(1)
    bad = f.copy()
    bad[5, 2] = -1
    ne = ctypes.c_int64()
    assert L.gmr_mesh_graph_size(bad.ctypes.data, len(f), len(v), ctypes.byref(ne)) == _lib.GMR_ERR_INVALID_ARG
    edges, off, ent = _graph(f, len(v))
    st = L.gmr_build_mesh_graph(f.ctypes.data, len(f), len(v), len(edges) + 1, edges.ctypes.data, off.ctypes.data,
                                ent.ctypes.data)
    assert st == _lib.GMR_ERR_INVALID_ARG


def test_regularizer_and_vector_adam_argument_checks():
    from paper_2602_14493_amd import _lib
    L = _lib.load()
    nb = ctypes.c_size_t()
    assert L.gmr_regularizers_scratch_size(10, 20, ctypes.byref(nb)) == _lib.GMR_OK and nb.value == 30 * 16 + 2 * 8
    dummy = ctypes.c_void_p(256)   # never dereferenced: every call below fails its host-side checks
    st = L.gmr_regularizers(dummy, 10, dummy, 20, dummy, dummy, 0.0, 1.0, 1.0, dummy, 30 * 16 + 15, dummy, dummy,
                            None)
    assert st == _lib.GMR_ERR_WORKSPACE
    st = L.gmr_regularizers(dummy, 10, dummy, 20, dummy, dummy, float("nan"), 1.0, 1.0, dummy, 30 * 16 + 16, dummy,
                            dummy, None)
    assert st == _lib.GMR_ERR_INVALID_ARG
    for b1, b2, eps in [(1.0, 0.999, 1e-8), (0.9, -0.1, 1e-8), (0.9, 0.999, 0.0)]:
        st = L.gmr_vector_adam_step(dummy, dummy, dummy, dummy, 10, 1e-3, b1, b2, eps, dummy, None)
        assert st == _lib.GMR_ERR_INVALID_ARG
    assert L.gmr_vector_adam_step(None, dummy, dummy, dummy, 10, 1e-3, 0.9, 0.999, 1e-8, dummy,
                                  None) == _lib.GMR_ERR_INVALID_ARG
    # the reconstruction backward needs rgb, target and mask, and finite weights
    o = _lib.load().gmr_default_options()
    st = L.gmr_render_bwd_recon(dummy, None, ctypes.byref(o), dummy, dummy, dummy, dummy, dummy, dummy, 1.0, None,
                                1.0, dummy, dummy, dummy, 0, dummy, dummy, None, dummy, 1 << 20, None)
    assert st == _lib.GMR_ERR_INVALID_ARG
    st = L.gmr_render_bwd_recon(dummy, None, ctypes.byref(o), dummy, dummy, dummy, dummy, dummy, dummy, 1.0, dummy,
                                float("inf"), dummy, dummy, dummy, 0, dummy, dummy, None, dummy, 1 << 20, None)
    assert st == _lib.GMR_ERR_INVALID_ARG
