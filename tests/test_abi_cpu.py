"""CPU-only checks of the C-ABI library: it loads, exports every symbol include/gmr.h declares,
and its pure-host entry points (defaults, view table, workspace sizing, adjacency, argument
validation) behave as documented.  No kernel is launched."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "gmr.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gmr_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    from paper_2602_14493_amd import _lib
    L = _lib.load()
    syms = header_symbols()
    assert len(syms) >= 15
    for s in syms:
        assert hasattr(L, s), s
    assert set(syms) == set(_lib.EXPORTED)


def test_missing_library_fails_loudly(monkeypatch):
    from paper_2602_14493_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", "/nonexistent/libgmr.so")
    with pytest.raises(RuntimeError, match="not built"):
        _lib.load()


def test_default_options():
    import paper_2602_14493_amd as gmr
    o = gmr.default_options()
    assert o.cov_mode == 0 and o.tile_w == 16 and o.tile_h == 16 and o.raster_mode == 0 and o.px_per_lane == 1
    assert o.lane_lists == 1 and o.sh_degree == 0 and o.composited_lists == 2046
    assert ctypes.sizeof(o) == 72 and type(o).instance_capacity.offset == 64
    assert o.alpha_min == np.float32(1 / 255) and o.alpha_max == np.float32(0.99) and o.t_eps == np.float32(1e-4)
    assert o.dilation == np.float32(0.3) and tuple(o.bg) == (0.0, 0.0, 0.0)


def test_view_table_and_workspace_sizes():
    import paper_2602_14493_amd as gmr
    from paper_2602_14493_amd import _lib
    W = wl.make_workload(4, scale=0.25)
    b = gmr.Batch.from_workload(W)
    o = gmr.default_options(instance_capacity=1 << 20)
    n = ctypes.c_size_t()
    _lib.call("gmr_view_table_size", ctypes.byref(b.c), ctypes.byref(o), ctypes.byref(n))
    assert n.value == 80 + 128 * W.num_views + 4 * (2 * (W.num_meshes + 1) + W.num_views)
    buf = np.zeros(n.value, np.uint8)
    _lib.call("gmr_view_table_fill", ctypes.byref(b.c), ctypes.byref(o), buf.ctypes.data, n.value)
    hdr = buf[:80].view(np.int32)
    assert hdr[0] == W.num_views and hdr[1] == W.num_meshes and hdr[2] == 16 and hdr[3] == 16
    tiles = sum(((c.width + 15) // 16) * ((c.height + 15) // 16) for c in W.cams)
    assert hdr[4] == tiles and hdr[7] == 4 * tiles
    fv_total = sum(int(W.face_offsets[m + 1] - W.face_offsets[m]) for m in W.view_mesh)
    assert buf[32:40].view(np.int64)[0] == fv_total
    ws, saved = ctypes.c_size_t(), ctypes.c_size_t()
    _lib.call("gmr_workspace_size", ctypes.byref(b.c), ctypes.byref(o), ctypes.byref(ws), ctypes.byref(saved))
    # per pixel T_final + list position; per raster item its composited list (a count word, then
    # 2046 16-bit positions: 1024 words)
    assert saved.value == 8 * W.num_pixels + 1024 * 4 * hdr[7]
    for cap, words in ((0, 0), (1, 2), (7, 5), (8, 5), (8190, 4096)):
        o.composited_lists = cap
        _lib.call("gmr_workspace_size", ctypes.byref(b.c), ctypes.byref(o), ctypes.byref(ws), ctypes.byref(saved))
        assert saved.value == 8 * W.num_pixels + words * 4 * hdr[7]
    assert ws.value >= (1 << 20) * 24 + fv_total * (48 + 16 + 4 + 32)


@pytest.mark.parametrize("field,value", [("cov_mode", 3), ("tile_w", 12), ("tile_h", 72), ("alpha_min", 0.0),
                                         ("t_eps", 1.5), ("raster_mode", 3), ("px_per_lane", 3),
                                         ("lane_lists", 2), ("lane_lists", -1), ("sh_degree", 4), ("sh_degree", -1),
                                         ("composited_lists", -1), ("composited_lists", 8191),
                                         ("instance_capacity", 0), ("instance_capacity", 1 << 30)])
def test_invalid_options_rejected(field, value):
    import paper_2602_14493_amd as gmr
    from paper_2602_14493_amd import _lib
    W = wl.make_workload(1)
    b = gmr.Batch.from_workload(W)
    o = gmr.default_options(instance_capacity=1 << 16)
    setattr(o, field, value)
    ws, saved = ctypes.c_size_t(), ctypes.c_size_t()
    st = _lib.load().gmr_workspace_size(ctypes.byref(b.c), ctypes.byref(o), ctypes.byref(ws), ctypes.byref(saved))
    assert st == _lib.GMR_ERR_INVALID_ARG
    assert len(_lib.load().gmr_last_error()) > 0


def test_invalid_batch_rejected():
    import paper_2602_14493_amd as gmr
    from paper_2602_14493_amd import _lib
    W = wl.make_workload(1)
    o = gmr.default_options(instance_capacity=1 << 16)
    for bad in ("view_mesh", "size", "near"):
        cams = W.cam_array().copy()
        vm = W.view_mesh.copy()
        if bad == "view_mesh":
            vm[0] = 5
        elif bad == "size":
            cams[0, 16] = 0
        else:
            cams[0, 18] = -1.0
        b = gmr.Batch(W.vert_offsets, W.face_offsets, vm, cams)
        ws, saved = ctypes.c_size_t(), ctypes.c_size_t()
        st = _lib.load().gmr_workspace_size(ctypes.byref(b.c), ctypes.byref(o), ctypes.byref(ws), ctypes.byref(saved))
        assert st == _lib.GMR_ERR_INVALID_ARG, bad


def test_build_adjacency_matches_numpy():
    from paper_2602_14493_amd import _lib
    v, f = wl.icosphere(2)
    off = np.zeros(len(v) + 1, np.int32)
    ent = np.zeros(3 * len(f), np.int32)
    _lib.call("gmr_build_adjacency", f.ctypes.data, len(f), len(v), off.ctypes.data, ent.ctypes.data)
    flat = f.reshape(-1)
    for vid in range(len(v)):
        want = np.nonzero(flat == vid)[0]
        np.testing.assert_array_equal(ent[off[vid]:off[vid + 1]], want)
    bad = f.copy()
    bad[3, 1] = len(v)
    st = _lib.load().gmr_build_adjacency(bad.ctypes.data, len(f), len(v), off.ctypes.data, ent.ctypes.data)
    assert st == _lib.GMR_ERR_INVALID_ARG


def test_product_path_never_touches_the_oracle():
    """Nothing in the package (Python or HIP/C++ sources) imports, links or loads the oracle."""
    pkg = os.path.join(ROOT, "paper_2602_14493_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".cpp", ".h")):
                txt = open(os.path.join(dirpath, fn)).read()
                assert not re.search(r"\boracle\b|gmr_oracle|gmro_", txt), os.path.join(dirpath, fn)


def test_bench_refuses_several_gpus():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True)
    assert r.returncode != 0 and "one GPU" in r.stderr


def test_bench_traffic_hash_tracks_code_not_comments(tmp_path, monkeypatch):
    """The stored HBM-byte counters stay valid across a reworded comment and go stale (null) when
    the kernel's code changes."""
    import shutil
    import bench
    src = os.path.join(ROOT, "paper_2602_14493_amd", "csrc")
    fake = tmp_path / "paper_2602_14493_amd" / "csrc"
    fake.mkdir(parents=True)
    for f in ("k_raster.hip", "gmr_common.h"):
        shutil.copy(os.path.join(src, f), fake / f)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.source_hash("raster_bwd")
    key = ("icosphere_s5_8x512", "raster_bwd", "16x16", 1, 0, 1)
    monkeypatch.setitem(bench.TRAFFIC, key, {"fetch": 3, "write": 4, "src": h0})  # counters of this code
    with open(fake / "k_raster.hip", "a") as f:
        f.write("\n// a reworded note\n/* and a block\n   comment */\n")
    assert bench.source_hash("raster_bwd") == h0
    assert bench.measured_traffic("icosphere_s5_8x512", "raster_bwd", "16x16", 1, 0, 1) == 7
    with open(fake / "k_raster.hip", "a") as f:
        f.write("static int added_code = 1;\n")
    assert bench.source_hash("raster_bwd") != h0
    assert bench.measured_traffic("icosphere_s5_8x512", "raster_bwd", "16x16", 1, 0, 1) is None


def test_status_strings():
    from paper_2602_14493_amd import _lib
    L = _lib.load()
    assert L.gmr_status_string(0) == b"ok"
    assert b"workspace" in L.gmr_status_string(2)


def test_noalloc_workspace_limit_matches_header():
    from paper_2602_14493_amd import _lib
    txt = open(os.path.join(ROOT, "include", "gmr.h")).read()
    m = re.search(r"#define GMR_NOALLOC_WORKSPACE_BYTES \(\(size_t\)(\d+) << (\d+)\)", txt)
    assert m and int(m.group(1)) << int(m.group(2)) == _lib.NOALLOC_WORKSPACE_BYTES
