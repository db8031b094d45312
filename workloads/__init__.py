"""Seeded synthetic inputs for the Gaussian Mesh Renderer hot path.

This module is shared by the FP64 oracle (``oracle/``), the tests and the
bench, and holds none of the renderer's arithmetic: it only builds meshes,
per-vertex colours, pinhole cameras and batch descriptors.  The paper's
datasets (17 objects, 253 hemisphere views each; Sec. 3.1) are not available,
so these synthetic meshes and Fibonacci-sphere views stand in for them.

Everything is generated in float64 with ``numpy.random.default_rng(seed)`` and
cast to float32 at the end.  Draw order inside one workload: geometry noise,
then colours, then batch shape draws.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "icosphere", "uv_sphere", "torus", "fibonacci_dirs", "look_at_camera",
    "Camera", "Workload", "make_workload", "WORKLOAD_NAMES",
]


# ----------------------------------------------------------------------------------------------
# meshes (float64 vertices, int32 faces)
# ----------------------------------------------------------------------------------------------

def icosphere(subdiv: int):
    """Unit icosphere: an icosahedron, then `subdiv` rounds of 4-way midpoint splits with the
    midpoints pushed back onto the unit sphere.  subdiv=2 -> 162 verts / 320 faces,
    subdiv=5 -> 10242 / 20480."""
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0),
         (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    verts = [np.array(p, dtype=np.float64) / math.sqrt(1 + t * t) for p in v]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
             (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
             (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
             (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(subdiv):
        cache: dict[tuple[int, int], int] = {}

        def mid(a: int, b: int) -> int:
            key = (a, b) if a < b else (b, a)
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    return np.stack(verts).astype(np.float64), np.asarray(faces, dtype=np.int32)


def geodesic_sphere(freq: int):
    """Unit geodesic sphere of frequency `freq`: every icosahedron face split into freq^2
    triangles on its barycentric grid, points pushed onto the sphere, shared points merged.
    20 freq^2 faces, 10 freq^2 + 2 vertices (freq = 45: 40,500 faces)."""
    base_v, base_f = icosphere(0)
    index: dict[tuple[int, int, int], int] = {}
    verts: list[np.ndarray] = []

    def vid(p):
        p = p / np.linalg.norm(p)
        key = tuple(int(round(x * 1e9)) for x in p)
        if key not in index:
            index[key] = len(verts)
            verts.append(p)
        return index[key]

    faces = []
    for a, b, c in base_f:
        A, B, C = base_v[a], base_v[b], base_v[c]
        grid = {}
        for i in range(freq + 1):
            for j in range(freq + 1 - i):
                grid[i, j] = vid(A + (B - A) * (i / freq) + (C - A) * (j / freq))
        for i in range(freq):
            for j in range(freq - i):
                faces.append((grid[i, j], grid[i + 1, j], grid[i, j + 1]))
                if i + j < freq - 1:
                    faces.append((grid[i + 1, j], grid[i + 1, j + 1], grid[i, j + 1]))
    return np.stack(verts), np.asarray(faces, dtype=np.int32)


def uv_sphere(n_az: int, n_polar: int, radius_fn=None):
    """UV sphere with `n_az` azimuth segments and `n_polar` polar bands: two pole vertices,
    n_polar-1 rings of n_az vertices, pole fans and quads split into two triangles.
    500 x 400 -> 199,502 verts / 399,000 faces.  `radius_fn(theta, phi)` displaces radially
    (theta = polar angle, phi = azimuth)."""
    rings = n_polar - 1
    theta = np.pi * np.arange(1, n_polar) / n_polar                 # [rings]
    phi = 2.0 * np.pi * np.arange(n_az) / n_az                      # [n_az]
    th, ph = np.meshgrid(theta, phi, indexing="ij")
    r = np.ones_like(th) if radius_fn is None else radius_fn(th, ph)
    ring_pts = np.stack([r * np.sin(th) * np.cos(ph), r * np.cos(th), r * np.sin(th) * np.sin(ph)],
                        axis=-1).reshape(-1, 3)
    r_n = 1.0 if radius_fn is None else float(radius_fn(np.array(0.0), np.array(0.0)))
    r_s = 1.0 if radius_fn is None else float(radius_fn(np.array(np.pi), np.array(0.0)))
    verts = np.concatenate([[[0.0, r_n, 0.0]], ring_pts, [[0.0, -r_s, 0.0]]], axis=0)
    north, south = 0, 1 + rings * n_az

    def ring(i, j):
        return 1 + i * n_az + (j % n_az)

    faces = []
    for j in range(n_az):
        faces.append((north, ring(0, j + 1), ring(0, j)))
    for i in range(rings - 1):
        for j in range(n_az):
            a, b = ring(i, j), ring(i, j + 1)
            c, d = ring(i + 1, j), ring(i + 1, j + 1)
            faces.append((a, b, d))
            faces.append((a, d, c))
    for j in range(n_az):
        faces.append((south, ring(rings - 1, j), ring(rings - 1, j + 1)))
    return verts.astype(np.float64), np.asarray(faces, dtype=np.int32)


def torus(n_u: int, n_v: int, R: float = 1.0, r: float = 0.35):
    """Torus in the xz plane (axis +y), an n_u x n_v grid of quads split into two triangles each.
    1690 x 592 -> 1,000,480 verts / 2,000,960 faces."""
    u = 2.0 * np.pi * np.arange(n_u) / n_u
    v = 2.0 * np.pi * np.arange(n_v) / n_v
    uu, vv = np.meshgrid(u, v, indexing="ij")
    rho = R + r * np.cos(vv)
    verts = np.stack([rho * np.cos(uu), r * np.sin(vv), rho * np.sin(uu)], axis=-1).reshape(-1, 3)
    i = np.arange(n_u)[:, None]
    j = np.arange(n_v)[None, :]
    a = i * n_v + j
    b = ((i + 1) % n_u) * n_v + j
    c = i * n_v + (j + 1) % n_v
    d = ((i + 1) % n_u) * n_v + (j + 1) % n_v
    f1 = np.stack([a, b, d], axis=-1).reshape(-1, 3)
    f2 = np.stack([a, d, c], axis=-1).reshape(-1, 3)
    faces = np.stack([f1, f2], axis=1).reshape(-1, 3)
    return verts.astype(np.float64), faces.astype(np.int32)


def vertex_normals(verts, faces):
    """Area-weighted vertex normals (used only to displace vertices radially/along normals)."""
    v0, v1, v2 = verts[faces[:, 0]], verts[faces[:, 1]], verts[faces[:, 2]]
    fn = np.cross(v1 - v0, v2 - v0)
    n = np.zeros_like(verts)
    for k in range(3):
        np.add.at(n, faces[:, k], fn)
    return n / np.linalg.norm(n, axis=1, keepdims=True)


# ----------------------------------------------------------------------------------------------
# cameras
# ----------------------------------------------------------------------------------------------

@dataclass
class Camera:
    """Pinhole camera, OpenCV axes (+x right, +y down, +z forward), world->camera p = R x + t.
    Pixel (i, j) has its centre at (i + 0.5, j + 0.5)."""
    R: np.ndarray          # [3,3] float32, row-major
    t: np.ndarray          # [3] float32
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    near: float = 0.01
    far: float = 1e10

    def as_array(self) -> np.ndarray:
        """[R(9), t(3), fx, fy, cx, cy, W, H, near, far] as float64 (values are float32-exact)."""
        return np.concatenate([self.R.reshape(-1).astype(np.float64), self.t.astype(np.float64),
                               np.array([self.fx, self.fy, self.cx, self.cy, self.width, self.height,
                                         self.near, self.far], dtype=np.float64)])


def look_at_camera(eye, target=(0.0, 0.0, 0.0), width=128, height=128, fov_deg=60.0,
                   fov_axis="x", near=0.01, far=1e10) -> Camera:
    """Look-at pinhole camera.  World up is +y, falling back to +z when the view direction is
    within ~8 degrees of it.  `fov_axis` 'x' makes fx = (W/2)/tan(fov/2); 'y' makes
    fy = (H/2)/tan(fov/2).  Square pixels: fx = fy.  Principal point at the image centre."""
    eye = np.asarray(eye, dtype=np.float64)
    fwd = np.asarray(target, dtype=np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    up = np.array([0.0, 1.0, 0.0])
    if abs(float(fwd @ up)) > 0.99:
        up = np.array([0.0, 0.0, 1.0])
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd]).astype(np.float32)
    t = (-(R.astype(np.float64) @ eye)).astype(np.float32)
    half = math.tan(math.radians(fov_deg) / 2.0)
    f = (width / 2.0) / half if fov_axis == "x" else (height / 2.0) / half
    f = float(np.float32(f))
    return Camera(R=R, t=t, fx=f, fy=f, cx=float(width) / 2.0, cy=float(height) / 2.0,
                  width=int(width), height=int(height), near=float(np.float32(near)),
                  far=float(np.float32(far)))


def fibonacci_dirs(n: int) -> np.ndarray:
    """n unit vectors on a Fibonacci sphere: y_i = 1 - 2(i + 1/2)/n, golden-angle azimuth."""
    i = np.arange(n, dtype=np.float64)
    y = 1.0 - 2.0 * (i + 0.5) / n
    rad = np.sqrt(np.maximum(0.0, 1.0 - y * y))
    ga = math.pi * (3.0 - math.sqrt(5.0))
    th = ga * i
    return np.stack([rad * np.cos(th), y, rad * np.sin(th)], axis=-1)


def hemisphere_dirs(n: int) -> np.ndarray:
    """n unit vectors spread uniformly over the upper (y >= 0) hemisphere: y_i = 1 - (i + 1/2)/n,
    golden-angle azimuth."""
    i = np.arange(n, dtype=np.float64)
    y = 1.0 - (i + 0.5) / n
    rad = np.sqrt(np.maximum(0.0, 1.0 - y * y))
    th = math.pi * (3.0 - math.sqrt(5.0)) * i
    return np.stack([rad * np.cos(th), y, rad * np.sin(th)], axis=-1)


# ----------------------------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------------------------

@dataclass
class Workload:
    """One batch: M meshes (flat vertex/face arrays with CSR offsets; face indices are GLOBAL
    into the flat vertex array), per-vertex colours, and views (each bound to one mesh)."""
    name: str
    verts: np.ndarray            # [V,3] float32 (optimised / rendered geometry)
    faces: np.ndarray            # [F,3] int32, global vertex indices
    colors: np.ndarray           # [V,3] float32
    vert_offsets: np.ndarray     # [M+1] int64
    face_offsets: np.ndarray     # [M+1] int64
    view_mesh: np.ndarray        # [NV] int32
    cams: list                   # [NV] Camera
    target_verts: np.ndarray | None = None   # [V,3] float32 noise-free geometry for the target
    info: dict = field(default_factory=dict)

    @property
    def num_meshes(self) -> int:
        return len(self.vert_offsets) - 1

    @property
    def num_views(self) -> int:
        return len(self.cams)

    @property
    def num_pixels(self) -> int:
        return int(sum(c.width * c.height for c in self.cams))

    def pixel_offsets(self) -> np.ndarray:
        p = [0]
        for c in self.cams:
            p.append(p[-1] + c.width * c.height)
        return np.asarray(p, dtype=np.int64)

    def cam_array(self) -> np.ndarray:
        return np.stack([c.as_array() for c in self.cams])

    def mesh(self, m: int):
        """(verts, faces-local, colors) of mesh m."""
        v0, v1 = int(self.vert_offsets[m]), int(self.vert_offsets[m + 1])
        f0, f1 = int(self.face_offsets[m]), int(self.face_offsets[m + 1])
        return self.verts[v0:v1], self.faces[f0:f1] - v0, self.colors[v0:v1]


WORKLOAD_NAMES = {
    1: "icosphere_s2_1x128",
    2: "icosphere_s5_8x512",
    3: "uvsphere_500x400_4x1024",
    4: "batch16_mixed",
    5: "torus_2M_32x1920x1080",
}


def _single(name, verts, faces, colors, cams, target_verts=None, info=None) -> Workload:
    nv, nf = len(verts), len(faces)
    return Workload(name=name, verts=verts.astype(np.float32), faces=faces.astype(np.int32),
                    colors=colors.astype(np.float32),
                    vert_offsets=np.array([0, nv], dtype=np.int64),
                    face_offsets=np.array([0, nf], dtype=np.int64),
                    view_mesh=np.zeros(len(cams), dtype=np.int32), cams=cams,
                    target_verts=None if target_verts is None else target_verts.astype(np.float32),
                    info=info or {})


def _fib_cams(n, size_wh, radius=3.0, fov_axis="x"):
    w, h = size_wh
    return [look_at_camera(radius * d, width=w, height=h, fov_axis=fov_axis)
            for d in fibonacci_dirs(n)]


def make_workload(k: int, seed: int | None = None, scale: float = 1.0) -> Workload:
    """The five synthetic workloads.  `scale` < 1 shrinks image sides (and nothing else) for
    quick tests; scale=1 is the full size."""
    seed = k if seed is None else seed
    rng = np.random.default_rng(seed)

    def side(s):
        return max(8, int(round(s * scale)))

    if k == 1:
        v0, f = icosphere(2)
        v = v0 + rng.normal(0.0, 0.01, size=v0.shape)
        col = rng.uniform(0.0, 1.0, size=v0.shape)
        cams = [look_at_camera((0.0, 0.0, 3.0), width=side(128), height=side(128))]
        return _single(WORKLOAD_NAMES[1], v, f, col, cams, target_verts=v0)
    if k == 2:
        v0, f = icosphere(5)
        s = rng.normal(0.0, 0.02, size=len(v0))
        v = v0 + s[:, None] * vertex_normals(v0, f)
        col = rng.uniform(0.0, 1.0, size=v0.shape)
        cams = _fib_cams(8, (side(512), side(512)))
        return _single(WORKLOAD_NAMES[2], v, f, col, cams, target_verts=v0)
    if k == 3:
        def rad(th, ph):
            return 1.0 + 0.05 * np.sin(6.0 * th) * np.cos(8.0 * ph)
        v0, f = uv_sphere(500, 400)
        v, _ = uv_sphere(500, 400, rad)
        col = rng.uniform(0.0, 1.0, size=v0.shape)
        cams = _fib_cams(4, (side(1024), side(1024)))
        return _single(WORKLOAD_NAMES[3], v, f, col, cams, target_verts=v0)
    if k == 4:
        fcount = np.exp(rng.uniform(math.log(5e3), math.log(3e5), size=16))
        meshes = []
        for m in range(16):
            if m % 2 == 0:
                nu = max(3, int(round(math.sqrt(fcount[m] * 1.0 / (2 * 0.35)))))
                nv_ = max(3, int(round(fcount[m] / (2 * nu))))
                meshes.append(torus(nu, nv_))
            else:
                s = 4
                while s < 6 and 20 * 4 ** (s + 1) <= fcount[m]:
                    s += 1
                meshes.append(icosphere(s))
        vs, fs, cs, vo, fo = [], [], [], [0], [0]
        noise_all = [rng.normal(0.0, 0.02, size=mv.shape) for mv, _ in meshes]
        col_all = [rng.uniform(0.0, 1.0, size=mv.shape) for mv, _ in meshes]
        tv = []
        for (mv, mf), nz, cl in zip(meshes, noise_all, col_all):
            fs.append(mf + vo[-1])
            vs.append(mv + nz)
            tv.append(mv)
            cs.append(cl)
            vo.append(vo[-1] + len(mv))
            fo.append(fo[-1] + len(mf))
        n_views = rng.integers(1, 9, size=16)
        cams, vm = [], []
        for m in range(16):
            dirs = fibonacci_dirs(int(n_views[m]))
            sides = rng.choice([256, 512, 800], size=int(n_views[m]))
            for d, sd in zip(dirs, sides):
                cams.append(look_at_camera(3.0 * d, width=side(int(sd)), height=side(int(sd))))
                vm.append(m)
        return Workload(name=WORKLOAD_NAMES[4], verts=np.concatenate(vs).astype(np.float32),
                        faces=np.concatenate(fs).astype(np.int32),
                        colors=np.concatenate(cs).astype(np.float32),
                        vert_offsets=np.asarray(vo, dtype=np.int64),
                        face_offsets=np.asarray(fo, dtype=np.int64),
                        view_mesh=np.asarray(vm, dtype=np.int32), cams=cams,
                        target_verts=np.concatenate(tv).astype(np.float32))
    if k == 5:
        v0, f = torus(1690, 592)
        v = v0 + rng.normal(0.0, 0.01, size=v0.shape)
        col = rng.uniform(0.0, 1.0, size=v0.shape)
        cams = _fib_cams(32, (side(1920), side(1080)), fov_axis="y")
        return _single(WORKLOAD_NAMES[5], v, f, col, cams, target_verts=v0)
    raise ValueError(f"unknown workload {k}")


def random_mesh(rng, n_faces: int, spread: float = 0.6, size: float = 0.25):
    """Small soup of independent random triangles around the origin (tests only)."""
    c = rng.uniform(-spread, spread, size=(n_faces, 1, 3))
    tri = c + rng.normal(0.0, size, size=(n_faces, 3, 3))
    verts = tri.reshape(-1, 3)
    faces = np.arange(3 * n_faces, dtype=np.int32).reshape(-1, 3)
    return verts, faces
