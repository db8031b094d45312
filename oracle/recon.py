"""FP64 oracle of the reconstruction step around the renderer (Sec. 3.1, Implementation Details
and Loss Functions): silhouette binary cross-entropy on the rendered alpha, edge-length and
Laplacian-smoothing regularisers on the mesh, the VectorAdam update of the vertices, and the plain
Adam step of the torus optimisation workload.

TEST INFRASTRUCTURE ONLY (see the package docstring).  The paper names these terms without
formulas or weights; the readings taken here are:

* silhouette: mean over every pixel of every view of -(s log a + (1 - s) log(1 - a)), with the
  rendered alpha a = 1 - T_final clamped to [eps, 1 - eps] (eps = 1e-6) and a binary target mask s.
  The clamp is part of the definition, so the derivative is (a - s) / (a (1 - a)) inside it and 0
  where it is active.
* edge length: mean over the mesh's unique edges of (|v_i - v_j| - l0)^2, target length l0
  (default 0: the common form, which with the other terms keeps edges short and even).
* Laplacian smoothing: mean over vertices of |(1/deg i) sum over neighbours j of v_j - v_i|, the
  uniform-weight Laplacian (neighbours = vertices sharing an edge).
* VectorAdam: Adam whose second moment is kept per vertex on the squared norm of the 3-vector
  gradient (so the update of a vertex is equivariant under rotations of the gradients):
  m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) |g|^2,
  p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
* Adam (the optimiser of the 2M-face torus workload: vertices only, lr 1e-3, betas (0.9, 0.999),
  eps 1e-8): the same update with the second moment kept per coordinate, v = b2 v + (1 - b2) g^2,
  in the bias-corrected form of Kingma & Ba's Adam (ICLR 2015, Algorithm 1).
Each function returns the loss and its gradient in float64.
"""
from __future__ import annotations

import numpy as np

BCE_EPS = 1e-6


def mesh_edges(faces) -> np.ndarray:
    """Unique undirected edges [E, 2] (i < j) of a triangle list, sorted lexicographically.  An
    edge joins two distinct vertices: the corner pair of a degenerate face with a repeated index
    is not an edge."""
    f = np.asarray(faces, np.int64)
    e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]])
    e = np.sort(e, axis=1)
    e = e[e[:, 0] != e[:, 1]]
    return np.unique(e, axis=0).reshape(-1, 2)


def neighbours(num_verts: int, edges) -> list[np.ndarray]:
    """Per vertex, the ascending array of vertices it shares an edge with."""
    nb = [[] for _ in range(num_verts)]
    for i, j in np.asarray(edges, np.int64):
        nb[i].append(j)
        nb[j].append(i)
    return [np.array(sorted(x), np.int64) for x in nb]


def silhouette_bce(alpha, mask, weight: float = 1.0):
    """weight * mean BCE of the clamped alpha against the mask; returns (loss, dL/dalpha)."""
    a = np.asarray(alpha, np.float64).reshape(-1)
    s = np.asarray(mask, np.float64).reshape(-1)
    ac = np.clip(a, BCE_EPS, 1.0 - BCE_EPS)
    n = a.size
    loss = -(s * np.log(ac) + (1.0 - s) * np.log(1.0 - ac)).sum() * weight / n
    inside = (a > BCE_EPS) & (a < 1.0 - BCE_EPS)
    grad = np.where(inside, (ac - s) / (ac * (1.0 - ac)), 0.0) * weight / n
    return float(loss), grad


def edge_length(verts, edges, l0: float = 0.0, weight: float = 1.0):
    """weight * mean over edges of (|v_i - v_j| - l0)^2; returns (loss, dL/dverts [V,3])."""
    v = np.asarray(verts, np.float64)
    e = np.asarray(edges, np.int64)
    d = v[e[:, 0]] - v[e[:, 1]]
    ln = np.linalg.norm(d, axis=1)
    r = ln - l0
    E = len(e)
    loss = float((r * r).sum() * weight / E)
    # d/dv_i (|d| - l0)^2 = 2 (|d| - l0) d / |d|, and the opposite for v_j
    coef = np.where(ln > 0.0, 2.0 * r / np.where(ln > 0.0, ln, 1.0), 0.0) * weight / E
    ge = coef[:, None] * d
    g = np.zeros_like(v)
    np.add.at(g, e[:, 0], ge)
    np.add.at(g, e[:, 1], -ge)
    return loss, g


def laplacian_smoothing(verts, nbrs, weight: float = 1.0):
    """weight * mean over vertices of the norm of the uniform Laplacian; returns (loss, grad)."""
    v = np.asarray(verts, np.float64)
    V = len(v)
    lap = np.zeros_like(v)
    for i in range(V):
        if len(nbrs[i]):
            lap[i] = v[nbrs[i]].mean(axis=0) - v[i]
    nrm = np.linalg.norm(lap, axis=1)
    loss = float(nrm.sum() * weight / V)
    # u_i = d|lap_i| / d lap_i; lap_i depends on v_i with coefficient -1 and on each neighbour j
    # with coefficient 1/deg i
    u = np.where(nrm[:, None] > 0.0, lap / np.where(nrm > 0.0, nrm, 1.0)[:, None], 0.0) * weight / V
    g = -u.copy()
    for i in range(V):
        if len(nbrs[i]):
            g[nbrs[i]] += u[i] / len(nbrs[i])
    return loss, g


def vector_adam_step(p, g, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One VectorAdam step at step number t >= 1 (the first step has t = 1).  p, g, m: [V,3];
    v: [V].  Returns the new (p, m, v)."""
    p = np.asarray(p, np.float64)
    g = np.asarray(g, np.float64)
    m = b1 * np.asarray(m, np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1.0 - b2) * (g * g).sum(axis=1)
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh)[:, None] + eps), m, v


def adam_step(p, g, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam step at step number t >= 1 (the first step has t = 1), elementwise over arrays of
    any shape: m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2, then the bias-corrected moments
    m / (1 - b1^t) and v / (1 - b2^t) give p - lr m_hat / (sqrt(v_hat) + eps).  Returns the new
    (p, m, v)."""
    if t < 1:
        raise ValueError("Adam's step number starts at 1")
    p = np.asarray(p, np.float64)
    g = np.asarray(g, np.float64)
    m = b1 * np.asarray(m, np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
