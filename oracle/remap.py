"""Grid-to-grid remapping by linear interpolation over the source mesh's
triangles, in 3-D on the sphere (oracle; test infrastructure only).

The paper remaps a field from a fine "O32" grid to a coarse "F8" grid with a
linear element-based interpolation in 3-D on the sphere (Section 4.3,
Figures 4-6) and defers the algorithm to its reference [10].  Readings used
here:

* Target grids.  ``F<M>`` is the regular (full) Gaussian grid: 2M rows at the
  Gaussian colatitudes (the roots of P_2M), each with 4M points at longitude
  2 pi j / (4M), j = 0..4M-1, numbered row by row from north to south and
  west to east.  ``O<M>`` targets are octahedral grids as in ``grid``.
* Element.  A source triangle (a, b, c) (unit vectors, stored outward
  counter-clockwise) is the flat triangle through its three nodes.  A target
  point p (unit vector) belongs to the triangle that the ray from the centre
  of the sphere through p meets: the triple products
  D_a = det(p, b, c), D_b = det(a, p, c), D_c = det(a, b, p)
  are all >= 0 and their sum D = p . ((b - a) x (c - a)) is > 0 (the front
  side; the cone through the antipodal triangle has all three <= 0).
* Weights.  The ray meets the triangle's plane at q = t p with
  t = (a . n) / (p . n), n = (b - a) x (c - a); the linear interpolant of the
  nodal values at q has the barycentric coordinates of q as weights, which
  are w = (D_a, D_b, D_c) / D (the scale t cancels).  The remapped value is
  w_a f_a + w_b f_b + w_c f_c, level by level.
* Points on an edge or at a node lie in several triangles; each gives the
  same value up to rounding (the weights of the nodes not shared are zero).
  A triangle counts as containing p when D > 0 and its smallest triple
  product is >= -DET_TOL; the oracle takes the containing triangle whose
  smallest weight is largest (ties: the lowest triangle index), so its
  choice is deterministic; tests compare values, not triangle indices.

Point location is brute force: every triangle is tested against every target
point (in blocks of targets), which is slow but obviously complete.
"""

import math
import re

import numpy as np

from .grid import OGrid, _libm, gaussian_colatitudes

# containment tolerance on the triple products (points on an edge or at a
# node): products of unit vectors carry rounding of about 1e-15, while the
# normalised weights D_x / D carry that divided by D ~ h^2, too much for a
# fixed tolerance on fine meshes
DET_TOL = 1e-14


class TargetGrid:
    """Points of a target grid: ``F<M>`` (regular Gaussian) or ``O<M>``."""

    def __init__(self, name):
        m = re.fullmatch(r"([FfOo])(\d+)", name.strip())
        if not m or int(m.group(2)) < 1:
            raise ValueError(f"not a target grid name: {name!r}")
        kind, M = m.group(1).upper(), int(m.group(2))
        self.name = f"{kind}{M}"
        if kind == "O":
            g = OGrid(M)
            self.row_size = g.row_size.copy()
            self.theta = g.theta.copy()
            self.lon = g.lon.copy()
            self.xyz = g.xyz.copy()
            self.npoints = g.nnodes
            return
        nrows = 2 * M
        self.theta = gaussian_colatitudes(nrows)
        self.row_size = np.full(nrows, 4 * M, dtype=np.int64)
        n = 4 * M
        j = np.tile(np.arange(n, dtype=np.float64), nrows)
        row = np.repeat(np.arange(nrows), n)
        self.lon = (2.0 * math.pi * j) / n
        sinlat = _libm(math.cos, self.theta)[row]
        coslat = _libm(math.sin, self.theta)[row]
        xyz = np.empty((nrows * n, 3), dtype=np.float64)
        xyz[:, 0] = coslat * _libm(math.cos, self.lon)
        xyz[:, 1] = coslat * _libm(math.sin, self.lon)
        xyz[:, 2] = sinlat
        self.xyz = xyz
        self.npoints = nrows * n


def _det(a, b, c):
    """det(a, b, c) = a . (b x c), row-wise."""
    return np.einsum("...i,...i->...", a, np.cross(b, c))


def triple_products(a, b, c, p):
    """(D_a, D_b, D_c) of the module docstring, stacked on the last axis.
    Arrays broadcast row-wise (last axis = xyz)."""
    return np.stack([_det(p, b, c), _det(a, p, c), _det(a, b, p)], axis=-1)


def triangle_weights(a, b, c, p):
    """Barycentric weights of the ray through p in the plane of (a, b, c):
    (D_a, D_b, D_c) / D, and D itself."""
    dd = triple_products(a, b, c, p)
    d = dd[..., 0] + dd[..., 1] + dd[..., 2]
    with np.errstate(divide="ignore", invalid="ignore"):   # D = 0: ray in the plane
        return dd / d[..., None], d


def locate(src_xyz, tris, points, block=64):
    """For every point, the containing source triangle and its weights.

    Brute force: each block of points is tested against all triangles; among
    the triangles with D > 0 and every triple product >= -DET_TOL the one
    with the largest smallest weight wins (lowest index on ties).  Raises if
    a point lies in no triangle.
    Returns (tri [P] int64, nodes [P][3] int64, weights [P][3] float64)."""
    a = src_xyz[tris[:, 0]]
    b = src_xyz[tris[:, 1]]
    c = src_xyz[tris[:, 2]]
    P = points.shape[0]
    tri = np.empty(P, dtype=np.int64)
    for s in range(0, P, block):
        p = points[s:s + block][:, None, :]                   # [B,1,3]
        dd = triple_products(a[None], b[None], c[None], p)     # [B,T,3]
        d = dd.sum(axis=-1)
        # D = p . ((b - a) x (c - a)) > 0: the ray meets the front side
        inside = (d > 0) & (dd.min(axis=-1) >= -DET_TOL)
        with np.errstate(divide="ignore", invalid="ignore"):
            score = np.where(inside, dd.min(axis=-1) / d, -np.inf)
        best = np.argmax(score, axis=1)                        # first maximum
        ok = np.isfinite(score[np.arange(best.size), best])
        if not ok.all():
            raise RuntimeError(f"points {np.nonzero(~ok)[0][:5] + s} lie in no triangle")
        tri[s:s + block] = best
    nodes = tris[tri]
    w, _ = triangle_weights(src_xyz[nodes[:, 0]], src_xyz[nodes[:, 1]], src_xyz[nodes[:, 2]], points)
    return tri, nodes, w


def locate_near(src_xyz, tris, points, cos_max):
    """``locate`` restricted to the triangles whose first node is within an
    angle acos(cos_max) of each point (for single points of large meshes);
    complete whenever that angle exceeds the largest triangle's extent."""
    out_t = np.empty(points.shape[0], dtype=np.int64)
    out_n = np.empty((points.shape[0], 3), dtype=np.int64)
    out_w = np.empty((points.shape[0], 3), dtype=np.float64)
    first = src_xyz[tris[:, 0]]
    for i, p in enumerate(points):
        cand = np.nonzero(first @ p >= cos_max)[0]
        t, n, w = locate(src_xyz, tris[cand], p[None, :])
        out_t[i], out_n[i], out_w[i] = cand[t[0]], n[0], w[0]
    return out_t, out_n, out_w


def apply(nodes, weights, f):
    """Remapped field: out[t] = sum_j weights[t, j] * f[nodes[t, j]] for a
    field f of shape [V, ...] (levels and components trailing)."""
    f = np.asarray(f, dtype=np.float64)
    shape = (-1,) + (1,) * (f.ndim - 1)
    out = np.zeros((nodes.shape[0],) + f.shape[1:], dtype=np.float64)
    for j in range(3):
        out += weights[:, j].reshape(shape) * f[nodes[:, j]]
    return out


def apply_adjoint(nodes, weights, y, nnodes):
    """Transpose of ``apply`` for the plain Euclidean inner product: the
    value of target point t, weighted by w[t, j], is added to its node
    nodes[t, j]; shape [nnodes, ...] with y's trailing axes."""
    y = np.asarray(y, dtype=np.float64)
    out = np.zeros((nnodes,) + y.shape[1:], dtype=np.float64)
    shape = (-1,) + (1,) * (y.ndim - 1)
    for j in range(3):
        np.add.at(out, nodes[:, j], weights[:, j].reshape(shape) * y)
    return out

