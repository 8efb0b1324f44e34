"""Median dual of the triangulated sphere (oracle; test infrastructure only).

The paper does not define the dual; this is the reading used throughout:

* Points: the edge midpoint m_e = normalize(X_a + X_b) and the triangle
  centre c_T = normalize(X_i + X_j + X_k) (vertex indices i < j < k), both
  projected radially onto the unit sphere.
* The dual face of edge e is the geodesic polyline c_T1 -> m_e -> c_T2 over
  the two triangles sharing e.  Along a great-circle arc from p to q the
  conormal is the constant unit vector along p x q, so the arc's integrated
  conormal is R * angle(p, q) * unit(p x q).
* S_e (metres) is the sum of the two arc terms, each oriented so that its dot
  product with X_b - X_a is positive: S_e points from a to b.
* V_i (square metres) is the area of node i's median cell, the sum over its
  triangles T = (i, j, k) of the spherical triangles (X_i, m_ij, c_T) and
  (X_i, c_T, m_ik), each from the Van Oosterom-Strackee formula
  tan(Omega/2) = |a.(b x c)| / (1 + a.b + b.c + c.a).
  The cells tile the sphere, so sum V_i = 4 pi R^2.
* Local basis at node i: east (-sin lon, cos lon, 0) and
  north (-sin lat cos lon, -sin lat sin lon, cos lat).
* Closure C_i = sum over node i's edges of sign(i, e) S_e.  On a sphere it is
  not zero (it carries the curvature term of the surface divergence theorem)
  and is nearly radial.

The positions m_e and c_T are evaluated in a fixed order (sum, then
sqrt((s0*s0 + s1*s1) + s2*s2), then division), because position errors are
amplified by 1/h in every difference of nearby points.  Differences are taken
before cross products (m x c is evaluated as m x (c - m)), which keeps the
relative rounding of S_e and of the sub-triangle areas at the eps level.
"""

import numpy as np


def _normalize_rows(s):
    nrm = np.sqrt((s[:, 0] * s[:, 0] + s[:, 1] * s[:, 1]) + s[:, 2] * s[:, 2])
    return s / nrm[:, None]


def _dot(a, b):
    return (a[..., 0] * b[..., 0] + a[..., 1] * b[..., 1]) + a[..., 2] * b[..., 2]


def edge_midpoints(xyz, edges):
    return _normalize_rows(xyz[edges[:, 0]] + xyz[edges[:, 1]])


def tri_centres(xyz, tris):
    srt = np.sort(tris, axis=1)
    return _normalize_rows((xyz[srt[:, 0]] + xyz[srt[:, 1]]) + xyz[srt[:, 2]])


def arc_conormal(p, q, radius):
    """R * angle(p, q) * unit(p x q) for unit vectors p, q (rows)."""
    w = np.cross(p, q - p)
    wn = np.sqrt(_dot(w, w))
    ang = np.arctan2(wn, _dot(p, q))
    return (radius * ang / wn)[:, None] * w


def solid_angle(a, b, c):
    """Area of the spherical triangle (a, b, c) on the unit sphere."""
    num = np.abs(_dot(a, np.cross(b - a, c - a)))
    den = 1.0 + _dot(a, b) + _dot(b, c) + _dot(c, a)
    return 2.0 * np.arctan2(num, den)


class DualGeometry:
    """S_e, V_i, local basis and closure of the median dual; see module doc."""

    def __init__(self, mesh, radius):
        grid = mesh.grid
        R = float(radius)
        self.radius = R
        X = grid.xyz
        E = mesh.edges
        a, b = E[:, 0], E[:, 1]
        self.m = edge_midpoints(X, E)
        self.c = tri_centres(X, mesh.tris)

        d = X[b] - X[a]
        S = np.zeros((mesh.nedges, 3))
        for side in range(2):
            t = arc_conormal(self.m, self.c[mesh.edge_tris[:, side]], R)
            flip = _dot(t, d) < 0
            t[flip] *= -1.0
            S += t
        self.S = S

        vol = np.zeros(mesh.nnodes)
        T = mesh.tris
        for r in range(3):
            i = T[:, r]
            m_ij = self.m[mesh.tri_edge[:, r]]
            m_ik = self.m[mesh.tri_edge[:, (r + 2) % 3]]
            om = solid_angle(X[i], m_ij, self.c) + solid_angle(X[i], self.c, m_ik)
            vol += np.bincount(i, weights=om, minlength=mesh.nnodes)
        self.V = R * R * vol

        self.east = np.stack([-grid.sinlon, grid.coslon, np.zeros(grid.nnodes)], axis=1)
        self.north = np.stack([-grid.sinlat * grid.coslon,
                               -grid.sinlat * grid.sinlon,
                               grid.coslat], axis=1)

        C = np.zeros((mesh.nnodes, 3))
        contrib = mesh.sgn[:, None] * self.S[mesh.eid]
        for comp in range(3):
            C[:, comp] = np.bincount(mesh.slot_node, weights=contrib[:, comp],
                                     minlength=mesh.nnodes)
        self.C = C


def build_dual(mesh, radius=6371220.0):
    return DualGeometry(mesh, radius)
