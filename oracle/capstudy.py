"""Alternative treatments of the polar caps, for the accuracy study only
(oracle; test infrastructure only; no GPU kernel computes these).

The report's Nabla operators (Section 2.3) come with no definition of how
the mesh is closed at the poles; the main oracle reads it as a ladder of 18
triangles over each 20-point polar row, with the spherical median dual (the
"S" reading).  Two alternatives are built here so that the cap error of the
ladder can be compared with them:

* Fan caps.  A node at each pole and a fan of 20 triangles from it to the
  polar row.  Everything else (zipper bands, spherical median dual, the
  operators of ``oracle.nabla``) is unchanged, so the operators of
  ``oracle.nabla`` run on it as they stand.  Pole nodes are appended after
  the grid's nodes (north pole, then south pole) with longitude 0, so their
  local basis is east = (0, 1, 0) and north = (-1, 0, 0) at the north pole,
  (1, 0, 0) at the south pole.  The pole nodes have 20 neighbours, beyond the
  library's 7-slot node tables, which is why no GPU kernel is built for it.

* Variant L: the median dual taken in the (longitude, latitude) plane.  The
  same zipper bands, drawn as plane triangles (longitudes unwrapped within
  each triangle across the zero meridian).  Dual points: plane edge
  midpoints and triangle centroids.  There are no caps: each polar-row node's
  cell runs from its band cell up to the pole line (latitude +-pi/2) between
  the longitudes of its row edges' midpoints, so the cells tile the plane
  rectangle [0, 2 pi) x [-pi/2, pi/2].  A row edge of a polar row has one
  triangle; its dual face continues from the edge midpoint straight to the
  pole line.  The stretch of pole line that closes node j's cell is the dual
  face of a "pole edge" from j to the antipodal node j + n0/2 of the same
  row; its plane normal points to the pole at both ends (+lat in the north,
  -lat in the south), not opposite ways as for other edges.  Plane normals
  S_e = (S_lon, S_lat) (radians) are the face segments turned by a quarter
  turn, oriented from a to b; A_i is the plane area of node i's cell.
  Operators with the sphere's metric (R the radius, phi the latitude):

    gradient    G_i = (1/A_i) [sum_e sign(i,e) 0.5 (f_a + f_b) S_e
                               + sum_pole 0.5 (f_i + f_i') S_pole],
                east = G_lon / (R cos phi_i),  north = G_lat / R;
    divergence  div_i = 1/(R cos phi_i A_i) [sum_e sign(i,e) (0.5 (u_a + u_b) S_lon
                               + 0.5 (v_a cos phi_a + v_b cos phi_b) S_lat)
                               + sum_pole S_lat 0.5 cos phi_0 (v_i - v_i')],
    Laplacian   div(grad f),

  where across a pole edge the antipodal node's (east, north) frame is
  turned by half a turn relative to node i's, so its vector components
  change sign (u_i' -> -u_i', v_i' -> -v_i').  The cell's physical area is
  taken as R^2 cos phi_i A_i (the volume weight of the conservation sum).
  Plane cells close, so the gradient of a constant is zero with no closure
  term; the divergence's fluxes cancel in pairs (pole edges included), so
  sum_i R^2 cos phi_i A_i div_i = 0.
"""

import math

import numpy as np

from .dual import DualGeometry
from .grid import OGrid
from .mesh import CAP_POINTS, OMesh, band_triangles


# ------------------------------------------------------------------ fan caps

class FanGrid:
    """The nodes of an O-grid followed by the north and the south pole."""

    def __init__(self, N):
        g = OGrid(N)
        self.base = g
        self.N, self.nrows, self.row_size, self.row_off = g.N, g.nrows, g.row_size, g.row_off
        V = g.nnodes
        self.nnodes = V + 2
        self.north, self.south = V, V + 1
        self.lon = np.concatenate([g.lon, [0.0, 0.0]])
        self.coslon = np.concatenate([g.coslon, [1.0, 1.0]])
        self.sinlon = np.concatenate([g.sinlon, [0.0, 0.0]])
        self.sinlat = np.concatenate([g.sinlat, [1.0, -1.0]])
        self.coslat = np.concatenate([g.coslat, [0.0, 0.0]])
        self.xyz = np.concatenate([g.xyz, [[0.0, 0.0, 1.0], [0.0, 0.0, -1.0]]])
        # row of each node: -1 for the poles
        self.node_row = np.concatenate([g.node_row, [-1, -1]])
        self.node_j = np.concatenate([g.node_j, [0, 0]])
        self.colat = np.concatenate([g.theta[g.node_row], [0.0, math.pi]])


def fan_triangles(grid):
    """Zipper bands plus a 20-triangle fan from each pole node to its polar row."""
    g = grid.base
    tris = [band_triangles(g)]
    for row, pole in ((0, grid.north), (g.nrows - 1, grid.south)):
        n0 = int(g.row_size[row])
        j = np.arange(n0)
        tris.append(np.stack([np.full(n0, pole), g.node(row, j), g.node(row, j + 1)], axis=1))
    return np.concatenate(tris, axis=0).astype(np.int64)


def build_fan_mesh(N, radius=6371220.0):
    """(mesh, dual geometry) of the O-grid closed by pole-node fans."""
    grid = FanGrid(N)
    mesh = OMesh(grid, fan_triangles(grid))
    return mesh, DualGeometry(mesh, radius)


# --------------------------------------------------------------- variant L

class LonLatMesh:
    """Variant L (see the module docstring): plane median dual of the zipper
    bands with pole strips and antipodal pole edges."""

    def __init__(self, N, radius=6371220.0):
        g = OGrid(N)
        self.grid = g
        self.radius = float(radius)
        V = g.nnodes
        self.nnodes = V
        tris = band_triangles(g)
        # unwrap longitudes within each triangle next to its first vertex
        lon = g.lon[tris]
        lon = lon - 2.0 * math.pi * np.round((lon - lon[:, :1]) / (2.0 * math.pi))
        lat = g.lat[tris]
        # unique edges of the band triangles, a < b
        sides = [(0, 1), (1, 2), (2, 0)]
        pa_ = np.concatenate([tris[:, p] for p, _ in sides])
        pb_ = np.concatenate([tris[:, q] for _, q in sides])
        lo, hi = np.minimum(pa_, pb_), np.maximum(pa_, pb_)
        keys, inv = np.unique(lo * V + hi, return_inverse=True)
        self.edges = np.stack([keys // V, keys % V], axis=1)
        E = self.edges.shape[0]
        T = tris.shape[0]
        # per (triangle, side): the face segment from the edge midpoint to
        # the centroid, turned a quarter turn and oriented from a to b
        clon, clat = lon.mean(axis=1), lat.mean(axis=1)
        S = np.zeros((E, 2))
        ntri = np.zeros(E, dtype=np.int64)
        area = np.zeros(V)
        for s, (p, q) in enumerate(sides):
            e = inv[s * T:(s + 1) * T]
            mlon = 0.5 * (lon[:, p] + lon[:, q])
            mlat = 0.5 * (lat[:, p] + lat[:, q])
            dlon, dlat = clon - mlon, clat - mlat
            nrm = np.stack([dlat, -dlon], axis=1)
            a_is_p = tris[:, p] < tris[:, q]
            ablon = np.where(a_is_p, lon[:, q] - lon[:, p], lon[:, p] - lon[:, q])
            ablat = np.where(a_is_p, lat[:, q] - lat[:, p], lat[:, p] - lat[:, q])
            flip = nrm[:, 0] * ablon + nrm[:, 1] * ablat < 0
            nrm[flip] *= -1.0
            np.add.at(S, e, nrm)
            np.add.at(ntri, e, 1)
        # plane cell areas: the quadrilateral (X_i, m_ij, c_T, m_ik) of each
        # triangle corner, by the shoelace formula
        for r in range(3):
            i, j, k = r, (r + 1) % 3, (r + 2) % 3
            px = np.stack([lon[:, i], 0.5 * (lon[:, i] + lon[:, j]), clon, 0.5 * (lon[:, i] + lon[:, k])], axis=1)
            py = np.stack([lat[:, i], 0.5 * (lat[:, i] + lat[:, j]), clat, 0.5 * (lat[:, i] + lat[:, k])], axis=1)
            a = 0.5 * np.abs(np.sum(px * np.roll(py, -1, axis=1) - np.roll(px, -1, axis=1) * py, axis=1))
            np.add.at(area, tris[:, i], a)
        # polar rows: row edges with one triangle get the strip face up to
        # the pole line; each node gets its strip rectangle and a pole edge
        n0 = CAP_POINTS
        dl = 2.0 * math.pi / n0
        pole_a, pole_b, pole_sgn = [], [], []
        for row, sgn in ((0, 1.0), (g.nrows - 1, -1.0)):
            lat0 = float(g.lat[g.row_off[row]])
            h = 0.5 * math.pi - abs(lat0)
            nodes = g.row_off[row] + np.arange(n0)
            area[nodes] += dl * h
            for j in range(n0):
                a, b = nodes[j], nodes[(j + 1) % n0]
                e = int(np.searchsorted(keys, min(a, b) * V + max(a, b)))
                assert keys[e] == min(a, b) * V + max(a, b) and ntri[e] == 1
                # vertical face of length h between node j and its eastern
                # neighbour: the normal from the edge's a = min to b = max
                # points east unless the edge wraps past the zero meridian
                S[e, 0] += h if a < b else -h
            for j in range(n0 // 2):
                pole_a.append(nodes[j])
                pole_b.append(nodes[j + n0 // 2])
                pole_sgn.append(sgn)
        if np.any((ntri == 0) | (ntri > 2)):
            raise RuntimeError("inconsistent band edges")
        self.S = S
        self.area = area
        self.pole = np.stack([pole_a, pole_b], axis=1)
        self.pole_S = np.array(pole_sgn) * dl          # the lat component at both ends
        self.lat = g.lat
        self.coslat = g.coslat

    # node-wise scatter of edge terms: +t at a, -t at b
    def _edge_scatter(self, t):
        a, b = self.edges[:, 0], self.edges[:, 1]
        out = np.zeros((self.nnodes,) + t.shape[1:])
        np.add.at(out, a, t)
        np.subtract.at(out, b, t)
        return out

    def gradient(self, f):
        """f [V][L] -> (east, north) [V][L][2]."""
        a, b = self.edges[:, 0], self.edges[:, 1]
        fe = 0.5 * (f[a] + f[b])
        G = np.stack([self._edge_scatter(fe * self.S[:, c][:, None]) for c in range(2)], axis=2)
        pa_, pb_ = self.pole[:, 0], self.pole[:, 1]
        fp = 0.5 * (f[pa_] + f[pb_])
        for end in (pa_, pb_):
            np.add.at(G[:, :, 1], end, fp * self.pole_S[:, None])
        G /= self.area[:, None, None]
        R = self.radius
        return np.stack([G[:, :, 0] / (R * self.coslat[:, None]), G[:, :, 1] / R], axis=2)

    def divergence(self, uv):
        """(east, north) [V][L][2] -> [V][L]."""
        a, b = self.edges[:, 0], self.edges[:, 1]
        u, v = uv[:, :, 0], uv[:, :, 1]
        vc = v * self.coslat[:, None]
        flux = 0.5 * (u[a] + u[b]) * self.S[:, 0][:, None] + 0.5 * (vc[a] + vc[b]) * self.S[:, 1][:, None]
        out = self._edge_scatter(flux)
        pa_, pb_ = self.pole[:, 0], self.pole[:, 1]
        c0 = self.coslat[pa_][:, None]
        # across the pole the neighbour's frame is turned by half a turn
        np.add.at(out, pa_, self.pole_S[:, None] * 0.5 * c0 * (v[pa_] - v[pb_]))
        np.add.at(out, pb_, self.pole_S[:, None] * 0.5 * c0 * (v[pb_] - v[pa_]))
        return out / (self.radius * self.coslat[:, None] * self.area[:, None])

    def laplacian(self, f):
        return self.divergence(self.gradient(f))

    def cell_area(self):
        """Physical area taken for each cell: R^2 cos(lat) A_i."""
        return self.radius ** 2 * self.coslat * self.area


def build_lonlat_mesh(N, radius=6371220.0):
    return LonLatMesh(N, radius)
