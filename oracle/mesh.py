"""Triangulation, edges and node-to-edge CSR of an O-grid (oracle; test
infrastructure only).

The paper describes a mesh as elements that link grid points, with
connectivity lists of elements, edges and nodes (Section 2.3, Figure 1), and
leaves the structured-mesh generator undefined.  Readings used here:

* Band between rows a = k and b = k+1 ("zipper"): walking east from the zero
  meridian, each step advances the row whose next point comes first in
  longitude.  Longitudes are compared exactly as integers,
  (p+1) * n_b  versus  (q+1) * n_a.  On a tie the row with fewer points
  advances first; with equal counts (the equator band) the northern row does.
  Advancing a adds triangle (a_p, a_p+1, b_q); advancing b adds
  (a_p, b_q, b_q+1) (indices modulo the row size).  A band therefore holds
  n_a + n_b triangles.  The walk is a merge of the two rows' sorted event
  lists, which is how it is evaluated here.
* Polar caps: each 20-point polar row is closed by a ladder of 18 triangles
  (j, j+1, 19-j) and (j+1, 18-j, 19-j), j = 0..8, in row-local indices.  No
  node sits at the pole.  The 17 chords of each ladder are the "pole edges".
* Every triangle is stored counter-clockwise as seen from outside the sphere
  (decided here from the sign of a triple product), rotated so its smallest
  node index comes first, and the triangle list is sorted lexicographically.
* Edges are the unique unordered node pairs (a, b), a < b, sorted
  lexicographically; edge e points from a to b, and sign(i, e) is +1 at a,
  -1 at b.
* CSR: node i's slots are its incident edges ordered by neighbour index;
  each slot stores (neighbour, edge id, sign), and rev[s] is the position of
  i in the neighbour's own slot list.
"""

import numpy as np

from .grid import OGrid

CAP_POINTS = 20


def _band(grid, k):
    """Zipper triangles of the band between rows k and k+1 (unoriented)."""
    na = int(grid.row_size[k])
    nb = int(grid.row_size[k + 1])
    keys = np.concatenate([np.arange(1, na + 1, dtype=np.int64) * nb,
                           np.arange(1, nb + 1, dtype=np.int64) * na])
    is_a = np.concatenate([np.ones(na, dtype=bool), np.zeros(nb, dtype=bool)])
    # tie priority: the row with fewer points first, the northern row when equal
    a_first = na <= nb
    prio = np.where(is_a, 0 if a_first else 1, 1 if a_first else 0)
    order = np.lexsort((prio, keys))
    ev_a = is_a[order]
    p = np.cumsum(ev_a) - ev_a            # a-advances before this event
    q = np.cumsum(~ev_a) - (~ev_a)        # b-advances before this event
    A = lambda j: grid.node(k, j)         # noqa: E731
    B = lambda j: grid.node(k + 1, j)     # noqa: E731
    t0 = A(p)
    t1 = np.where(ev_a, A(p + 1), B(q))
    t2 = np.where(ev_a, B(q), B(q + 1))
    return np.stack([t0, t1, t2], axis=1)


def _cap(grid, row):
    """Ladder triangles closing a 20-point polar row (unoriented)."""
    n0 = int(grid.row_size[row])
    assert n0 == CAP_POINTS
    tris = []
    for j in range(n0 // 2 - 1):
        tris.append((j, j + 1, n0 - 1 - j))
        tris.append((j + 1, n0 - 2 - j, n0 - 1 - j))
    loc = np.array(tris, dtype=np.int64)
    return grid.row_off[row] + loc


def _orient_outward_ccw(xyz, tris):
    """Reorder each triangle so that it is counter-clockwise seen from outside."""
    a = xyz[tris[:, 0]]
    b = xyz[tris[:, 1]]
    c = xyz[tris[:, 2]]
    vol = np.einsum("ij,ij->i", a, np.cross(b - a, c - a))
    if np.any(vol == 0.0):
        raise RuntimeError("degenerate triangle")
    out = tris.copy()
    flip = vol < 0
    out[flip, 1], out[flip, 2] = tris[flip, 2], tris[flip, 1]
    return out


def _canonical(tris):
    """Rotate each triangle to start at its smallest index; sort the list."""
    r = np.argmin(tris, axis=1)
    idx = (r[:, None] + np.arange(3)[None, :]) % 3
    rot = np.take_along_axis(tris, idx, axis=1)
    order = np.lexsort((rot[:, 2], rot[:, 1], rot[:, 0]))
    return rot[order]


def band_triangles(grid):
    """Zipper triangles of every band between consecutive rows (unoriented)."""
    return np.concatenate([_band(grid, k) for k in range(grid.nrows - 1)], axis=0).astype(np.int64)


class OMesh:
    """Connectivity of the triangulated O-grid; see the module docstring.

    ``tris`` replaces the ladder-capped triangulation by another closed
    triangulation of ``grid``'s nodes (any orientation; e.g. other polar
    caps); such a mesh flags no pole edges."""

    def __init__(self, grid, tris=None):
        self.grid = grid
        V = grid.nnodes
        self.nnodes = V
        ladder = tris is None
        if ladder:
            parts = [_cap(grid, 0), band_triangles(grid), _cap(grid, grid.nrows - 1)]
            tris = np.concatenate(parts, axis=0).astype(np.int64)
        tris = _orient_outward_ccw(grid.xyz, np.asarray(tris, dtype=np.int64))
        self.tris = _canonical(tris)
        T = self.tris.shape[0]
        self.ntris = T

        # unique undirected edges, lexicographic
        lo = np.minimum(self.tris, np.roll(self.tris, -1, axis=1))
        hi = np.maximum(self.tris, np.roll(self.tris, -1, axis=1))
        keys = (lo * V + hi).ravel()
        ukeys, inv = np.unique(keys, return_inverse=True)
        self.edges = np.stack([ukeys // V, ukeys % V], axis=1)
        E = self.edges.shape[0]
        self.nedges = E
        # tri_edge[t, s] = edge of side (t_s, t_{s+1})
        self.tri_edge = inv.reshape(T, 3)
        side_order = np.argsort(inv, kind="stable")
        counts = np.bincount(inv, minlength=E)
        if not np.all(counts == 2):
            raise RuntimeError("an edge is not shared by exactly two triangles")
        self.edge_tris = (side_order // 3).reshape(E, 2)   # ascending per edge

        # node -> slot CSR, slots ordered by neighbour index
        a, b = self.edges[:, 0], self.edges[:, 1]
        src = np.concatenate([a, b])
        dst = np.concatenate([b, a])
        eid = np.concatenate([np.arange(E), np.arange(E)])
        sgn = np.concatenate([np.ones(E, np.int64), -np.ones(E, np.int64)])
        order = np.lexsort((dst, src))
        self.slot_node = src[order]
        self.nbr = dst[order]
        self.eid = eid[order]
        self.sgn = sgn[order]
        self.off = np.zeros(V + 1, dtype=np.int64)
        np.cumsum(np.bincount(src, minlength=V), out=self.off[1:])
        skeys = self.slot_node * V + self.nbr          # sorted ascending
        back = np.searchsorted(skeys, self.nbr * V + self.slot_node)
        assert np.all(skeys[back] == self.nbr * V + self.slot_node)
        self.rev = back - self.off[self.nbr]
        self.degree = np.diff(self.off)

        # pole edges: chords of the polar ladders
        if not ladder:
            self.is_pole = np.zeros(E, dtype=bool)
            return
        ra = grid.node_row[a]
        rb = grid.node_row[b]
        polar = (ra == rb) & ((ra == 0) | (ra == grid.nrows - 1))
        dj = (grid.node_j[b] - grid.node_j[a]) % CAP_POINTS
        self.is_pole = polar & (dj != 1) & (dj != CAP_POINTS - 1)


def build_mesh(name_or_N):
    """Build the oracle connectivity for an octahedral grid name or N."""
    return OMesh(OGrid(name_or_N))
