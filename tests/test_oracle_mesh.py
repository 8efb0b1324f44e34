"""Pins of the oracle's triangulation, edges and CSR (brute force, closed
forms, symmetries)."""
import numpy as np
import pytest

import oracle
from oracle.dual import solid_angle
from _oracle_cache import mesh_and_dual


@pytest.mark.parametrize("N", [1, 2, 4, 16, 32])
def test_closed_form_counts(N):
    m, _ = mesh_and_dual(N)
    V = 4 * N * N + 36 * N
    assert m.nnodes == V
    assert m.nedges == 3 * V - 6          # closed triangulated sphere
    assert m.ntris == 2 * V - 4
    assert m.nnodes - m.nedges + m.ntris == 2
    assert int(m.is_pole.sum()) == 34     # 17 ladder chords per cap


@pytest.mark.parametrize("N", [2, 4, 32])
def test_degree_histogram(N):
    m, _ = mesh_and_dual(N)
    deg = np.bincount(m.degree)
    assert deg[5] == 16 and deg[7] == 4 and deg.sum() == m.nnodes
    assert deg[6] == m.nnodes - 20 and m.degree.max() == 7


@pytest.mark.parametrize("N", [1, 4, 24])
def test_topology_brute_force(N):
    m, _ = mesh_and_dual(N)
    T = m.tris
    # every directed edge appears exactly once (consistent orientation)
    directed = {}
    for t in T:
        for s in range(3):
            key = (int(t[s]), int(t[(s + 1) % 3]))
            assert key not in directed
            directed[key] = 1
    for (a, b) in list(directed):
        assert (b, a) in directed
    # every node's triangle fan is one closed cycle
    nxt = {}
    for t in T:
        for s in range(3):
            i, j, k = int(t[s]), int(t[(s + 1) % 3]), int(t[(s + 2) % 3])
            nxt.setdefault(i, {})[j] = k
    for i, ring in nxt.items():
        start = next(iter(ring))
        cur, steps = start, 0
        while True:
            cur = ring[cur]
            steps += 1
            if cur == start:
                break
        assert steps == len(ring) == m.degree[i]
    # canonical storage: smallest index first, list sorted
    assert np.all(T[:, 0] < T[:, 1]) and np.all(T[:, 0] < T[:, 2])
    assert np.all(np.diff(T[:, 0]) >= 0)


@pytest.mark.parametrize("N", [4, 32])
def test_triangles_tile_the_sphere(N):
    m, _ = mesh_and_dual(N)
    X = m.grid.xyz
    T = m.tris
    a, b, c = X[T[:, 0]], X[T[:, 1]], X[T[:, 2]]
    vol = np.einsum("ij,ij->i", a, np.cross(b, c))
    assert np.all(vol > 0)                       # outward counter-clockwise
    area = solid_angle(a, b, c).sum()
    np.testing.assert_allclose(area, 4 * np.pi, rtol=1e-14)


@pytest.mark.parametrize("N", [4, 32])
def test_edges_and_csr(N):
    m, _ = mesh_and_dual(N)
    E = m.edges
    assert np.all(E[:, 0] < E[:, 1])
    keys = E[:, 0] * m.nnodes + E[:, 1]
    assert np.all(np.diff(keys) > 0)             # unique, lexicographic
    for i in [0, 19, 20, m.nnodes // 2, m.nnodes - 1]:
        s0, s1 = m.off[i], m.off[i + 1]
        nb = m.nbr[s0:s1]
        assert np.all(np.diff(nb) > 0)
        for s in range(s0, s1):
            e = m.eid[s]
            assert set(E[e]) == {i, nb[s - s0]}
            assert m.sgn[s] == (1 if E[e, 0] == i else -1)
            n = nb[s - s0]
            back = m.off[n] + m.rev[s]
            assert m.nbr[back] == i and m.eid[back] == e
    # rev is an involution on directed slots
    back = m.off[m.nbr] + m.rev
    assert np.all(m.off[m.nbr[back]] + m.rev[back] == np.arange(m.nbr.size))


def test_band_structure():
    m, _ = mesh_and_dual(8)
    g = m.grid
    rows = g.node_row[m.tris]
    span = rows.max(axis=1) - rows.min(axis=1)
    assert np.all(span <= 1)
    caps = span == 0
    assert caps.sum() == 36
    # band (k, k+1) holds n_k + n_{k+1} triangles
    lo = rows.min(axis=1)
    for k in range(g.nrows - 1):
        assert np.sum((lo == k) & ~caps) == g.row_size[k] + g.row_size[k + 1]


def _rotation_perm(g, quarter=1):
    shift = (g.row_size[g.node_row] // 4) * quarter
    return g.row_off[g.node_row] + (g.node_j + shift) % g.row_size[g.node_row]


def _mirror_perm(g):
    r = g.nrows - 1 - g.node_row
    return g.row_off[r] + g.node_j


def test_band_rotation_symmetry():
    m, _ = mesh_and_dual(16)
    g = m.grid
    P = _rotation_perm(g)
    rows = g.node_row[m.tris]
    band = rows.max(axis=1) > rows.min(axis=1)
    mapped = {tuple(sorted(t)) for t in P[m.tris[band]]}
    orig = {tuple(sorted(t)) for t in m.tris[band]}
    assert mapped == orig


def test_mirror_symmetry_except_equator_band():
    m, _ = mesh_and_dual(16)
    g = m.grid
    P = _mirror_perm(g)
    rows = g.node_row[m.tris]
    lo = rows.min(axis=1)
    eq = (lo == g.N - 1) & (rows.max(axis=1) == g.N)
    mapped = {tuple(sorted(t)) for t in P[m.tris[~eq]]}
    orig = {tuple(sorted(t)) for t in m.tris[~eq]}
    assert mapped == orig
    assert {tuple(sorted(t)) for t in P[m.tris[eq]]} != {tuple(sorted(t)) for t in m.tris[eq]}


def test_pole_edges_are_chords():
    m, _ = mesh_and_dual(8)
    g = m.grid
    pe = m.edges[m.is_pole]
    assert np.all(g.node_row[pe[:, 0]] == g.node_row[pe[:, 1]])
    assert set(g.node_row[pe[:, 0]]) == {0, g.nrows - 1}
    # each cap: ring edges (20) + chords (17) inside row 0
    in_row0 = (g.node_row[m.edges[:, 0]] == 0) & (g.node_row[m.edges[:, 1]] == 0)
    assert in_row0.sum() == 37


def test_build_by_name():
    m = oracle.build_mesh("O2")
    assert m.nnodes == 88
